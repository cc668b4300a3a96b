"""Python binding of libmpt (ctypes).  Argument marshalling only: every step of
the hot path runs in the HIP kernels of libmpt.so; torch provides device
memory and the stream.  Names follow the C ABI in include/mpt.h."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpt.so")

MPT_OK, MPT_E_ARG, MPT_E_HIP, MPT_E_NOMEM, MPT_E_SINGULAR, MPT_E_NOTPD, MPT_E_UNSUPPORTED = range(7)


class MptError(RuntimeError):
    pass


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p), ("row_blocks", C.c_int32),
                ("pad_", C.c_int32)]


class _Rom(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_ref", C.c_int32), ("KM", C.c_void_p), ("A0", C.c_void_p),
                ("CM", C.c_void_p), ("g", C.c_void_p), ("G", C.c_void_p), ("Dp", C.c_void_p),
                ("s_ref", C.c_void_p), ("E", C.c_void_p), ("N0", C.c_void_p),
                ("alpha", C.c_double), ("alpha_lb", C.c_double), ("dirs", C.c_int32 * 3),
                ("pad_", C.c_int32)]


class _Pencil(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_ref", C.c_int32), ("H", C.c_void_p), ("T", C.c_void_p),
                ("f", C.c_void_p), ("Z", C.c_void_p), ("W", C.c_void_p), ("S", C.c_void_p),
                ("alpha", C.c_double), ("alpha_lb", C.c_double)]


class _Tuning(C.Structure):
    _fields_ = [("omegas_per_item", C.c_int32), ("waves_per_group", C.c_int32),
                ("groups_per_cu", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    """Load libmpt.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MptError(f"{LIB_PATH} is missing: build it with paper_2307_05590_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, D, S = C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_size_t
        sig = {
            "mpt_create": ([I32, P, P], I32),
            "mpt_destroy": ([P], I32),
            "mpt_set_stream": ([P, P], I32),
            "mpt_last_error": ([P], C.c_char_p),
            "mpt_max_reduced_dim": ([], I32),
            "mpt_pod_basis_ws_size": ([I64, I32], S),
            "mpt_pod_basis": ([P, P, I64, I64, I32, D, I32, P, I64, P, P, P, S], I32),
            "mpt_project_ws_size": ([I64, I32, I64, I32], S),
            "mpt_project": ([P, P, P, D, P, P, P, D, P, I64, I32, P, I64, P, P, I32, P,
                             P, P, P, P, P, P, P, P, P, P, S], I32),
            "mpt_project_dirs": ([P, P, P, D, P, P, P, D, P, I64, I32, P, P, I64, P, P, I32, P,
                                  P, P, P, P, P, P, P, P, P, P, S], I32),
            "mpt_residual_gram_ws_size": ([I64, I32], S),
            "mpt_residual_gram": ([P, P, I64, P, I64, I64, I32, P, P, S], I32),
            "mpt_sweep_adjoint_materials_ws_size": ([I64], S),
            "mpt_sweep_adjoint_materials": ([P, P, P, P, P, P, I64, P, P, P, P, P, S], I32),
            "mpt_signature": ([P, P, P, I64, P, D, P, P], I32),
            "mpt_signature_adjoint": ([P, P, P, I64, P, D, P, P, P, P], I32),
            "mpt_select_snapshots_ws_size": ([I32], S),
            "mpt_select_snapshots_static": ([P, P, I64, P, P, I32, I32, P, P, P], I32),
            "mpt_sweep_batched_ws_size": ([P, I32, P, P], S),
            "mpt_spmm": ([P, P, P, I64, I32, P, I64], I32),
            "mpt_sweep": ([P, P, P, I64, P, P, P], I32),
            "mpt_select_snapshots": ([P, P, I64, P, P, I32, I32, P, P, P, P, S], I32),
            "mpt_sweep_batched": ([P, P, P, I32, P, P, P, P, P, I32, P, S], I32),
            "mpt_sweep_adjoint": ([P, P, P, I64, P, P, P, P], I32),
            "mpt_sweep_adjoint_batched": ([P, P, P, I32, P, P, P, P, P, P, P, S], I32),
            "mpt_pencil_bytes": ([I32, I32], S),
            "mpt_pencil_reduce": ([P, P, P, S, P], I32),
            "mpt_project_pencil": ([P, P, P, D, P, P, P, D, P, I64, I32, P, I64, P, P, I32, P,
                                    P, P, P, P, P, P, P, P, P, P, S, P, S, D, P], I32),
            "mpt_sweep_pencil": ([P, P, P, I64, P, P, P], I32),
            "mpt_pencil_batched_bytes": ([P, I32, P], S),
            "mpt_tensors_fmm_ws_size": ([I64, I32], S),
            "mpt_tensors_fmm": ([P, P, P, P, P, I64, I32, P, I64, P, P, I64, P, D, P, P, S], I32),
            "mpt_select_snapshots_threshold": ([P, P, I64, P, P, I32, D, P, P, P, P, P, S], I32),
            "mpt_tensors_im_ws_size": ([I64, I64, I32], S),
            "mpt_tensors_im": ([P, P, P, P, P, P, I64, I64, I32, P, I64, P, P, I64, P, D, P, P, S],
                               I32),
            "mpt_sweep_pencil_batched": ([P, P, I32, P, P, P, S, P, P], I32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _ld(t):
    """Leading dimension of a row-major matrix view (unit column stride)."""
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise MptError("expected a row-major matrix with unit column stride")
    return max(int(t.stride(0)), int(t.shape[1]))


class Handle:
    """One libmpt handle bound to a device and (by default) torch's current stream."""

    def __init__(self, device=None, stream=None):
        dev = torch.device(device or "cuda")
        self.index = dev.index if dev.index is not None else torch.cuda.current_device()
        self.h = C.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream(self.index)
        self._check(lib().mpt_create(self.index, C.c_void_p(st.cuda_stream), C.byref(self.h)))
        self.stream = st

    def _check(self, status):
        if status != MPT_OK:
            msg = lib().mpt_last_error(self.h).decode() if self.h else ""
            raise MptError(f"libmpt status {status}: {msg}")

    def use_current_stream(self):
        st = torch.cuda.current_stream(self.index)
        if st != self.stream:
            self._check(lib().mpt_set_stream(self.h, C.c_void_p(st.cuda_stream)))
            self.stream = st

    def close(self):
        if self.h:
            lib().mpt_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles = {}


def handle(device=None) -> Handle:
    dev = torch.device(device or "cuda")
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _handles:
        _handles[idx] = Handle(torch.device("cuda", idx))
    h = _handles[idx]
    h.use_current_stream()
    return h


def _dev_check(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise MptError("libmpt expects contiguous CUDA tensors")


def _dev_check_rows(t):
    """A CUDA row-major matrix whose rows may be longer than its columns
    (passed with its leading dimension)."""
    if not t.is_cuda:
        raise MptError("libmpt expects CUDA tensors")
    _ld(t)


@dataclass
class Csr:
    """CSR matrix on the device (int32 indices, float64 values)."""

    n: int
    rowptr: torch.Tensor
    colind: torch.Tensor
    val: torch.Tensor
    row_blocks: int = 1  # layout hint: equal row blocks sharing one spatial order

    @classmethod
    def from_scipy(cls, K, device="cuda", row_blocks=1):
        K = K.tocsr()
        K.sort_indices()
        return cls(K.shape[0], torch.as_tensor(K.indptr.astype("int32"), device=device),
                   torch.as_tensor(K.indices.astype("int32"), device=device),
                   torch.as_tensor(K.data.astype("float64"), device=device), int(row_blocks))

    def struct(self):
        return _Csr(self.n, self.val.numel(), _ptr(self.rowptr), _ptr(self.colind), _ptr(self.val),
                    self.row_blocks, 0)


# Stability constant of Lemma 4.1 for the reference norms X + s C_sigma
ALPHA_LB = 2.0 / (3.0 + 10.0 ** 0.5)


@dataclass
class Rom:
    """Reduced model of one object (device tensors, complex128 / float64)."""

    M: int
    KM: torch.Tensor
    A0: torch.Tensor
    CM: torch.Tensor
    g: torch.Tensor  # (3, M)
    G: torch.Tensor  # (n_ref, 2M+3, 2M+3): residual Gram per reference shift
    Dp: torch.Tensor  # (n_ref, M, M): conjugation-defect form per shift
    s_ref: torch.Tensor  # (n_ref,) ascending, s_ref[0] = 0
    E: torch.Tensor  # (3, 3)
    N0: torch.Tensor  # (3, 3)
    alpha: float
    alpha_lb: float = ALPHA_LB
    dirs: tuple = (0, 0, 0)  # per-direction block widths, or zeros (joint basis)

    @property
    def n_ref(self):
        return int(self.s_ref.numel())

    def struct(self):
        _dev_check(self.KM, self.A0, self.CM, self.g, self.G, self.Dp, self.s_ref, self.E, self.N0)
        return _Rom(self.M, self.n_ref, _ptr(self.KM), _ptr(self.A0), _ptr(self.CM), _ptr(self.g),
                    _ptr(self.G), _ptr(self.Dp), _ptr(self.s_ref), _ptr(self.E), _ptr(self.N0),
                    float(self.alpha), float(self.alpha_lb), (C.c_int32 * 3)(*self.dirs), 0)

    @classmethod
    def from_host(cls, d, alpha, alpha_lb=ALPHA_LB, device="cuda"):
        """From host arrays: KM, A0, CM (M x M), g (3 x M), G (n_ref x L x L),
        Dp (n_ref x M x M), s_ref (n_ref), E, N0."""
        t = lambda a, dt: torch.as_tensor(a, dtype=dt, device=device).contiguous()
        cd, rd = torch.complex128, torch.float64
        M = d["KM"].shape[0]
        return cls(M, t(d["KM"], cd), t(d["A0"], cd), t(d["CM"], cd), t(d["g"], cd),
                   t(d["G"], cd), t(d["Dp"], cd), t(d["s_ref"], rd), t(d["E"], rd), t(d["N0"], rd),
                   alpha, alpha_lb)


def mpt_spmm(K: Csr, U: torch.Tensor) -> torch.Tensor:
    h = handle(U.device)
    _dev_check_rows(U)
    N, M = U.shape
    Y = torch.empty((N, M), dtype=U.dtype, device=U.device)
    k = K.struct()
    h._check(lib().mpt_spmm(h.h, C.byref(k), _ptr(U), _ld(U), M, _ptr(Y), M))
    return Y


def mpt_residual_gram(Z: torch.Tensor, XinvZ: torch.Tensor) -> torch.Tensor:
    """Residual Gram G_s = (Z^H Y + Y^H Z) / 2 with Y = (X + s C)^{-1} Z (Lemma 4.1):
    Z and Y are N x (2M+3) complex128 on the device; returns G (2M+3)^2."""
    h = handle(Z.device)
    _dev_check(Z)
    _dev_check(XinvZ)
    N, L = Z.shape
    if XinvZ.shape != Z.shape or (L - 3) % 2:
        raise MptError("Z and X^-1 Z must both be N x (2M+3)")
    M = (L - 3) // 2
    G = torch.empty((L, L), dtype=torch.complex128, device=Z.device)
    n = lib().mpt_residual_gram_ws_size(N, M)
    if n == 0:
        raise MptError(f"unsupported sizes N={N} M={M}")
    ws = torch.empty(n, dtype=torch.uint8, device=Z.device)
    h._check(lib().mpt_residual_gram(h.h, _ptr(Z), L, _ptr(XinvZ), L, N, M, _ptr(G), _ptr(ws), n))
    return G


def mpt_pod_basis(D: torch.Tensor, tol_sigma: float, M_cap: int):
    """a1: returns (U (N x M, a view of rows of length M_cap), sigma (ncol), M).
    Synchronises to read M."""
    h = handle(D.device)
    _dev_check(D)
    N, ncol = D.shape
    ws = torch.empty(lib().mpt_pod_basis_ws_size(N, ncol), dtype=torch.uint8, device=D.device)
    U = torch.empty((N, M_cap), dtype=torch.complex128, device=D.device)
    sigma = torch.empty(ncol, dtype=torch.float64, device=D.device)
    M = C.c_int(0)
    h._check(lib().mpt_pod_basis(h.h, _ptr(D), ncol, N, ncol, float(tol_sigma), int(M_cap), _ptr(U),
                                 M_cap, _ptr(sigma), C.byref(M), _ptr(ws), ws.numel()))
    return U[:, :M.value], sigma, M.value


def mpt_project(K: Csr, c, eps_h, w, o, vol, alpha, U, cond, Vt, lam, s_ref, alpha_lb=ALPHA_LB,
                keep_Y=False):
    """a2: Galerkin projection and the certificate data (one residual Gram and
    defect form per reference shift in s_ref) -> Rom (and optionally Y = K U).
    Vt, lam: eigenvectors (rows) and eigenvalues of the conductor block of
    X^{-1} scaled by sqrt(c) on both sides."""
    h = handle(U.device)
    _dev_check(c, w, o, vol, cond, Vt, lam, s_ref)
    _dev_check_rows(U)
    N, M = U.shape
    nc = cond.numel()
    nr = s_ref.numel()
    dev = U.device
    cd, rd = torch.complex128, torch.float64
    KM = torch.empty((M, M), dtype=cd, device=dev)
    A0 = torch.empty_like(KM)
    CM = torch.empty_like(KM)
    g = torch.empty((3, M), dtype=cd, device=dev)
    G = torch.empty((nr, 2 * M + 3, 2 * M + 3), dtype=cd, device=dev)
    Dp = torch.empty((nr, M, M), dtype=cd, device=dev)
    E = torch.empty((3, 3), dtype=rd, device=dev)
    N0 = torch.empty((3, 3), dtype=rd, device=dev)
    Y = torch.empty((N, M), dtype=cd, device=dev) if keep_Y else None
    ws = torch.empty(lib().mpt_project_ws_size(N, M, nc, nr), dtype=torch.uint8, device=dev)
    k = K.struct()
    h._check(lib().mpt_project(h.h, C.byref(k), _ptr(c), float(eps_h), _ptr(w), _ptr(o), _ptr(vol),
                               float(alpha), _ptr(U), _ld(U), M, _ptr(cond), nc, _ptr(Vt), _ptr(lam),
                               nr, _ptr(s_ref), _ptr(KM), _ptr(A0), _ptr(CM), _ptr(g), _ptr(G),
                               _ptr(Dp), _ptr(E), _ptr(N0), _ptr(Y), _ptr(ws), ws.numel()))
    rom = Rom(M, KM, A0, CM, g, G, Dp, s_ref, E, N0, float(alpha), float(alpha_lb))
    return (rom, Y) if keep_Y else rom


def mpt_project_dirs(K: Csr, c, eps_h, w, o, vol, alpha, Us, cond, Vt, lam, s_ref,
                     alpha_lb=ALPHA_LB):
    """a2 for one basis per direction: Us = (U_1, U_2, U_3) -> Rom of the
    concatenated basis with dirs = their widths (Dp: n_ref x 3 x M x M)."""
    U = torch.cat(list(Us), 1).contiguous()
    h = handle(U.device)
    _dev_check(c, w, o, vol, U, cond, Vt, lam, s_ref)
    N, M = U.shape
    dirs = tuple(int(u.shape[1]) for u in Us)
    nc = cond.numel()
    nr = s_ref.numel()
    dev = U.device
    cd, rd = torch.complex128, torch.float64
    KM = torch.empty((M, M), dtype=cd, device=dev)
    A0 = torch.empty_like(KM)
    CM = torch.empty_like(KM)
    g = torch.empty((3, M), dtype=cd, device=dev)
    G = torch.empty((nr, 2 * M + 3, 2 * M + 3), dtype=cd, device=dev)
    Dp = torch.empty((nr, 3, M, M), dtype=cd, device=dev)
    E = torch.empty((3, 3), dtype=rd, device=dev)
    N0 = torch.empty((3, 3), dtype=rd, device=dev)
    ws = torch.empty(lib().mpt_project_ws_size(N, M, nc, nr), dtype=torch.uint8, device=dev)
    k = K.struct()
    dv = (C.c_int32 * 3)(*dirs)
    h._check(lib().mpt_project_dirs(h.h, C.byref(k), _ptr(c), float(eps_h), _ptr(w), _ptr(o),
                                    _ptr(vol), float(alpha), _ptr(U), M, M, dv, _ptr(cond), nc,
                                    _ptr(Vt), _ptr(lam), nr, _ptr(s_ref), _ptr(KM), _ptr(A0),
                                    _ptr(CM), _ptr(g), _ptr(G), _ptr(Dp), _ptr(E), _ptr(N0),
                                    None, _ptr(ws), ws.numel()))
    return Rom(M, KM, A0, CM, g, G, Dp, s_ref, E, N0, float(alpha), float(alpha_lb), dirs), U


def mpt_sweep(rom: Rom, omega: torch.Tensor, want_a: bool = False):
    """a3+a4: (n x 18 outputs [R~ | I | Delta], status[, a (n x 3 x M)])."""
    h = handle(omega.device)
    _dev_check(omega)
    n = omega.numel()
    out = torch.empty((n, 18), dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    a = torch.empty((n, 3, rom.M), dtype=torch.complex128, device=omega.device) if want_a else None
    r = rom.struct()
    h._check(lib().mpt_sweep(h.h, C.byref(r), _ptr(omega), n, _ptr(out), _ptr(a), _ptr(st)))
    return (out, st, a) if want_a else (out, st)


class Pencil:
    """Hessenberg-triangular form of one object's reduced pencil (device buffer)."""

    def __init__(self, buf, st: _Pencil, rom: Rom):
        self.buf = buf  # keeps the device buffer alive
        self.st = st
        self.M = st.M
        self.rom = rom

    def parts(self):
        """Views (H, T column-major as stored; f; Z) as complex tensors."""
        M = self.M
        base = self.buf.data_ptr()

        def view(ptr, shape):
            off = ptr - base
            n = shape[0] * shape[1] * 16
            return self.buf[off:off + n].view(torch.complex128).view(*shape)
        return (view(self.st.H, (M, M)), view(self.st.T, (M, M)), view(self.st.f, (3, M)),
                view(self.st.Z, (M, M)))


def mpt_pencil_reduce(rom: Rom) -> Pencil:
    """Reduce (A0, C_M) to Hessenberg-triangular form (asynchronous)."""
    h = handle(rom.A0.device)
    nb = lib().mpt_pencil_bytes(rom.M, rom.n_ref)
    if nb == 0:
        raise MptError(f"the pencil form takes 1 <= M <= 96 (M = {rom.M})")
    buf = torch.empty(nb, dtype=torch.uint8, device=rom.A0.device)
    r = rom.struct()
    st = _Pencil()
    h._check(lib().mpt_pencil_reduce(h.h, C.byref(r), _ptr(buf), nb, C.byref(st)))
    return Pencil(buf, st, rom)


def mpt_project_pencil(K: Csr, c, eps_h, w, o, vol, alpha, U, cond, Vt, lam, s_ref,
                       alpha_lb=ALPHA_LB):
    """a2 and the pencil reduction in one call (the reduction runs beside the
    certificate data on a private stream) -> (Rom, Pencil), equal to
    mpt_project followed by mpt_pencil_reduce."""
    h = handle(U.device)
    _dev_check(c, w, o, vol, cond, Vt, lam, s_ref)
    _dev_check_rows(U)
    N, M = U.shape
    nc = cond.numel()
    nr = s_ref.numel()
    dev = U.device
    cd, rd = torch.complex128, torch.float64
    KM = torch.empty((M, M), dtype=cd, device=dev)
    A0 = torch.empty_like(KM)
    CM = torch.empty_like(KM)
    g = torch.empty((3, M), dtype=cd, device=dev)
    G = torch.empty((nr, 2 * M + 3, 2 * M + 3), dtype=cd, device=dev)
    Dp = torch.empty((nr, M, M), dtype=cd, device=dev)
    E = torch.empty((3, 3), dtype=rd, device=dev)
    N0 = torch.empty((3, 3), dtype=rd, device=dev)
    ws = torch.empty(lib().mpt_project_ws_size(N, M, nc, nr), dtype=torch.uint8, device=dev)
    nb = lib().mpt_pencil_bytes(M, nr)
    if nb == 0:
        raise MptError(f"the pencil form takes 1 <= M <= 96 and n_ref <= 64 (M = {M}, n_ref = {nr})")
    buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    st = _Pencil()
    k = K.struct()
    h._check(lib().mpt_project_pencil(
        h.h, C.byref(k), _ptr(c), float(eps_h), _ptr(w), _ptr(o), _ptr(vol), float(alpha), _ptr(U),
        _ld(U), M, _ptr(cond), nc, _ptr(Vt), _ptr(lam), nr, _ptr(s_ref), _ptr(KM), _ptr(A0),
        _ptr(CM), _ptr(g), _ptr(G), _ptr(Dp), _ptr(E), _ptr(N0), None, _ptr(ws), ws.numel(),
        _ptr(buf), nb, float(alpha_lb), C.byref(st)))
    rom = Rom(M, KM, A0, CM, g, G, Dp, s_ref, E, N0, float(alpha), float(alpha_lb))
    return rom, Pencil(buf, st, rom)


def mpt_sweep_pencil(pen: Pencil, omega: torch.Tensor, want_a: bool = False):
    """Sweep on the pencil form: same outputs as mpt_sweep."""
    h = handle(omega.device)
    _dev_check(omega)
    n = omega.numel()
    out = torch.empty((n, 18), dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    a = torch.empty((n, 3, pen.M), dtype=torch.complex128, device=omega.device) if want_a else None
    h._check(lib().mpt_sweep_pencil(h.h, C.byref(pen.st), _ptr(omega), n, _ptr(out), _ptr(a),
                                    _ptr(st)))
    return (out, st, a) if want_a else (out, st)


def mpt_tensors_fmm(K: Csr, c, w, U, cond, a, omega, N0, alpha, ws=None):
    """Full matrix method on q = U a: (n x 12 [R~ | I], ws)."""
    h = handle(U.device)
    _dev_check(c, w, cond, a, omega, N0)
    _dev_check_rows(U)
    N, M = U.shape
    n = omega.numel()
    out = torch.empty((n, 12), dtype=torch.float64, device=U.device)
    nb = lib().mpt_tensors_fmm_ws_size(N, M)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=U.device)
    k = K.struct()
    h._check(lib().mpt_tensors_fmm(h.h, C.byref(k), _ptr(c), _ptr(w), _ptr(U), _ld(U), M, _ptr(cond),
                                   cond.numel(), _ptr(a), _ptr(omega), n, _ptr(N0), float(alpha),
                                   _ptr(out), _ptr(ws), ws.numel()))
    return out, ws


def mpt_tensors_im(curl: Csr, face_w, c, w, U, cond, a, omega, N0, alpha, ws=None):
    """Integration-method analogue (sums over faces of the curl): (n x 12, ws)."""
    h = handle(U.device)
    _dev_check(face_w, c, w, cond, a, omega, N0)
    _dev_check_rows(U)
    N, M = U.shape
    n = omega.numel()
    out = torch.empty((n, 12), dtype=torch.float64, device=U.device)
    nb = lib().mpt_tensors_im_ws_size(N, curl.n, M)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=U.device)
    k = curl.struct()
    h._check(lib().mpt_tensors_im(h.h, C.byref(k), _ptr(face_w), _ptr(c), _ptr(w), _ptr(U), N,
                                  _ld(U), M, _ptr(cond), cond.numel(), _ptr(a), _ptr(omega), n, _ptr(N0),
                                  float(alpha), _ptr(out), _ptr(ws), ws.numel()))
    return out, ws


def mpt_select_snapshots(omega, out, snap, n_star):
    """a5: (new omegas (n_star, NaN if missing), per-interval Lambda_n, Lambda)."""
    h = handle(omega.device)
    _dev_check(omega, out, snap)
    dev = omega.device
    new = torch.empty(n_star, dtype=torch.float64, device=dev)
    lam = torch.empty(snap.numel() - 1, dtype=torch.float64, device=dev)
    Lmax = torch.empty(1, dtype=torch.float64, device=dev)
    ws = torch.empty(lib().mpt_select_snapshots_ws_size(snap.numel()), dtype=torch.uint8, device=dev)
    h._check(lib().mpt_select_snapshots(h.h, _ptr(omega), omega.numel(), _ptr(out), _ptr(snap),
                                        snap.numel(), n_star, _ptr(new), _ptr(lam), _ptr(Lmax),
                                        _ptr(ws), ws.numel()))
    return new, lam, Lmax


def mpt_select_snapshots_static(omega, out, snap, n_star, new=None, lam=None, Lmax=None):
    """a5 without a workspace (the library's static scratch; n_snap <= 4096).
    Output tensors may be passed in, so that the call allocates nothing."""
    h = handle(omega.device)
    _dev_check(omega, out, snap)
    dev = omega.device
    if new is None:
        new = torch.empty(n_star, dtype=torch.float64, device=dev)
    if lam is None:
        lam = torch.empty(snap.numel() - 1, dtype=torch.float64, device=dev)
    if Lmax is None:
        Lmax = torch.empty(1, dtype=torch.float64, device=dev)
    h._check(lib().mpt_select_snapshots_static(h.h, _ptr(omega), omega.numel(), _ptr(out),
                                               _ptr(snap), snap.numel(), n_star, _ptr(new),
                                               _ptr(lam), _ptr(Lmax)))
    return new, lam, Lmax


def mpt_select_snapshots_threshold(omega, out, snap, theta):
    """Threshold variant: (new omegas (n_snap - 1, NaN-padded), count, per-interval
    Lambda_n, Lambda)."""
    h = handle(omega.device)
    _dev_check(omega, out, snap)
    dev = omega.device
    ni = snap.numel() - 1
    new = torch.empty(ni, dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    lam = torch.empty(ni, dtype=torch.float64, device=dev)
    Lmax = torch.empty(1, dtype=torch.float64, device=dev)
    ws = torch.empty(lib().mpt_select_snapshots_ws_size(snap.numel()), dtype=torch.uint8, device=dev)
    h._check(lib().mpt_select_snapshots_threshold(h.h, _ptr(omega), omega.numel(), _ptr(out),
                                                  _ptr(snap), snap.numel(), float(theta), _ptr(new),
                                                  _ptr(cnt), _ptr(lam), _ptr(Lmax), _ptr(ws),
                                                  ws.numel()))
    return new, cnt, lam, Lmax


class Dictionary:
    """Device-side array of Rom structs plus concatenated frequency lists."""

    def __init__(self, roms, omegas, device="cuda"):
        self.roms = list(roms)
        self.n_obj = len(self.roms)
        self._structs = (_Rom * self.n_obj)(*[r.struct() for r in self.roms])
        raw = bytes(self._structs)
        self.dev_structs = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        off = [0]
        for w in omegas:
            off.append(off[-1] + int(w.numel()))
        self.off = (C.c_int64 * (self.n_obj + 1))(*off)
        self.offsets = off
        self.omega = torch.cat([w.to(device=device, dtype=torch.float64) for w in omegas]).contiguous()
        self._ws = {}

    def workspace(self, tune=None):
        """Device workspace of the batched sweeps for a tuning (kept: a
        recorded graph refers to it)."""
        key = None if tune is None else tuple(int(x) for x in tune)
        if key not in self._ws:
            t = None if tune is None else _Tuning(key[0], key[1], key[2], 0)
            n = lib().mpt_sweep_batched_ws_size(self._structs, self.n_obj, self.off,
                                                 C.byref(t) if t is not None else None)
            if n == 0:
                raise MptError("bad dictionary for the batched sweep")
            self._ws[key] = torch.empty(n, dtype=torch.uint8, device=self.omega.device)
        return self._ws[key]


def mpt_sweep_batched(dic: Dictionary, tune=None, use_graph=True, out=None, status=None):
    """a6: all objects in one persistent launch (a HIP graph when use_graph)."""
    h = handle(dic.omega.device)
    n = dic.omega.numel()
    if out is None:
        out = torch.empty((n, 18), dtype=torch.float64, device=dic.omega.device)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=dic.omega.device)
    t = None
    if tune is not None:
        t = _Tuning(int(tune[0]), int(tune[1]), int(tune[2]), 0)
    ws = dic.workspace(tune)
    h._check(lib().mpt_sweep_batched(h.h, dic._structs, _ptr(dic.dev_structs), dic.n_obj, dic.off,
                                     _ptr(dic.omega), _ptr(out), _ptr(status),
                                     C.byref(t) if t is not None else None, int(bool(use_graph)),
                                     _ptr(ws), ws.numel()))
    return out, status


def mpt_sweep_pencil_batched(dic: Dictionary, out=None, status=None, buf=None):
    """Pencil form for a dictionary: every object reduced and swept in one call
    (equal to mpt_sweep_pencil object by object).  Returns (out, status, buf);
    pass buf back to reuse the pencil storage."""
    h = handle(dic.omega.device)
    n = dic.omega.numel()
    dev = dic.omega.device
    if out is None:
        out = torch.empty((n, 18), dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=dev)
    nb = lib().mpt_pencil_batched_bytes(dic._structs, dic.n_obj, dic.off)
    if nb == 0:
        raise MptError("the pencil form takes 1 <= M <= 96 for every object")
    if buf is None or buf.numel() < nb:
        buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    h._check(lib().mpt_sweep_pencil_batched(h.h, dic._structs, dic.n_obj, dic.off, _ptr(dic.omega),
                                            _ptr(buf), buf.numel(), _ptr(out), _ptr(status)))
    return out, status, buf


def mpt_sweep_adjoint(rom: Rom, omega, dout):
    """a7: (dL/domega (n), sigma dL/dsigma (1), status)."""
    h = handle(omega.device)
    _dev_check(omega, dout)
    n = omega.numel()
    dom = torch.empty(n, dtype=torch.float64, device=omega.device)
    sds = torch.empty(1, dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    r = rom.struct()
    h._check(lib().mpt_sweep_adjoint(h.h, C.byref(r), _ptr(omega), n, _ptr(dout), _ptr(dom),
                                     _ptr(sds), _ptr(st)))
    return dom, sds, st


def mpt_sweep_adjoint_materials(rom: Rom, part1: Rom, omega, dout):
    """Per-material sigma sensitivities of a two-material object: part1 is the
    reduced model projected with material 1's conductivities alone (its CM, g
    and E are used).  Returns (dL/domega (n), [sigma_1 dL/dsigma_1,
    sigma_2 dL/dsigma_2] (2), status)."""
    h = handle(omega.device)
    _dev_check(omega, dout, part1.CM, part1.g, part1.E)
    if part1.M != rom.M:
        raise MptError("material part and model must share the basis")
    n = omega.numel()
    dom = torch.empty(n, dtype=torch.float64, device=omega.device)
    sds = torch.empty(2, dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    ws = torch.empty(lib().mpt_sweep_adjoint_materials_ws_size(n), dtype=torch.uint8,
                     device=omega.device)
    r = rom.struct()
    h._check(lib().mpt_sweep_adjoint_materials(h.h, C.byref(r), _ptr(part1.CM), _ptr(part1.g),
                                               _ptr(part1.E), _ptr(omega), n, _ptr(dout),
                                               _ptr(dom), _ptr(sds), _ptr(st), _ptr(ws),
                                               ws.numel()))
    return dom, sds, st


def mpt_sweep_adjoint_batched(dic: Dictionary, dout):
    h = handle(dic.omega.device)
    n = dic.omega.numel()
    dom = torch.empty(n, dtype=torch.float64, device=dic.omega.device)
    sds = torch.empty(dic.n_obj, dtype=torch.float64, device=dic.omega.device)
    st = torch.empty(n, dtype=torch.int32, device=dic.omega.device)
    ws = dic.workspace(None)
    h._check(lib().mpt_sweep_adjoint_batched(h.h, dic._structs, _ptr(dic.dev_structs), dic.n_obj,
                                             dic.off, _ptr(dic.omega), _ptr(dout), _ptr(dom),
                                             _ptr(sds), _ptr(st), _ptr(ws), ws.numel()))
    return dom, sds, st


def mpt_signature(rom: Rom, omega, sigma, sigma0):
    """Sweep outputs (n x 18) at conductivity sigma (device tensor, 1 value)
    for a model projected at sigma0, and status."""
    h = handle(omega.device)
    _dev_check(omega, sigma)
    n = omega.numel()
    out = torch.empty((n, 18), dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    r = rom.struct()
    h._check(lib().mpt_signature(h.h, C.byref(r), _ptr(omega), n, _ptr(sigma), float(sigma0),
                                 _ptr(out), _ptr(st)))
    return out, st


def mpt_signature_adjoint(rom: Rom, omega, sigma, sigma0, dout):
    """(dL/domega (n), dL/dsigma (1), status) for upstream gradients dout."""
    h = handle(omega.device)
    _dev_check(omega, sigma, dout)
    n = omega.numel()
    dom = torch.empty(n, dtype=torch.float64, device=omega.device)
    dsg = torch.empty(1, dtype=torch.float64, device=omega.device)
    st = torch.empty(n, dtype=torch.int32, device=omega.device)
    r = rom.struct()
    h._check(lib().mpt_signature_adjoint(h.h, C.byref(r), _ptr(omega), n, _ptr(sigma),
                                         float(sigma0), _ptr(dout), _ptr(dom), _ptr(dsg),
                                         _ptr(st)))
    return dom, dsg, st


class SweepFn(torch.autograd.Function):
    """Differentiable signature sweep of one object.

    forward(omega, sigma) -> (n, 12) [R~ (6) | I (6)] at conductivity sigma, the
    reduced model having been projected at sigma0; the scaling and the chain
    rule run in the library (mpt_signature, mpt_signature_adjoint)."""

    @staticmethod
    def forward(ctx, omega, sigma, rom, sigma0):
        om = omega.detach().contiguous()
        sg = sigma.detach().reshape(1).contiguous()
        out, st = mpt_signature(rom, om, sg, sigma0)
        ctx.save_for_backward(om, sg)
        ctx.rom, ctx.sigma0, ctx.sig_shape = rom, sigma0, sigma.shape
        return out[:, :12]

    @staticmethod
    def backward(ctx, grad):
        om, sg = ctx.saved_tensors
        dout = torch.zeros((om.numel(), 18), dtype=torch.float64, device=om.device)
        dout[:, :12] = grad
        dom, dsg, _ = mpt_signature_adjoint(ctx.rom, om, sg, ctx.sigma0, dout)
        g_omega = dom if ctx.needs_input_grad[0] else None
        g_sigma = dsg.reshape(ctx.sig_shape) if ctx.needs_input_grad[1] else None
        return g_omega, g_sigma, None, None


def signature(omega, sigma, rom, sigma0):
    return SweepFn.apply(omega, sigma, rom, sigma0)
