"""GPU parity: every hot-path step through the C ABI against the CPU oracle.

Tolerances: tensors R~ and I 1e-10 normwise per frequency (each part relative
to its own largest entry); certificates 1e-8 relative above the rounding floor
of the G-form (64 eps |w|^T|G||w|), absolute below; integer decisions exact."""
import numpy as np
import pytest

from oracle import rom as R
from tests import _cases
from tests._gpu_helpers import (PAIRS, delta_floor, oracle_rom, random_rom, tensor_errors,
                                term_scales)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mpt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_05590_amd import mpt as m
    m.lib()  # fails loudly when the library is missing
    return m


# D'_s formed separately by two projections of one basis (GPU and oracle)
# agree to this much of max |A_s| at the shifts inside the band: it comes from
# Cholesky solves with A_s = A0 + s C_M, whose condition reaches ~1e12 when
# the basis holds gradient-like fields (measured up to 1.6e-9 at 48^3, M = 48)
DP_REL = 1e-8


def _dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _check_sweep(mpt, host, cert, rom_o, alpha, omega, tag, form="lu"):
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(omega, torch.float64)
    if form == "pencil":
        pen = mpt.mpt_pencil_reduce(rom)
        out, st, a_gpu = mpt.mpt_sweep_pencil(pen, w, want_a=True)
        tag = f"{tag} (pencil)"
    else:
        out, st, a_gpu = mpt.mpt_sweep(rom, w, want_a=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert int(st.abs().max()) == 0, tag
    ref, a = R.sweep(rom_o, omega, cert, alpha)
    scales = term_scales(ref, omega, rom_o["N0"], rom_o["E"], alpha)
    eR, eI = tensor_errors(out, ref, scales)
    print(f"{tag}: max err R~ {eR.max():.2e} I {eI.max():.2e}", flush=True)
    assert eR.max() <= 1e-10, tag
    assert eI.max() <= 1e-10, tag
    # reduced solutions: forward error of a backward-stable solve, <= c eps cond(A)
    ag = np.swapaxes(a_gpu.cpu().numpy(), 1, 2)  # (n, M, 3)
    A0 = host["A0"]
    cond = np.array([np.linalg.cond(A0 - 1j * w_ * host["CM"]) for w_ in omega])
    ea = np.linalg.norm(ag - a, axis=(1, 2)) / np.linalg.norm(a, axis=(1, 2))
    print(f"{tag}: solution err / (eps cond) max {np.max(ea / (2.2e-16 * cond)):.2e}", flush=True)
    assert np.all(ea <= 1e3 * 2.2e-16 * cond + 1e-14), tag
    # certificates: the same quadratic forms at the GPU's own solution
    dref = R.pack(R.certificate_gform(cert["G"], cert["Dp"], cert["s_ref"], ag, omega, alpha))
    fl = delta_floor(cert, ag, omega, alpha)
    d = np.abs(out[:, 12:] - dref)
    print(f"{tag}: Delta err / floor max {np.max(d / fl):.2e}", flush=True)
    assert np.all(d <= 1e-8 * np.abs(dref) + fl), tag
    return out


@pytest.mark.parametrize("M", [1, 16, 17, 31, 47, 64, 65, 80, 96])
def test_sweep_random_roms(mpt, M):
    rom_o, cert, host, alpha = random_rom(M, seed=M)
    omega = np.logspace(1, 6, 131)
    rom_o["KM"] = host["KM"]
    _check_sweep(mpt, host, cert, rom_o, alpha, omega, f"random M={M}")


@pytest.mark.parametrize("M", [3, 10, 33, 48])
def test_sweep_ellipsoid_rom(mpt, M):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 6, 257)
    out = _check_sweep(mpt, host, cert, rom_o, fo.alpha, omega, f"ellipsoid16 M={M}")
    # against the explicit mesh sums (the IM analogue) at a few frequencies
    sel = np.arange(0, 257, 32)
    a = R.reduced_solve(rom_o, omega[sel])
    Rt, I = R.tensors_mesh(fo, U, a, omega[sel], c.w, rom_o["N0"])
    ref = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    sc = term_scales(ref, omega[sel], rom_o["N0"], rom_o["E"], fo.alpha)
    eR, eI = tensor_errors(out[sel, :12], ref, sc)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10


def test_sweep_magnetic_rom(mpt):
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :12]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    assert np.abs(rom_o["N0"]).max() > 0
    _check_sweep(mpt, host, cert, rom_o, fo.alpha, np.logspace(1, 6, 65), "magnetic10 M=12")


def test_sweep_empty_and_bad_args(mpt):
    rom_o, cert, host, alpha = random_rom(5, seed=1)
    rom = mpt.Rom.from_host(host, alpha)
    out, st = mpt.mpt_sweep(rom, torch.empty(0, dtype=torch.float64, device="cuda"))
    assert out.shape == (0, 18)
    # an M above the library's limit is rejected on the host before any launch
    bad = mpt.Rom.from_host(host, alpha)
    bad.M = mpt.lib().mpt_max_reduced_dim() + 1
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep(bad, torch.ones(3, dtype=torch.float64, device="cuda"))


def test_sweep_singular_flag(mpt):
    """A zero pencil (A0 = C_M = 0) must be flagged, not silently returned."""
    rom_o, cert, host, alpha = random_rom(4, seed=2)
    host = dict(host)
    host["A0"] = np.zeros((4, 4))
    host["CM"] = np.zeros((4, 4))
    rom = mpt.Rom.from_host(host, alpha)
    out, st = mpt.mpt_sweep(rom, _dev([1.0, 2.0], torch.float64))
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == mpt.MPT_E_SINGULAR)


def test_sweep_deterministic(mpt):
    rom_o, cert, host, alpha = random_rom(40, seed=3)
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(np.logspace(1, 6, 500), torch.float64)
    o1, _ = mpt.mpt_sweep(rom, w)
    o2, _ = mpt.mpt_sweep(rom, w)
    assert torch.equal(o1, o2)


# ------------------------------------------------- pencil form of the sweep
@pytest.mark.parametrize("M", [1, 2, 3, 16, 17, 31, 47, 48, 64, 65, 80, 96])
def test_pencil_random_roms(mpt, M):
    rom_o, cert, host, alpha = random_rom(M, seed=M)
    omega = np.logspace(1, 6, 131)
    rom_o["KM"] = host["KM"]
    _check_sweep(mpt, host, cert, rom_o, alpha, omega, f"random M={M}", form="pencil")


@pytest.mark.parametrize("M", [10, 48])
def test_pencil_ellipsoid_rom(mpt, M):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    _check_sweep(mpt, host, cert, rom_o, fo.alpha, np.logspace(1, 6, 257), f"ellipsoid16 M={M}",
                 form="pencil")


def test_pencil_magnetic_rom(mpt):
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :12]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    _check_sweep(mpt, host, cert, rom_o, fo.alpha, np.logspace(1, 6, 65), "magnetic10 M=12",
                 form="pencil")


@pytest.mark.parametrize("M", [2, 17, 48, 64, 96])
def test_pencil_structure(mpt, M):
    """H upper Hessenberg and T upper triangular (exact zeros), Z unitary, and
    the generalised eigenvalues of (H, T) those of (A0, C_M)."""
    import scipy.linalg as sl

    rom_o, cert, host, alpha = random_rom(M, seed=100 + M)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    H, T, f, Z = (x.cpu().numpy() for x in pen.parts())
    H, T = H.T, T.T  # stored column-major
    assert np.all(np.tril(H, -2) == 0) and np.all(np.tril(T, -1) == 0)
    assert np.abs(Z.conj().T @ Z - np.eye(M)).max() <= 64 * M * 2.2e-16
    ev_ref = np.sort_complex(sl.eigvals(host["CM"], host["A0"]))
    ev = np.sort_complex(sl.eigvals(T, H))
    assert np.abs(ev - ev_ref).max() <= 1e-9 * np.abs(ev_ref).max()


def test_pencil_matches_lu_sweep(mpt):
    rom_o, cert, host, alpha = random_rom(40, seed=7)
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(np.logspace(1, 6, 1000), torch.float64)
    o1, s1 = mpt.mpt_sweep(rom, w)
    o2, s2 = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(rom), w)
    torch.cuda.synchronize()
    assert int(s1.abs().max()) == 0 and int(s2.abs().max()) == 0
    o1, o2 = o1.cpu().numpy(), o2.cpu().numpy()
    for part in range(3):
        a, b = o1[:, 6 * part:6 * part + 6], o2[:, 6 * part:6 * part + 6]
        scale = np.abs(a).max(axis=1, keepdims=True)
        assert np.all(np.abs(a - b) <= 1e-9 * scale), part


def test_pencil_empty_bad_args_singular_deterministic(mpt):
    rom_o, cert, host, alpha = random_rom(5, seed=1)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    out, st = mpt.mpt_sweep_pencil(pen, torch.empty(0, dtype=torch.float64, device="cuda"))
    assert out.shape == (0, 18)
    assert mpt.lib().mpt_pencil_bytes(97, 3) == 0 and mpt.lib().mpt_pencil_bytes(96, 3) > 0
    assert mpt.lib().mpt_pencil_bytes(16, 0) == 0 and mpt.lib().mpt_pencil_bytes(16, 65) == 0
    bad = mpt.Rom.from_host(host, alpha)
    bad.M = 97
    with pytest.raises(mpt.MptError):
        mpt.mpt_pencil_reduce(bad)
    # a zero pencil is flagged
    z = dict(host)
    z["A0"] = np.zeros((5, 5))
    z["CM"] = np.zeros((5, 5))
    pz = mpt.mpt_pencil_reduce(mpt.Rom.from_host(z, alpha))
    out, st = mpt.mpt_sweep_pencil(pz, _dev([1.0, 2.0], torch.float64))
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == mpt.MPT_E_SINGULAR)
    # deterministic, ragged batch tail
    rom_o, cert, host, alpha = random_rom(40, seed=3)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    w = _dev(np.logspace(1, 6, 501), torch.float64)
    o1, _ = mpt.mpt_sweep_pencil(pen, w)
    o2, _ = mpt.mpt_sweep_pencil(pen, w)
    assert torch.equal(o1, o2)


# ------------------------------------------- full matrix method on q = U a
@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("magnetic10", 12), ("ellipsoid16", 70)])
def test_project_pencil_equals_two_calls(mpt, case, M):
    """mpt_project_pencil (the reduction forked beside the certificate data)
    gives exactly mpt_project followed by mpt_pencil_reduce: every rom
    matrix, the pencil's H, T, f, Z and the sweep outputs (which read the
    rest of the pencil), bit for bit."""
    c = getattr(_cases, case)()
    if M <= c.D.shape[1]:
        U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    else:  # beyond the snapshots: a random orthonormal basis (the M > 64 reduction)
        rng = np.random.default_rng(M)
        N = c.D.shape[0]
        U = np.linalg.qr(rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M)))[0]
    ops = c.ops
    args = (mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
            _dev(c.w, torch.float64), _dev(c.o, torch.float64), _dev(ops.vol, torch.float64),
            ops.alpha, _dev(U, torch.complex128), _dev(ops.cond_idx, torch.int32),
            _dev(c.Vt, torch.float64), _dev(c.lam, torch.float64), _dev(c.s_ref, torch.float64))
    w = _dev(np.logspace(1, 6, 333), torch.float64)
    for rep in range(2):  # the second call reuses the handle's private stream and events
        rom1 = mpt.mpt_project(*args)
        pen1 = mpt.mpt_pencil_reduce(rom1)
        rom2, pen2 = mpt.mpt_project_pencil(*args)
        torch.cuda.synchronize()
        for name in ("KM", "A0", "CM", "g", "G", "Dp", "E", "N0"):
            assert torch.equal(getattr(rom1, name), getattr(rom2, name)), name
        for a, b in zip(pen1.parts(), pen2.parts()):
            assert torch.equal(a, b)
        o1, s1 = mpt.mpt_sweep_pencil(pen1, w)
        o2, s2 = mpt.mpt_sweep_pencil(pen2, w)
        assert torch.equal(o1, o2) and torch.equal(s1, s2)
    print(f"{case} M={M}: fused projection + reduction identical", flush=True)


@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("ellipsoid16", 48), ("magnetic10", 12)])
def test_fmm_matches_oracle_and_reduced_sweep(mpt, case, M):
    """GPU FMM vs the oracle's FMM on the same reduced solutions, and vs the
    reduced matrix method of the sweep (equal up to rounding)."""
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    ops = c.ops
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 6, 37)  # three batches of 16 with a ragged tail
    a = R.reduced_solve(rom_o, omega)  # (n, M, 3)
    out, _ = mpt.mpt_tensors_fmm(mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64),
                                 _dev(c.w, torch.float64), _dev(U, torch.complex128),
                                 _dev(ops.cond_idx, torch.int32),
                                 _dev(np.swapaxes(a, 1, 2), torch.complex128),
                                 _dev(omega, torch.float64), _dev(rom_o["N0"], torch.float64),
                                 fo.alpha)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    ref = np.empty((omega.size, 12))
    for k, w_ in enumerate(omega):
        Rt, I = R.tensors_fmm(fo, U @ a[k], w_, c.w, rom_o["N0"])
        ref[k, :6], ref[k, 6:] = R.pack(Rt[None])[0], R.pack(I[None])[0]
    sc = term_scales(ref, omega, rom_o["N0"], rom_o["E"], fo.alpha)
    eR, eI = tensor_errors(out, ref, sc)
    print(f"{case} M={M} FMM vs oracle: R~ {eR.max():.2e} I {eI.max():.2e}", flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10
    # the reduced matrix method (the GPU sweep) reaches the same tensors
    sw, st = mpt.mpt_sweep(mpt.Rom.from_host(host, fo.alpha), _dev(omega, torch.float64))
    torch.cuda.synchronize()
    eR, eI = tensor_errors(sw.cpu().numpy()[:, :12], ref, sc)
    print(f"{case} M={M} MM (GPU sweep) vs FMM: R~ {eR.max():.2e} I {eI.max():.2e}", flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10


@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("magnetic10", 12)])
def test_im_matches_oracle_mesh_sums(mpt, case, M):
    """Integration-method analogue on the GPU (sums over faces of the curl of
    q = U a) vs the oracle's explicit mesh sums on the same reduced solutions."""
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    ops = c.ops
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 6, 21)
    a = R.reduced_solve(rom_o, omega)
    curl = ops.grid.curl()
    fw = 1.0 / (ops.mu_f * ops.grid.h)
    out, _ = mpt.mpt_tensors_im(mpt.Csr.from_scipy(curl), _dev(fw, torch.float64),
                                _dev(ops.c, torch.float64), _dev(c.w, torch.float64),
                                _dev(U, torch.complex128), _dev(ops.cond_idx, torch.int32),
                                _dev(np.swapaxes(a, 1, 2), torch.complex128),
                                _dev(omega, torch.float64), _dev(rom_o["N0"], torch.float64),
                                fo.alpha)
    torch.cuda.synchronize()
    Rt, I = R.tensors_mesh(fo, U, a, omega, c.w, rom_o["N0"])
    ref = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    sc = term_scales(ref, omega, rom_o["N0"], rom_o["E"], fo.alpha)
    eR, eI = tensor_errors(out.cpu().numpy(), ref, sc)
    print(f"{case} M={M} IM vs oracle mesh sums: R~ {eR.max():.2e} I {eI.max():.2e}", flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10


# -------------------------------------------- residual Gram from X^{-1} Z
@pytest.mark.parametrize("case,M", [("ellipsoid16", 4), ("ellipsoid16", 40), ("magnetic10", 12)])
def test_residual_gram_matches_oracle(mpt, case, M):
    c = getattr(_cases, case)()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    Z, Y = c.fs.residual_columns(U, c.w)
    G = mpt.mpt_residual_gram(_dev(Z, torch.complex128), _dev(Y, torch.complex128)).cpu().numpy()
    ref = R.residual_gram_from(Z, Y)
    # rounding of a length-N sum of products, entry by entry
    scale = np.abs(Z).T @ np.abs(Y)
    scale = 0.5 * (scale + scale.T)
    err = np.abs(G - ref) / (64 * 2.2e-16 * scale + 1e-300)
    print(f"{case} M={M} L={2 * M + 3}: residual Gram err / (64 eps |Z|^T|Y|) max {err.max():.2e}",
          flush=True)
    assert np.all(np.abs(G - ref) <= 64 * 2.2e-16 * scale)
    assert np.array_equal(G, G.conj().T)


def test_residual_gram_bad_args(mpt):
    Z = torch.zeros((50, 9), dtype=torch.complex128, device="cuda")
    with pytest.raises(mpt.MptError):
        mpt.mpt_residual_gram(Z, torch.zeros((50, 8), dtype=torch.complex128, device="cuda"))
    with pytest.raises(mpt.MptError):
        Z8 = torch.zeros((50, 8), dtype=torch.complex128, device="cuda")
        mpt.mpt_residual_gram(Z8, Z8)  # 8 is not 2M+3
    big = torch.zeros((10, 2 * 97 + 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(mpt.MptError):
        mpt.mpt_residual_gram(big, big)  # M = 97 > 96


# ------------------------------------------------------------ selection (a5)
def test_select_matches_oracle(mpt):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :8]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 5, 400)
    # the certificates of a real reduced model, computed by the oracle; both
    # selections take the same array
    out, _ = R.sweep(rom_o, omega, cert, fo.alpha)
    snaps = c.snap
    new, lam, Lmax = mpt.mpt_select_snapshots(_dev(omega, torch.float64), _dev(out, torch.float64),
                                              _dev(snaps, torch.float64), 2)
    torch.cuda.synchronize()
    ref_new, ref_L, ref_lam = R.select_snapshots(omega, out[:, 12:], snaps, 2)
    assert np.array_equal(new.cpu().numpy(), ref_new)
    assert Lmax.item() == ref_L
    assert np.array_equal(lam.cpu().numpy(), ref_lam)


@pytest.mark.parametrize("theta", [1.0, 0.7, 0.3, 1e-6])
def test_select_threshold_matches_oracle(mpt, theta):
    rng = np.random.default_rng(int(theta * 1000) + 5)
    n = 3000
    om = np.sort(rng.uniform(10.0, 1e6, n))
    out = np.zeros((n, 18))
    out[:, 12:] = rng.uniform(0.0, 1.0, (n, 6))
    out[100:140, 12:] = 2.0  # a tie block across an interval
    snaps = np.sort(np.r_[rng.uniform(10.0, 1e6, 9), 5.0, 2e6])
    new, cnt, lam, L = mpt.mpt_select_snapshots_threshold(_dev(om, torch.float64),
                                                          _dev(out, torch.float64),
                                                          _dev(snaps, torch.float64), theta)
    torch.cuda.synchronize()
    ref, Lr, lam_r = R.select_snapshots_threshold(om, out[:, 12:], snaps, theta)
    k = int(cnt.item())
    assert k == ref.size and float(L.item()) == Lr
    assert np.array_equal(new.cpu().numpy()[:k], ref)
    assert np.all(np.isnan(new.cpu().numpy()[k:]))
    assert np.array_equal(lam.cpu().numpy(), lam_r)


def test_select_ties_and_empty_intervals(mpt):
    omega = np.arange(1.0, 11.0)
    out = np.zeros((10, 18))
    out[1, 14] = 5.0
    out[2, 12] = 5.0
    out[4, 15] = 7.0
    out[9, 17] = 6.0
    snaps = np.array([1.0, 4.0, 7.0, 10.0, 20.0, 30.0])
    new, lam, Lmax = mpt.mpt_select_snapshots(_dev(omega, torch.float64), _dev(out, torch.float64),
                                              _dev(snaps, torch.float64), 3)
    torch.cuda.synchronize()
    # omega 10 is a snapshot: in no interval, never selected again
    assert list(new.cpu().numpy()) == [5.0, 2.0, 8.0]
    assert Lmax.item() == 7.0
    lam = lam.cpu().numpy()
    assert list(lam[:3]) == [5.0, 7.0, 0.0] and np.all(np.isneginf(lam[3:]))


# --------------------------------------------------------------- spmm / a2
def test_spmm_matches_scipy(mpt):
    c = _cases.ellipsoid16()
    K = mpt.Csr.from_scipy(c.ops.K)
    # the Yee ordering: three equal blocks (edge orientations) in one spatial order
    K3 = mpt.Csr.from_scipy(c.ops.K, row_blocks=3)
    rng = np.random.default_rng(0)
    for M in (1, 7, 16, 33, 48, 96):
        U = rng.standard_normal((c.ops.N, M)) + 1j * rng.standard_normal((c.ops.N, M))
        Ud = _dev(U, torch.complex128)
        Y = mpt.mpt_spmm(K, Ud).cpu().numpy()
        ref = c.ops.K @ U
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max(), M
        # the layout hint changes the schedule only: every row is summed in the same order
        assert np.array_equal(mpt.mpt_spmm(K3, Ud).cpu().numpy(), Y), M


def test_spmm_row_blocks_ragged_and_rejected(mpt):
    # a random sparse matrix whose row count is a multiple of 5 but not of 7,
    # with empty rows and rows longer than one gather batch
    import scipy.sparse as sp
    rng = np.random.default_rng(3)
    n = 5 * 613
    A = sp.random(n, n, density=6.0 / n, random_state=4, format="csr")
    A = (A + sp.diags(rng.standard_normal(n)) + sp.csr_matrix(
        (rng.standard_normal(40), (np.full(40, 17), np.arange(40)), ), shape=(n, n))).tocsr()
    A[100:140] = 0.0
    A.eliminate_zeros()
    U = rng.standard_normal((n, 5)) + 1j * rng.standard_normal((n, 5))
    Ud = _dev(U, torch.complex128)
    Y1 = mpt.mpt_spmm(mpt.Csr.from_scipy(A), Ud).cpu().numpy()
    Y5 = mpt.mpt_spmm(mpt.Csr.from_scipy(A, row_blocks=5), Ud).cpu().numpy()
    ref = A @ U
    assert np.abs(Y1 - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.array_equal(Y5, Y1)
    for bad in (7, -1):
        with pytest.raises(mpt.MptError):
            mpt.mpt_spmm(mpt.Csr.from_scipy(A, row_blocks=bad), Ud)


@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("magnetic10", 12), ("ellipsoid16", 70)])
def test_project_pencil_equals_two_calls(mpt, case, M):
    """mpt_project_pencil (the reduction forked beside the certificate data)
    gives exactly mpt_project followed by mpt_pencil_reduce: every rom
    matrix, the pencil's H, T, f, Z and the sweep outputs (which read the
    rest of the pencil), bit for bit."""
    c = getattr(_cases, case)()
    if M <= c.D.shape[1]:
        U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    else:  # beyond the snapshots: a random orthonormal basis (the M > 64 reduction)
        rng = np.random.default_rng(M)
        N = c.D.shape[0]
        U = np.linalg.qr(rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M)))[0]
    ops = c.ops
    args = (mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
            _dev(c.w, torch.float64), _dev(c.o, torch.float64), _dev(ops.vol, torch.float64),
            ops.alpha, _dev(U, torch.complex128), _dev(ops.cond_idx, torch.int32),
            _dev(c.Vt, torch.float64), _dev(c.lam, torch.float64), _dev(c.s_ref, torch.float64))
    w = _dev(np.logspace(1, 6, 333), torch.float64)
    for rep in range(2):  # the second call reuses the handle's private stream and events
        rom1 = mpt.mpt_project(*args)
        pen1 = mpt.mpt_pencil_reduce(rom1)
        rom2, pen2 = mpt.mpt_project_pencil(*args)
        torch.cuda.synchronize()
        for name in ("KM", "A0", "CM", "g", "G", "Dp", "E", "N0"):
            assert torch.equal(getattr(rom1, name), getattr(rom2, name)), name
        for a, b in zip(pen1.parts(), pen2.parts()):
            assert torch.equal(a, b)
        o1, s1 = mpt.mpt_sweep_pencil(pen1, w)
        o2, s2 = mpt.mpt_sweep_pencil(pen2, w)
        assert torch.equal(o1, o2) and torch.equal(s1, s2)
    print(f"{case} M={M}: fused projection + reduction identical", flush=True)


@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("ellipsoid16", 48), ("magnetic10", 12)])
def test_project_matches_oracle(mpt, case, M):
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    ops = c.ops
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
                          _dev(c.w, torch.float64), _dev(c.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, _dev(U, torch.complex128),
                          _dev(ops.cond_idx, torch.int32), _dev(c.Vt, torch.float64),
                          _dev(c.lam, torch.float64), _dev(c.s_ref, torch.float64))
    torch.cuda.synchronize()
    for name in ("KM", "A0", "CM", "g", "E", "N0"):
        got = getattr(rom, name).cpu().numpy()
        ref = host[name]
        err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
        print(f"{case} M={M} {name}: {err:.2e}", flush=True)
        assert err <= 1e-12, name
    # G_s: weighted Grams of B = V^T sqrt(c) [w | U] over the n_c conductor
    # rows, compared entry by entry with the magnitude of their terms
    # (|B| |B| weighted by |phi|, |chi| or |s chi|); on the X U block A0 -
    # (s chi Gram) also carries the normwise error of A0 itself (max |A0|)
    cond = ops.cond_idx
    lam, V, dc = c.spec
    Zc = np.concatenate([dc[:, None] * c.w[cond], dc[:, None] * U[cond]], 1)
    Bm = np.abs(V.T) @ np.abs(Zc)
    L = M + 3
    got = rom.G.cpu().numpy()
    worst = 0.0
    for k, s in enumerate(c.s_ref):
        chi = 1.0 / (1.0 + s * lam)
        mags = [Bm.T @ (np.abs(f)[:, None] * Bm) for f in (lam * chi, chi, s * chi)]
        Gmag = np.zeros((2 * M + 3, 2 * M + 3))
        for a in range(2 * M + 3):
            for b in range(2 * M + 3):
                xa, xb = 3 <= a < 3 + M, 3 <= b < 3 + M
                ia = a if a < 3 + M else a - M
                ib = b if b < 3 + M else b - M
                f = 2 if (xa and xb) else (1 if (xa or xb) else 0)
                Gmag[a, b] = mags[f][ia, ib] + (np.abs(host["A0"]).max() if f == 2 else 0)
        err = np.abs(got[k] - cert["G"][k]) / np.maximum(Gmag, 1e-300)
        if err.max() > worst:
            worst = err.max()
            print(f"  shift {s:.3g}: worst at {np.unravel_index(err.argmax(), err.shape)}",
                  flush=True)
    print(f"{case} M={M} G_s: {worst:.2e} (relative to term magnitude)", flush=True)
    assert worst <= 1e-12
    # D'_s: Cholesky and triangular solves of A_s = A0 + s C_M.  A_0 = A0 has
    # cond ~ |K_M| / (eps h) (gradient-like basis content): two routes agree
    # to ~1e-10 |A_0| there (shift 0 serves only w below the first shift);
    # the shifts inside the band are far better conditioned
    Dg = rom.Dp.cpu().numpy()
    for k, s in enumerate(c.s_ref):
        As = host["A0"] + s * host["CM"]
        err = np.abs(Dg[k] - cert["Dp"][k]).max() / np.abs(As).max()
        print(f"{case} M={M} D'_s shift {s:.3g}: {err:.2e} of max |A_s|", flush=True)
        assert err <= (1e-8 if s == 0.0 else DP_REL), (k, s, err)
        assert np.array_equal(Dg[k], Dg[k].conj().T)


# ------------------------------------------------------------------- POD a1
@pytest.mark.parametrize("case,tol,cap", [("ellipsoid16", 1e-6, 48), ("ellipsoid16", 1e-12, 20),
                                          ("magnetic10", 1e-8, 24), ("sphere12", 1e-6, 16)])
def test_pod_basis_matches_svd(mpt, case, tol, cap):
    c = getattr(_cases, case)()
    D = c.D
    U_o, s_o, M_o = R.pod_basis(D, tol, cap)
    U, sig, M = mpt.mpt_pod_basis(_dev(D, torch.complex128), tol, cap)
    torch.cuda.synchronize()
    sig = sig.cpu().numpy()
    U = U.cpu().numpy()
    assert M == M_o
    # singular values from the truncation's cut up are resolved; the rest are
    # only bounded by it (pass 2 does not rotate pairs of columns far below)
    cut = max(tol, R.RANK_FLOOR) * s_o[0]
    live = s_o >= cut
    assert np.all(np.abs(sig - s_o)[live] <= 1e-10 * s_o[live] + 1e-13 * s_o[0])
    assert np.all(sig[~live] < cut)
    assert np.abs(U.conj().T @ U - np.eye(M)).max() <= 1e-12
    Pg = U @ (U.conj().T @ D)
    Po = U_o @ (U_o.conj().T @ D)
    assert np.linalg.norm(Pg - Po) <= 1e-12 * np.linalg.norm(D)


def test_end_to_end_ellipsoid(mpt):
    """GPU basis + projection + sweep against the oracle's SVD + projection +
    solves + mesh sums."""
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    ops = c.ops
    U_o, s_o, M = R.pod_basis(c.D, 1e-6, 48)
    rom_o, cert, host = oracle_rom(fo, U_o, c.w, c.o, c.spec, ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 6, 40)
    a = R.reduced_solve(rom_o, omega)
    Rt, I = R.tensors_mesh(fo, U_o, a, omega, c.w, rom_o["N0"])
    ref = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    U, sig, Mg = mpt.mpt_pod_basis(_dev(c.D, torch.complex128), 1e-6, 48)
    assert Mg == M
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
                          _dev(c.w, torch.float64), _dev(c.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, U,
                          _dev(ops.cond_idx, torch.int32), _dev(c.Vt, torch.float64),
                          _dev(c.lam, torch.float64), _dev(c.s_ref, torch.float64))
    out, st = mpt.mpt_sweep(rom, _dev(omega, torch.float64))
    torch.cuda.synchronize()
    sc = term_scales(ref, omega, rom_o["N0"], rom_o["E"], fo.alpha)
    eR, eI = tensor_errors(out.cpu().numpy()[:, :12], ref, sc)
    print(f"end-to-end: R~ {eR.max():.2e} I {eI.max():.2e}", flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10


# --------------------------------------------------------------- adjoint a7
def _objective_weights(out):
    """dJ/dout for J = sum_omega sum_{ij, all 9} I_ij^2 + (R~_ij - N0_ij)^2."""
    mult = np.array([1.0 if i == j else 2.0 for i, j in PAIRS])
    return mult, out


def test_adjoint_matches_forward_sensitivity(mpt):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :10]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    omega = np.logspace(1, 6, 97)
    rom = mpt.Rom.from_host(host, fo.alpha)
    w = _dev(omega, torch.float64)
    out, _ = mpt.mpt_sweep(rom, w)
    o = out.cpu().numpy()
    N0 = np.array([rom_o["N0"][i, j] for i, j in PAIRS])
    mult = np.array([1.0 if i == j else 2.0 for i, j in PAIRS])
    dout = np.zeros((omega.size, 18))
    dout[:, :6] = 2 * (o[:, :6] - N0) * mult
    dout[:, 6:12] = 2 * o[:, 6:12] * mult
    dom, sds, st = mpt.mpt_sweep_adjoint(rom, w, _dev(dout, torch.float64))
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    ref_w, ref_s = R.forward_sensitivity(rom_o, omega, fo.alpha, dout[:, :6], dout[:, 6:12])
    dom = dom.cpu().numpy()
    err = np.abs(dom - ref_w).max() / np.abs(ref_w).max()
    print(f"adjoint dJ/domega rel err {err:.2e}; sigma term {sds.item():.6e} vs {ref_s:.6e}")
    assert err <= 1e-8
    assert abs(sds.item() - ref_s) <= 1e-8 * abs(ref_s)


def _objective_dout(o, N0):
    """dJ/dout for J = sum (R~ - N0)^2 + I^2 over the stored pairs (off-diagonal
    pairs count twice)."""
    mult = np.array([1.0 if i == j else 2.0 for i, j in PAIRS])
    N0p = np.array([N0[i, j] for i, j in PAIRS])
    dout = np.zeros((o.shape[0], 18))
    dout[:, :6] = 2 * (o[:, :6] - N0p) * mult
    dout[:, 6:12] = 2 * o[:, 6:12] * mult
    return dout


def _part_rom(mpt, rom_o, part, alpha):
    M = part["CM"].shape[0]
    host = {"KM": rom_o["KM"], "A0": rom_o["KM"], "CM": part["CM"],
            "g": np.ascontiguousarray(part["g"].T), "G": np.eye(2 * M + 3)[None],
            "Dp": np.eye(M)[None], "s_ref": np.zeros(1), "E": part["E"], "N0": rom_o["N0"]}
    return mpt.Rom.from_host(host, alpha)


def test_material_adjoint_whole_model_is_sigma_identity(mpt):
    # one material: its part is the whole model, and sigma_1 dL/dsigma_1 is
    # sum_k omega_k dL/domega_k; nothing is left for a second material
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :10]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    rom = mpt.Rom.from_host(host, fo.alpha)
    omega = np.logspace(1, 6, 61)
    w = _dev(omega, torch.float64)
    out, _ = mpt.mpt_sweep(rom, w)
    dout = _dev(_objective_dout(out.cpu().numpy(), rom_o["N0"]), torch.float64)
    dom, sds, st = mpt.mpt_sweep_adjoint(rom, w, dout)
    whole = _part_rom(mpt, rom_o, {"CM": rom_o["CM"], "g": rom_o["g"], "E": rom_o["E"]}, fo.alpha)
    dom2, s12, st2 = mpt.mpt_sweep_adjoint_materials(rom, whole, w, dout)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0 and int(st2.abs().max()) == 0
    assert torch.equal(dom, dom2)
    s1, s2 = s12.cpu().numpy()
    print(f"whole-model part: {s1:.6e} vs sigma identity {sds.item():.6e}; rest {s2:.2e}", flush=True)
    assert abs(s1 - sds.item()) <= 1e-10 * abs(sds.item())
    assert abs(s2) <= 1e-10 * abs(sds.item())


def test_material_adjoint_matches_oracle(mpt):
    # two materials that both carry eddy currents (magnetic core in a shell)
    c = _cases.shell16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :10]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    sig = c.ops.sigma_e
    parts = []
    for s_m in np.unique(sig[sig > 0]):
        pr = R.project(fo.K, np.where(sig == s_m, fo.c, 0.0), fo.eps_h, c.w, U)
        parts.append({"CM": pr["CM"], "g": pr["g"], "E": pr["E"]})
    rom = mpt.Rom.from_host(host, fo.alpha)
    omega = np.logspace(1, 6, 97)
    w = _dev(omega, torch.float64)
    out, _ = mpt.mpt_sweep(rom, w)
    dout_h = _objective_dout(out.cpu().numpy(), rom_o["N0"])
    dom, s12, st = mpt.mpt_sweep_adjoint_materials(rom, _part_rom(mpt, rom_o, parts[0], fo.alpha),
                                                   w, _dev(dout_h, torch.float64))
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    ref = R.forward_sensitivity_materials(rom_o, parts, omega, fo.alpha, dout_h[:, :6],
                                          dout_h[:, 6:12])
    ref_w, _ = R.forward_sensitivity(rom_o, omega, fo.alpha, dout_h[:, :6], dout_h[:, 6:12])
    got = s12.cpu().numpy()
    print(f"per-material sigma terms {got} vs oracle {ref}", flush=True)
    assert np.abs(dom.cpu().numpy() - ref_w).max() <= 1e-8 * np.abs(ref_w).max()
    assert np.all(np.abs(got - ref) <= 1e-8 * np.abs(ref).max())


def test_autograd_fd_and_sigma_identity(mpt):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :10]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    rom = mpt.Rom.from_host(host, fo.alpha)
    sigma0 = 5.8e7
    omega = torch.tensor(np.logspace(1, 6, 33), dtype=torch.float64, device="cuda", requires_grad=True)
    sigma = torch.tensor(sigma0, dtype=torch.float64, device="cuda", requires_grad=True)
    N0 = torch.tensor([rom_o["N0"][i, j] for i, j in PAIRS], dtype=torch.float64, device="cuda")
    mult = torch.tensor([1.0 if i == j else 2.0 for i, j in PAIRS], dtype=torch.float64, device="cuda")

    def J(w, s):
        out = mpt.signature(w, s, rom, sigma0)
        return (mult * (out[:, 6:12] ** 2 + (out[:, :6] - N0) ** 2)).sum()

    val = J(omega, sigma)
    val.backward()
    gw = omega.grad.detach().cpu().numpy()
    gs = sigma.grad.item()
    # sigma dJ/dsigma = sum_k omega_k dJ/domega_k (model depends on omega sigma only)
    assert abs(sigma0 * gs - np.sum(omega.detach().cpu().numpy() * gw)) <= 1e-10 * abs(sigma0 * gs)
    with torch.no_grad():
        for k in (0, 9, 20, 32):
            h = 1e-6 * omega[k].item()
            e = torch.zeros_like(omega)
            e[k] = h
            fd = (J(omega + e, sigma) - J(omega - e, sigma)).item() / (2 * h)
            assert abs(fd - gw[k]) <= 1e-5 * abs(gw).max(), k
        hs = 1e-6 * sigma0
        fds = (J(omega, sigma + hs) - J(omega, sigma - hs)).item() / (2 * hs)
        assert abs(fds - gs) <= 1e-5 * abs(gs)


# --------------------------------------------------------------- batched a6
def _dictionary(mpt, n_obj=7):
    roms, omegas, refs = [], [], []
    rng = np.random.default_rng(11)
    for o in range(n_obj):
        M = [1, 8, 16, 20, 33, 48, 64][o % 7]
        rom_o, cert, host, alpha = random_rom(M, seed=100 + o)
        roms.append(mpt.Rom.from_host(host, alpha))
        n = int(rng.integers(1, 300))
        omegas.append(torch.tensor(np.sort(rng.uniform(10, 1e6, n)), dtype=torch.float64, device="cuda"))
    return roms, omegas


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_equals_per_object(mpt, use_graph):
    roms, omegas = _dictionary(mpt)
    dic = mpt.Dictionary(roms, omegas)
    outs = []
    for rep in range(3):
        out, st = mpt.mpt_sweep_batched(dic, tune=(4, 4, 2), use_graph=use_graph)
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum()  # eager work between replays
        outs.append(out.clone())
        assert int(st.abs().max()) == 0
    for o, (r, w) in enumerate(zip(roms, omegas)):
        ref, _ = mpt.mpt_sweep(r, w)
        a, b = dic.offsets[o], dic.offsets[o + 1]
        for out in outs:
            assert torch.equal(out[a:b], ref), o


def test_batched_graph_dropped_when_plan_rewritten(mpt):
    """graph(A), eager(B), graph(A) through one workspace: the eager call
    rewrites the work-item plan the recorded graph reads, so the library must
    record again for A; every call equals the per-object sweeps."""
    roms, omegas = _dictionary(mpt, 7)
    dicA = mpt.Dictionary(roms, omegas)
    dicB = mpt.Dictionary(roms[:3], [w[: max(1, w.numel() // 2)] for w in omegas[:3]])
    wsA = dicA.workspace((4, 4, 2))
    dicB._ws[(4, 4, 2)] = wsA  # B's plan is smaller: it fits A's workspace
    refs = []
    for dic in (dicA, dicB):
        refs.append([mpt.mpt_sweep(r, w)[0] for r, w in zip(dic.roms, omegas[:dic.n_obj])]
                    if dic is dicA else
                    [mpt.mpt_sweep(r, omegas[o][: max(1, omegas[o].numel() // 2)])[0]
                     for o, r in enumerate(dic.roms)])
    for dic, use_graph, ref in ((dicA, True, refs[0]), (dicB, False, refs[1]),
                                (dicA, True, refs[0])):
        out, st = mpt.mpt_sweep_batched(dic, tune=(4, 4, 2), use_graph=use_graph)
        torch.cuda.synchronize()
        assert int(st.abs().max()) == 0
        for o in range(dic.n_obj):
            a, b = dic.offsets[o], dic.offsets[o + 1]
            assert torch.equal(out[a:b], ref[o]), (use_graph, o)


def test_pencil_batched_equals_per_object(mpt):
    roms, omegas = _dictionary(mpt)
    # and one object above M = 64 (two rows per lane)
    rom_o, cert, host, alpha = random_rom(80, seed=180)
    roms.append(mpt.Rom.from_host(host, alpha))
    omegas.append(torch.tensor(np.logspace(1, 6, 77), dtype=torch.float64, device="cuda"))
    dic = mpt.Dictionary(roms, omegas)
    out, st, buf = mpt.mpt_sweep_pencil_batched(dic)
    out2, st2, _ = mpt.mpt_sweep_pencil_batched(dic, buf=buf)  # cached plan
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    assert torch.equal(out, out2)
    for o, (r, w) in enumerate(zip(roms, omegas)):
        ref, s1 = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(r), w)
        a, b = dic.offsets[o], dic.offsets[o + 1]
        assert torch.equal(out[a:b], ref), o


def test_batched_adjoint_equals_per_object(mpt):
    roms, omegas = _dictionary(mpt, 5)
    dic = mpt.Dictionary(roms, omegas)
    rng = np.random.default_rng(4)
    dout = torch.tensor(rng.standard_normal((dic.omega.numel(), 18)), device="cuda")
    dom, sds, st = mpt.mpt_sweep_adjoint_batched(dic, dout)
    torch.cuda.synchronize()
    for o, (r, w) in enumerate(zip(roms, omegas)):
        a, b = dic.offsets[o], dic.offsets[o + 1]
        d1, s1, _ = mpt.mpt_sweep_adjoint(r, w, dout[a:b].contiguous())
        assert torch.equal(dom[a:b], d1)
        assert abs(sds[o].item() - s1.item()) <= 1e-13 * abs(s1.item())


# ------------------------- batched forms against the oracle on real objects
def _gpu_rom(mpt, p, tol, cap):
    """GPU basis (fixed rank: tol, cap) and projection of a generated problem;
    returns (Rom, U on the host)."""
    ops = p.ops
    lam, Vt = p.cond_spectrum()
    U, sig, M = mpt.mpt_pod_basis(_dev(p.D, torch.complex128), tol, cap)
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K, row_blocks=3), _dev(ops.c, torch.float64),
                          ops.eps_h, _dev(p.w, torch.float64),
                          _dev(p.o, torch.float64) if np.any(p.o) else None,
                          _dev(ops.vol, torch.float64), ops.alpha, U,
                          _dev(ops.cond_idx, torch.int32), _dev(Vt, torch.float64),
                          _dev(lam, torch.float64), _dev(p.s_ref, torch.float64))
    return rom, U.cpu().numpy()


def _gpu_rom_on(mpt, p, U):
    """GPU projection of a generated problem onto a given host basis U."""
    ops = p.ops
    lam, Vt = p.cond_spectrum()
    return mpt.mpt_project(mpt.Csr.from_scipy(ops.K, row_blocks=3), _dev(ops.c, torch.float64),
                           ops.eps_h, _dev(p.w, torch.float64),
                           _dev(p.o, torch.float64) if np.any(p.o) else None,
                           _dev(ops.vol, torch.float64), ops.alpha, _dev(U, torch.complex128),
                           _dev(ops.cond_idx, torch.int32), _dev(Vt, torch.float64),
                           _dev(lam, torch.float64), _dev(p.s_ref, torch.float64))


def _oracle_on(p, U):
    """The oracle's reduced model on the GPU's basis U (same span, same basis)."""
    from oracle.grid import FullOrder
    ops = p.ops
    fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
    lam, Vt = p.cond_spectrum()
    spec = (lam, np.ascontiguousarray(Vt.T), np.sqrt(fo.c[ops.cond_idx]))
    return oracle_rom(fo, U, p.w, p.o, spec, ops.cond_idx, p.s_ref), fo


def _dp_abs(rom_o, cert):
    """Absolute uncertainty of D'_s per shift when the GPU projected it."""
    A0 = rom_o["KM"] + rom_o["eps_h"] * rom_o["UhU"]
    return [(1e-8 if s == 0.0 else DP_REL) * np.abs(A0 + s * rom_o["CM"]).max()
            for s in cert["s_ref"]]


def _check_against_oracle(out, rom_o, cert, omega, alpha, tag):
    ref, a = R.sweep(rom_o, omega, cert, alpha)
    sc = term_scales(ref, omega, rom_o["N0"], rom_o["E"], alpha)
    eR, eI = tensor_errors(out[:, :12], ref[:, :12], sc)
    fl = delta_floor(cert, a, omega, alpha, dp_abs=_dp_abs(rom_o, cert))
    d = np.abs(out[:, 12:] - ref[:, 12:])
    print(f"{tag}: R~ {eR.max():.2e} I {eI.max():.2e} Delta err/floor {np.max(d / fl):.2e}",
          flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10, tag
    assert np.all(d <= 1e-8 * np.abs(ref[:, 12:]) + fl), tag


@pytest.fixture(scope="module")
def dict32():
    """Nine objects of the 32^3 dictionary workload (ellipsoids, a cuboid and
    tori; mu_r 1, 8 and 32; random orientation; fixed rank M from 15 to 47;
    1354-3904 frequencies each), snapshots refined to 1e-6 as in the
    benchmark."""
    from synth.workloads import make_problem, region_green
    from synth.yee import YeeGrid
    g = YeeGrid(32)
    C = g.curl()
    print("dictionary32: region Green's function", flush=True)
    gr = region_green("dictionary32", g, verbose=True)
    probs = []
    for o in range(9):
        probs.append(make_problem("dictionary32", o, grid=g, curl=C, tol=1e-6, green=gr))
        pr = probs[-1]
        print(f"dictionary32 object {o}: {pr.draw.shape.kind} mu_r "
              f"{pr.draw.shape.materials[0][1]:g} M={pr.M_cap} n_omega={pr.omega.size}", flush=True)
    return probs


def test_batched_forms_match_oracle_on_dictionary_objects(mpt, dict32):
    """mpt_sweep_batched (LU, graph-captured) and mpt_sweep_pencil_batched on
    real dictionary objects, each object against the oracle's reduced model
    on the same basis: tensors to 1e-10, certificates within their floor."""
    roms, omegas, orc = [], [], []
    for p in dict32:
        rom, U = _gpu_rom(mpt, p, 0.0, p.M_cap)
        (rom_o, cert, _), fo = _oracle_on(p, U)
        roms.append(rom)
        omegas.append(_dev(p.omega, torch.float64))
        orc.append((rom_o, cert, p.omega, p.ops.alpha))
    dic = mpt.Dictionary(roms, omegas)
    out_lu, st_lu = mpt.mpt_sweep_batched(dic, use_graph=True)
    out_pe, st_pe, _ = mpt.mpt_sweep_pencil_batched(dic)
    torch.cuda.synchronize()
    assert int(st_lu.abs().max()) == 0 and int(st_pe.abs().max()) == 0
    out_lu, out_pe = out_lu.cpu().numpy(), out_pe.cpu().numpy()
    for o, (rom_o, cert, omega, alpha) in enumerate(orc):
        a, b = dic.offsets[o], dic.offsets[o + 1]
        sel = np.arange(0, omega.size, 7)
        for form, out in (("batched LU", out_lu), ("batched pencil", out_pe)):
            _check_against_oracle(out[a:b][sel], rom_o, cert, omega[sel], alpha,
                                  f"dictionary32 object {o} ({form}, M={rom_o['KM'].shape[0]})")


@pytest.fixture(scope="module")
def adj48():
    """Four objects of the 48^3 differentiated workload (M 10-27, 2000
    frequencies each), snapshots refined to 1e-6 as in the benchmark."""
    from synth.workloads import make_problem
    from synth.yee import YeeGrid
    g = YeeGrid(48)
    C = g.curl()
    probs = []
    for o in range(4):
        probs.append(make_problem("adjoint48", o, grid=g, curl=C, tol=1e-6, verbose=True))
        print(f"adjoint48 object {o}: M={probs[-1].M_cap}", flush=True)
    return probs


def test_batched_adjoint_matches_oracle(mpt, adj48):
    """mpt_sweep_adjoint_batched on four real 48^3 objects and one reduced
    model with M = 64 (the 64-wide bucket), each object against the oracle's
    forward sensitivities on the same basis: dL/domega and sigma dL/dsigma to
    1e-8 (the objective and its upstream gradient as in the benchmark)."""
    roms, omegas, orc = [], [], []
    for p in adj48:
        rom, U = _gpu_rom(mpt, p, 0.0, p.M_cap)
        (rom_o, cert, _), fo = _oracle_on(p, U)
        roms.append(rom)
        omegas.append(_dev(p.omega[::4], torch.float64))
        orc.append((rom_o, p.omega[::4], p.ops.alpha))
    c = _cases.ellipsoid16_k32()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :64]
    rom_o, cert, host = oracle_rom(fo, U, c.w, c.o, c.spec, c.ops.cond_idx, c.s_ref)
    roms.append(mpt.Rom.from_host(host, fo.alpha))
    om64 = np.logspace(1, 6, 301)
    omegas.append(_dev(om64, torch.float64))
    orc.append((rom_o, om64, fo.alpha))
    dic = mpt.Dictionary(roms, omegas)
    out, st = mpt.mpt_sweep_batched(dic, use_graph=False)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    dout = np.zeros((o.shape[0], 18))
    for k, (rom_o, omega, alpha) in enumerate(orc):
        a, b = dic.offsets[k], dic.offsets[k + 1]
        dout[a:b] = _objective_dout(o[a:b], rom_o["N0"])
    dom, sds, st = mpt.mpt_sweep_adjoint_batched(dic, _dev(dout, torch.float64))
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    dom, sds = dom.cpu().numpy(), sds.cpu().numpy()
    for k, (rom_o, omega, alpha) in enumerate(orc):
        a, b = dic.offsets[k], dic.offsets[k + 1]
        ref_w, ref_s = R.forward_sensitivity(rom_o, omega, alpha, dout[a:b, :6], dout[a:b, 6:12])
        err = np.abs(dom[a:b] - ref_w).max() / np.abs(ref_w).max()
        print(f"batched adjoint object {k} (M={rom_o['KM'].shape[0]}): dJ/domega {err:.2e}, "
              f"sigma term {sds[k]:.6e} vs {ref_s:.6e}", flush=True)
        assert err <= 1e-8
        assert abs(sds[k] - ref_s) <= 1e-8 * abs(ref_s)


def test_shell64_m96_matches_oracle(mpt):
    """The 64^3 two-material sphere at M = 96 (the largest reduced model):
    the LDS sweep for M > 64 and the pencil form, both against the oracle on
    the same basis at every 400th of 10^5 frequencies.  The 144 snapshots have
    numerical rank 45 at TOL 1e-8 (and the POD stops at the numerical rank),
    so the basis here is the first 96 left singular vectors of a host SVD:
    orthonormal, the last ones spanning directions of tiny singular value,
    and the reduced model the Galerkin projection onto them."""
    from synth import make_problem
    p = make_problem("shell64", verbose=True)
    U = np.linalg.svd(p.D, full_matrices=False)[0][:, :96]
    rom = _gpu_rom_on(mpt, p, U)
    assert rom.M == 96
    om = p.omega[::400]
    w = _dev(om, torch.float64)
    out, st = mpt.mpt_sweep(rom, w)
    out_p, st_p = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(rom), w)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0 and int(st_p.abs().max()) == 0
    (rom_o, cert, _), fo = _oracle_on(p, U)
    for form, o in (("LU, M > 64", out), ("pencil", out_p)):
        _check_against_oracle(o.cpu().numpy(), rom_o, cert, om, p.ops.alpha, f"shell64 M=96 ({form})")


def test_large_M_rejected_by_batched_and_adjoint(mpt):
    """The persistent batched and the adjoint kernels take M <= 64: a larger
    reduced model (valid for mpt_sweep) is refused on the host."""
    rom_o, cert, host, alpha = random_rom(70, seed=7)
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(np.logspace(1, 6, 8), torch.float64)
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep_adjoint(rom, w, torch.zeros((8, 18), dtype=torch.float64, device="cuda"))
    dic = mpt.Dictionary([rom], [w])
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep_batched(dic, use_graph=False)


def _rom_to_host(rom):
    """A Rom's matrices on the host, in the oracle's dict layout."""
    KM, CM, A0 = (x.cpu().numpy() for x in (rom.KM, rom.CM, rom.A0))
    r = {"KM": KM, "CM": CM, "A0": A0, "g": rom.g.cpu().numpy().T,
         "E": rom.E.cpu().numpy(), "N0": rom.N0.cpu().numpy()}
    cert = {"s_ref": rom.s_ref.cpu().numpy(), "G": list(rom.G.cpu().numpy()),
            "Dp": list(rom.Dp.cpu().numpy())}
    return r, cert


def _kM_sensitivity(rom_o, omega, alpha, scales, draws=3, seed=0):
    """Spread of R~ and I (relative to the S13 scales) when K_M alone is
    perturbed by Hermitian noise of 1e-16 max |K_M|: how far two correct
    projections of one basis can put the tensors apart at each frequency."""
    rng = np.random.default_rng(seed)
    a = R.reduced_solve(rom_o, omega)
    Rt, I = R.tensors_mm(rom_o, a, omega, rom_o["N0"], alpha)
    base = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    worst = np.zeros(omega.size)
    for _ in range(draws):
        Nn = rng.standard_normal(rom_o["KM"].shape) + 1j * rng.standard_normal(rom_o["KM"].shape)
        r2 = dict(rom_o)
        r2["KM"] = rom_o["KM"] + 1e-16 * np.abs(rom_o["KM"]).max() * 0.5 * (Nn + Nn.conj().T)
        a2 = R.reduced_solve(r2, omega)
        Rt2, I2 = R.tensors_mm(r2, a2, omega, rom_o["N0"], alpha)
        eR, eI = tensor_errors(np.concatenate([R.pack(Rt2), R.pack(I2)], 1), base, scales)
        worst = np.maximum(worst, np.maximum(eR, eI))
    return worst


def test_full_size_ellipsoid48_sampled(mpt):
    """The 48^3 workload at its full size (N = 318,096, 96 snapshot columns,
    M <= 48, 10^4 output frequencies) in the launch configuration the
    benchmark times, checked on every 250th frequency.
    (1) One reduced model: the GPU's projected matrices through the oracle's
        solves and formulas; tensors to 1e-10 normwise, certificates within
        their floor.
    (2) One basis: the oracle projects onto the GPU's basis U: K_M, C_M, g, E,
        N0 to 1e-12 normwise, G_s against the magnitude of its terms, D'_s.
    (3) End to end against the oracle's own SVD basis and projection.  At the
        lowest frequencies R~ is ill-conditioned in K_M (cond(A^M) ~ 1e12:
        a last-bit perturbation of K_M alone moves R~ by up to ~3e-10 of its
        scale), so the bound there is 1e-10 plus 8 times that measured
        spread; the samples above 1e-10 are counted and printed."""
    from synth import make_problem

    p = make_problem("ellipsoid48")
    ops = p.ops
    tol, cap = p.wl.tol_sigma, p.wl.m_cap
    lam, Vt = p.cond_spectrum()
    s_ref = p.s_ref
    print(f"ellipsoid48: N={ops.N} D={p.D.shape} residual={p.snap_residual:.1e} "
          f"n_ref={s_ref.size}", flush=True)
    U, sig, M = mpt.mpt_pod_basis(_dev(p.D, torch.complex128), tol, cap)
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K, row_blocks=3), _dev(ops.c, torch.float64),
                          ops.eps_h, _dev(p.w, torch.float64), _dev(p.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, U,
                          _dev(ops.cond_idx, torch.int32), _dev(Vt, torch.float64),
                          _dev(lam, torch.float64), _dev(s_ref, torch.float64))
    omega_d = _dev(p.omega, torch.float64)
    out, st = mpt.mpt_sweep(rom, omega_d)
    out_p, st_p = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(rom), omega_d)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0 and int(st_p.abs().max()) == 0
    out = out.cpu().numpy()
    out_p = out_p.cpu().numpy()
    U_g = U.cpu().numpy()
    from oracle.grid import FullOrder
    fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
    spec = (lam, np.ascontiguousarray(Vt.T), np.sqrt(fo.c[ops.cond_idx]))
    sel = np.arange(0, p.omega.size, 250)
    om = p.omega[sel]
    # (1) one reduced model
    rom_h, cert_h = _rom_to_host(rom)
    ref_h, a_h = R.sweep(rom_h, om, cert_h, ops.alpha)
    sc = term_scales(ref_h, om, rom_h["N0"], rom_h["E"], ops.alpha)
    fl = delta_floor(cert_h, a_h, om, ops.alpha)
    for form, o in (("lu", out), ("pencil", out_p)):
        eR, eI = tensor_errors(o[sel, :12], ref_h[:, :12], sc)
        d = np.abs(o[sel, 12:] - ref_h[:, 12:])
        print(f"full size, one reduced model ({form}): R~ {eR.max():.2e} I {eI.max():.2e} "
              f"Delta err/floor {np.max(d / fl):.2e}", flush=True)
        assert eR.max() <= 1e-10 and eI.max() <= 1e-10, form
        assert np.all(d <= 1e-8 * np.abs(ref_h[:, 12:]) + fl), form
    # (2) one basis, the oracle's projection
    rom_g, cert_g, host_g = oracle_rom(fo, U_g, p.w, p.o, spec, ops.cond_idx, s_ref)
    for name in ("KM", "A0", "CM", "g", "E", "N0"):
        got = getattr(rom, name).cpu().numpy()
        den = np.abs(host_g[name]).max()
        err = np.abs(got - host_g[name]).max() / den if den > 0 else np.abs(got).max()
        print(f"full size projection {name}: {err:.2e}", flush=True)
        assert err <= 1e-12, name
    Gg = rom.G.cpu().numpy()
    for k in range(s_ref.size):
        assert np.abs(Gg[k] - cert_g["G"][k]).max() <= 1e-10 * np.abs(cert_g["G"][k]).max(), k
    dpa = _dp_abs(rom_g, cert_g)
    Dg = rom.Dp.cpu().numpy()
    for k in range(s_ref.size):
        assert np.abs(Dg[k] - cert_g["Dp"][k]).max() <= dpa[k], k
    # (3) the oracle's own basis
    U_o, s_o, M_o = R.pod_basis(p.D, tol, cap)
    assert M == M_o
    s_g = sig.cpu().numpy()
    # the oracle's LAPACK SVD moves each singular value by up to ~eps ||D||
    # (Weyl), so small ones are compared to that floor as well
    k = int(np.sum(s_o / s_o[0] >= max(tol, R.RANK_FLOOR)))
    dsig = np.abs(s_g[:k] - s_o[:k])
    print(f"full size sigma: max |d sigma| / sigma_1 {dsig.max() / s_o[0]:.1e} "
          f"(sigma_M / sigma_1 = {s_o[k - 1] / s_o[0]:.1e})", flush=True)
    assert np.all(dsig <= 1e-9 * s_o[:k] + 64 * 2.2e-16 * s_o[0])
    rom_o, cert_o, _ = oracle_rom(fo, U_o, p.w, p.o, spec, ops.cond_idx, s_ref)
    ref, a_o = R.sweep(rom_o, om, cert_o, ops.alpha)
    sc = term_scales(ref, om, rom_o["N0"], rom_o["E"], ops.alpha)
    spread = _kM_sensitivity(rom_o, om, ops.alpha, sc)
    bound = 1e-10 + 8.0 * spread
    for form, o in (("lu", out), ("pencil", out_p)):
        eR, eI = tensor_errors(o[sel, :12], ref[:, :12], sc)
        over = int(np.sum((eR > 1e-10) | (eI > 1e-10)))
        print(f"full size, oracle basis ({form}): R~ {eR.max():.2e} I {eI.max():.2e}; "
              f"{over} of {sel.size} samples above 1e-10; K_M last-bit spread max "
              f"{spread.max():.2e}", flush=True)
        assert np.all(eR <= bound) and np.all(eI <= bound), form
    sub = sel[::8]
    Rt, I = R.tensors_mesh(fo, U_o, R.reduced_solve(rom_o, p.omega[sub]), p.omega[sub], p.w,
                           rom_o["N0"])
    im = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    eR, eI = tensor_errors(out[sub, :12], im, term_scales(im, p.omega[sub], rom_o["N0"],
                                                         rom_o["E"], ops.alpha))
    assert np.all(eR <= bound[::8]) and np.all(eI <= bound[::8])
