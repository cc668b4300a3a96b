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


def _dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _check_sweep(mpt, host, G, rom_o, alpha, omega, tag, form="lu"):
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
    ref, a = R.sweep(rom_o, omega, G, alpha)
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
    dref = R.pack(R.certificate_gform(G, ag, omega, alpha))
    fl = delta_floor(G, ag, omega, alpha)
    d = np.abs(out[:, 12:] - dref)
    print(f"{tag}: Delta err / floor max {np.max(d / (2.2e-16 * fl)):.2e}", flush=True)
    assert np.all(d <= 1e-8 * np.abs(dref) + 64 * 2.2e-16 * fl), tag
    return out


@pytest.mark.parametrize("M", [1, 16, 17, 31, 47, 64, 65, 80, 96])
def test_sweep_random_roms(mpt, M):
    rom_o, G, host, alpha = random_rom(M, seed=M)
    omega = np.logspace(1, 6, 131)
    rom_o["KM"] = host["KM"]
    _check_sweep(mpt, host, G, rom_o, alpha, omega, f"random M={M}")


@pytest.mark.parametrize("M", [3, 10, 33, 48])
def test_sweep_ellipsoid_rom(mpt, M):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    omega = np.logspace(1, 6, 257)
    out = _check_sweep(mpt, host, G, rom_o, fo.alpha, omega, f"ellipsoid16 M={M}")
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    assert np.abs(rom_o["N0"]).max() > 0
    _check_sweep(mpt, host, G, rom_o, fo.alpha, np.logspace(1, 6, 65), "magnetic10 M=12")


def test_sweep_empty_and_bad_args(mpt):
    rom_o, G, host, alpha = random_rom(5, seed=1)
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
    rom_o, G, host, alpha = random_rom(4, seed=2)
    host = dict(host)
    host["A0"] = np.zeros((4, 4))
    host["CM"] = np.zeros((4, 4))
    rom = mpt.Rom.from_host(host, alpha)
    out, st = mpt.mpt_sweep(rom, _dev([1.0, 2.0], torch.float64))
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == mpt.MPT_E_SINGULAR)


def test_sweep_deterministic(mpt):
    rom_o, G, host, alpha = random_rom(40, seed=3)
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(np.logspace(1, 6, 500), torch.float64)
    o1, _ = mpt.mpt_sweep(rom, w)
    o2, _ = mpt.mpt_sweep(rom, w)
    assert torch.equal(o1, o2)


# ------------------------------------------------- pencil form of the sweep
@pytest.mark.parametrize("M", [1, 2, 3, 16, 17, 31, 47, 48, 64, 65, 80, 96])
def test_pencil_random_roms(mpt, M):
    rom_o, G, host, alpha = random_rom(M, seed=M)
    omega = np.logspace(1, 6, 131)
    rom_o["KM"] = host["KM"]
    _check_sweep(mpt, host, G, rom_o, alpha, omega, f"random M={M}", form="pencil")


@pytest.mark.parametrize("M", [10, 48])
def test_pencil_ellipsoid_rom(mpt, M):
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    _check_sweep(mpt, host, G, rom_o, fo.alpha, np.logspace(1, 6, 257), f"ellipsoid16 M={M}",
                 form="pencil")


def test_pencil_magnetic_rom(mpt):
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :12]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    _check_sweep(mpt, host, G, rom_o, fo.alpha, np.logspace(1, 6, 65), "magnetic10 M=12",
                 form="pencil")


@pytest.mark.parametrize("M", [2, 17, 48, 64, 96])
def test_pencil_structure(mpt, M):
    """H upper Hessenberg and T upper triangular (exact zeros), Z unitary, and
    the generalised eigenvalues of (H, T) those of (A0, C_M)."""
    import scipy.linalg as sl

    rom_o, G, host, alpha = random_rom(M, seed=100 + M)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    H, T, f, Z = (x.cpu().numpy() for x in pen.parts())
    H, T = H.T, T.T  # stored column-major
    assert np.all(np.tril(H, -2) == 0) and np.all(np.tril(T, -1) == 0)
    assert np.abs(Z.conj().T @ Z - np.eye(M)).max() <= 64 * M * 2.2e-16
    ev_ref = np.sort_complex(sl.eigvals(host["CM"], host["A0"]))
    ev = np.sort_complex(sl.eigvals(T, H))
    assert np.abs(ev - ev_ref).max() <= 1e-9 * np.abs(ev_ref).max()


def test_pencil_matches_lu_sweep(mpt):
    rom_o, G, host, alpha = random_rom(40, seed=7)
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
    rom_o, G, host, alpha = random_rom(5, seed=1)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    out, st = mpt.mpt_sweep_pencil(pen, torch.empty(0, dtype=torch.float64, device="cuda"))
    assert out.shape == (0, 18)
    assert mpt.lib().mpt_pencil_bytes(97) == 0 and mpt.lib().mpt_pencil_bytes(96) > 0
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
    rom_o, G, host, alpha = random_rom(40, seed=3)
    pen = mpt.mpt_pencil_reduce(mpt.Rom.from_host(host, alpha))
    w = _dev(np.logspace(1, 6, 501), torch.float64)
    o1, _ = mpt.mpt_sweep_pencil(pen, w)
    o2, _ = mpt.mpt_sweep_pencil(pen, w)
    assert torch.equal(o1, o2)


# ------------------------------------------- full matrix method on q = U a
@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("ellipsoid16", 48), ("magnetic10", 12)])
def test_fmm_matches_oracle_and_reduced_sweep(mpt, case, M):
    """GPU FMM vs the oracle's FMM on the same reduced solutions, and vs the
    reduced matrix method of the sweep (equal up to rounding)."""
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    ops = c.ops
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, ops.cond_idx)
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, ops.cond_idx)
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    omega = np.logspace(1, 5, 400)
    # the certificates of a real reduced model, computed by the oracle; both
    # selections take the same array
    out, _ = R.sweep(rom_o, omega, G, fo.alpha)
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
    assert list(new.cpu().numpy()) == [5.0, 10.0, 2.0]
    assert Lmax.item() == 7.0
    lam = lam.cpu().numpy()
    assert list(lam[:4]) == [5.0, 7.0, 0.0, 6.0] and np.isneginf(lam[4])


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


@pytest.mark.parametrize("case,M", [("ellipsoid16", 10), ("ellipsoid16", 48), ("magnetic10", 12)])
def test_project_matches_oracle(mpt, case, M):
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :M]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
    ops = c.ops
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
                          _dev(c.w, torch.float64), _dev(c.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, _dev(U, torch.complex128),
                          _dev(ops.cond_idx, torch.int32), _dev(c.S, torch.float64))
    torch.cuda.synchronize()
    for name in ("KM", "A0", "CM", "g", "E", "N0"):
        got = getattr(rom, name).cpu().numpy()
        ref = host[name]
        err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
        print(f"{case} M={M} {name}: {err:.2e}", flush=True)
        assert err <= 1e-12, name
    # G: the blocks built from S = P^T X^{-1} P are sums with heavy cancellation
    # (S carries the 1/(eps h) gradient part), so each entry is compared with
    # the magnitude of its terms, |Z_c|^T |S| |Z_c|.
    got = rom.G.cpu().numpy()
    cond = ops.cond_idx
    Zc = np.concatenate([ops.c[cond, None] * c.w[cond], ops.c[cond, None] * U[cond]], 1)
    mag = np.abs(Zc).T @ np.abs(c.S) @ np.abs(Zc)
    wc = np.r_[0:3, 3 + M:3 + 2 * M]
    Gmag = np.zeros_like(got, dtype=float)
    Gmag[np.ix_(wc, wc)] = mag
    Gmag = np.maximum(Gmag, np.abs(G).max() * 1e-3)
    errG = np.max(np.abs(got - G) / Gmag)
    print(f"{case} M={M} G: {errG:.2e} (relative to term magnitude)", flush=True)
    assert errG <= 1e-12


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
    assert np.all(np.abs(sig - s_o) <= 1e-10 * s_o + 1e-13 * s_o[0])
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
    rom_o, G, host = oracle_rom(fo, U_o, c.w, c.o, c.S, ops.cond_idx)
    omega = np.logspace(1, 6, 40)
    a = R.reduced_solve(rom_o, omega)
    Rt, I = R.tensors_mesh(fo, U_o, a, omega, c.w, rom_o["N0"])
    ref = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    U, sig, Mg = mpt.mpt_pod_basis(_dev(c.D, torch.complex128), 1e-6, 48)
    assert Mg == M
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K), _dev(ops.c, torch.float64), ops.eps_h,
                          _dev(c.w, torch.float64), _dev(c.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, U,
                          _dev(ops.cond_idx, torch.int32), _dev(c.S, torch.float64))
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
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
    host = {"KM": rom_o["KM"], "A0": rom_o["KM"], "CM": part["CM"],
            "g": np.ascontiguousarray(part["g"].T), "G": np.eye(2 * part["CM"].shape[0] + 3),
            "E": part["E"], "N0": rom_o["N0"]}
    return mpt.Rom.from_host(host, alpha)


def test_material_adjoint_whole_model_is_sigma_identity(mpt):
    # one material: its part is the whole model, and sigma_1 dL/dsigma_1 is
    # sum_k omega_k dL/domega_k; nothing is left for a second material
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :10]
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
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
    rom_o, G, host = oracle_rom(fo, U, c.w, c.o, c.S, c.ops.cond_idx)
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
        rom_o, G, host, alpha = random_rom(M, seed=100 + o)
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


def test_pencil_batched_equals_per_object(mpt):
    roms, omegas = _dictionary(mpt)
    # and one object above M = 64 (two rows per lane)
    rom_o, G, host, alpha = random_rom(80, seed=180)
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


def test_large_M_rejected_by_batched_and_adjoint(mpt):
    """The persistent batched and the adjoint kernels take M <= 64: a larger
    reduced model (valid for mpt_sweep) is refused on the host."""
    rom_o, G, host, alpha = random_rom(70, seed=7)
    rom = mpt.Rom.from_host(host, alpha)
    w = _dev(np.logspace(1, 6, 8), torch.float64)
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep_adjoint(rom, w, torch.zeros((8, 18), dtype=torch.float64, device="cuda"))
    dic = mpt.Dictionary([rom], [w])
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep_batched(dic, use_graph=False)


def test_full_size_ellipsoid48_sampled(mpt):
    """The 48^3 workload at its full size (N = 318,096, 96 snapshot columns,
    M <= 48, 10^4 output frequencies) in the launch configuration the
    benchmark times; the oracle (its own LAPACK SVD, projection and residual
    Gram, per-frequency solves, mesh sums) checks a sample of the outputs."""
    from synth import make_problem

    p = make_problem("ellipsoid48")
    ops = p.ops
    tol, cap = p.wl.tol_sigma, p.wl.m_cap
    print(f"ellipsoid48: N={ops.N} D={p.D.shape} residual={p.snap_residual:.1e}", flush=True)
    U, sig, M = mpt.mpt_pod_basis(_dev(p.D, torch.complex128), tol, cap)
    rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K, row_blocks=3), _dev(ops.c, torch.float64),
                          ops.eps_h, _dev(p.w, torch.float64), _dev(p.o, torch.float64),
                          _dev(ops.vol, torch.float64), ops.alpha, U,
                          _dev(ops.cond_idx, torch.int32), _dev(p.S, torch.float64))
    omega_d = _dev(p.omega, torch.float64)
    out, st = mpt.mpt_sweep(rom, omega_d)
    new, lam, Lmax = mpt.mpt_select_snapshots(omega_d, out, _dev(np.sort(p.snap_omega),
                                                                 torch.float64), 2)
    out_p, st_p = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(rom), omega_d)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0 and int(st_p.abs().max()) == 0
    out = out.cpu().numpy()
    out_p = out_p.cpu().numpy()
    # oracle
    from oracle.grid import FullOrder
    fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
    U_o, s_o, M_o = R.pod_basis(p.D, tol, cap)
    assert M == M_o
    s_g = sig.cpu().numpy()
    k = int(np.sum(s_o / s_o[0] >= 1e-10))
    assert np.all(np.abs(s_g[:k] - s_o[:k]) <= 1e-9 * s_o[:k])
    rom_o, G, host = oracle_rom(fo, U_o, p.w, p.o, p.S, ops.cond_idx)
    sel = np.arange(0, p.omega.size, 250)
    ref, a_o = R.sweep(rom_o, p.omega[sel], G, ops.alpha)
    sc = term_scales(ref, p.omega[sel], rom_o["N0"], rom_o["E"], ops.alpha)
    # the GPU and the oracle solve in two different (equally valid) bases of
    # the same subspace, so where the reduced system is ill-conditioned their
    # backward-stable solves agree to ~eps cond(A^M(w)) only
    A0o = rom_o["KM"] + fo.eps_h * rom_o["UhU"]
    kap = np.array([np.linalg.cond(A0o - 1j * w_ * rom_o["CM"]) for w_ in p.omega[sel]])
    bound = 1e-10 + 64 * 2.2e-16 * kap
    for form, o in (("lu", out), ("pencil", out_p)):
        eR, eI = tensor_errors(o[sel, :12], ref[:, :12], sc)
        print(f"full size sampled ({form}): R~ {eR.max():.2e} I {eI.max():.2e}; cond max "
              f"{kap.max():.2e}; worst R~ err / (eps cond) {np.max(eR / (2.2e-16 * kap)):.2e} "
              f"at w={p.omega[sel][np.argmax(eR)]:.3e}", flush=True)
        assert np.all(eR <= bound) and np.all(eI <= bound), form
    # the integral-method analogue (explicit mesh sums) at a few of them
    sub = sel[::8]
    Rt, I = R.tensors_mesh(fo, U_o, R.reduced_solve(rom_o, p.omega[sub]), p.omega[sub], p.w,
                           rom_o["N0"])
    im = np.concatenate([R.pack(Rt), R.pack(I)], 1)
    eR, eI = tensor_errors(out[sub, :12], im, term_scales(im, p.omega[sub], rom_o["N0"],
                                                         rom_o["E"], ops.alpha))
    assert np.all(eR <= bound[::8]) and np.all(eI <= bound[::8])
    # certificates against the oracle's own, within the G-form rounding floor
    fl = delta_floor(G, a_o, p.omega[sel], ops.alpha)
    for form, o in (("lu", out), ("pencil", out_p)):
        d = np.abs(o[sel, 12:] - ref[:, 12:])
        print(f"full size Delta err / floor max ({form}) {np.max(d / (2.2e-16 * fl)):.2e}",
              flush=True)
        assert np.all(d <= 1e-8 * np.abs(ref[:, 12:]) + 64 * 2.2e-16 * fl), form
