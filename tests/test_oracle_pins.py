"""Pins of the CPU oracle (and of the seeded inputs) against what the paper and
the mathematics fix: closed forms, invariants, limits, exact identities, brute
force and library routines on tiny inputs.  No GPU needed."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import rom as R
from oracle.grid import FullOrder, Grid
from tests import _cases


# ----------------------------------------------------------------- grid
def test_oracle_and_input_operators_agree():
    """Two independent constructions of K, x (index formulas vs lookup tables)."""
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    assert (abs(fo.K - c.ops.K)).max() < 1e-14 * abs(fo.K).max()
    assert np.abs(fo.x - c.ops.x).max() == 0.0


def test_curl_of_gradient_vanishes_and_stokes():
    g = Grid(7)
    C = g.curl()
    n = g.n
    # node gradient on interior nodes
    nid = -np.ones((n + 1,) * 3, int)
    nodes = np.argwhere(np.ones((n - 1,) * 3, bool)) + 1
    nid[tuple(nodes.T)] = np.arange(len(nodes))
    rows, cols, vals = [], [], []
    for a in range(3):
        st = g.edge_start[a]
        e0 = g.table[a][tuple(st.T)]
        for nd, s in ((st + np.eye(3, dtype=int)[a], 1.0), (st, -1.0)):
            ii = nid[tuple(nd.T)]
            k = ii >= 0
            rows.append(e0[k]); cols.append(ii[k]); vals.append(np.full(k.sum(), s))
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.N, len(nodes)))
    assert abs(C @ G).max() == 0.0
    # Stokes: circulation of e_i x xi round an interior face is 2 h^2 (e_i . n_f)
    x = g.source_dofs()
    Cx = C @ x
    ax = g.face_normal_axis()
    interior = np.ones(C.shape[0], bool)
    f0 = 0
    for a, fs in enumerate(g.face_start):
        b, cc = (a + 1) % 3, (a + 2) % 3
        ok = (fs[:, b] >= 1) & (fs[:, b] <= n - 2) & (fs[:, cc] >= 1) & (fs[:, cc] <= n - 2)
        interior[f0:f0 + len(fs)] = ok
        f0 += len(fs)
    for i in range(3):
        expect = 2 * g.h ** 2 * (ax == i)
        assert np.allclose(Cx[interior, i], expect[interior], atol=1e-13)


def test_K_symmetric_psd_and_sparsity():
    c = _cases.ellipsoid16()
    K = c.ops.K
    assert abs(K - K.T).max() == 0.0
    assert np.diff(K.indptr).max() <= 13
    v = np.random.default_rng(0).standard_normal((K.shape[0], 4))
    assert np.all(np.einsum("ij,ij->j", v, K @ v) >= 0)


# ------------------------------------------------------------ snapshots
@pytest.mark.parametrize("case", ["ellipsoid16", "magnetic10"])
def test_snapshot_residual_and_reciprocity(case):
    c = getattr(_cases, case)()
    fo = c.oracle_fo()
    K = c.snap.size
    for k, om in enumerate(c.snap):
        q = c.D[:, [k, K + k, 2 * K + k]]
        r = fo.rhs(om, c.w)
        res = r - fo.A(om) @ q
        assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(r)
        # complex symmetry of A: w_i^T C q_j = w_j^T C q_i
        Mx = c.w.T @ (fo.c[:, None] * q)
        assert np.abs(Mx - Mx.T).max() <= 1e-9 * np.abs(Mx).max()


def test_snapshot_tensors_match_sparse_direct():
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    om = c.snap[5]
    q_ref = fo.full_solve(om, c.w)
    K = c.snap.size
    q = c.D[:, [5, K + 5, 2 * K + 5]]
    R1, I1 = R.tensors_fmm(fo, q, om, c.w, np.zeros((3, 3)))
    R2, I2 = R.tensors_fmm(fo, q_ref, om, c.w, np.zeros((3, 3)))
    assert np.abs(R1 - R2).max() <= 1e-9 * np.abs(R2).max()
    assert np.abs(I1 - I2).max() <= 1e-9 * np.abs(I2).max()


def test_theta0_magnetostatic_residual():
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    b = -((fo.K - fo.K1) @ c.ops.x)
    res = b - fo.X @ c.o
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b)


# ------------------------------------------------------------------ POD
def test_truncation_rule_examples():
    s = np.array([1.0, 0.5, 1e-3, 1e-3 * (1 - 1e-12), 1e-7, 1e-9])
    assert R.truncation_rank(s, 1e-6, 10) == 4  # s_5 = 1e-7 < 1e-6 dropped
    assert R.truncation_rank(s, 1e-8, 10) == 5
    assert R.truncation_rank(s, 1e-2, 10) == 2
    assert R.truncation_rank(s, 1e-8, 3) == 2  # cap 3 would split the 1e-3 pair
    assert R.truncation_rank(s, 1e-8, 4) == 4
    assert R.truncation_rank(s, 1e-10, 99) == 6


def test_fixed_rank_stops_at_the_numerical_rank():
    """tol = 0 keeps every singular value down to the rounding floor of FP64
    and none below: a rank-5 matrix of 12 columns gives M = 5, and the basis
    spans its column space."""
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((400, 5)) + 1j * rng.standard_normal((400, 5))) @ \
        (rng.standard_normal((5, 12)) * np.logspace(0, -9, 5)[:, None])
    U, s, M = R.pod_basis(A, 0.0, 12)
    assert M == 5 and s[5] / s[0] < 1e-14 and s[4] / s[0] > 1e-11
    assert np.abs(U @ (U.conj().T @ A) - A).max() <= 1e-13 * np.abs(A).max()


def test_pod_basis_reconstructs_and_is_orthonormal():
    c = _cases.ellipsoid16()
    U, s, M = R.pod_basis(c.D, 1e-6, 99)
    assert np.abs(U.conj().T @ U - np.eye(M)).max() < 1e-13
    proj = c.D - U @ (U.conj().T @ c.D)
    assert np.linalg.norm(proj, 2) <= 1.01 * s[M] if M < s.size else True
    # singular values squared are the eigenvalues of the Gram matrix (leading part)
    ev = np.sort(np.linalg.eigvalsh(c.D.conj().T @ c.D))[::-1]
    assert np.allclose(ev[:4], s[:4] ** 2, rtol=1e-10)


# ------------------------------------------------------- sweep / tensors
def _rom(c, M, fo=None):
    fo = fo or c.oracle_fo()
    U, s, _ = np.linalg.svd(c.D, full_matrices=False)
    U = U[:, :M]
    rom = R.project(fo.K, fo.c, fo.eps_h, c.w, U)
    rom["N0"] = R.static_tensor_mesh(fo, c.o)
    return fo, U, rom


def test_mm_equals_mesh_sums():
    """Section 9 (Conclusions): IM, FMM and MM give the same tensors up to rounding."""
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 10)
    om = np.logspace(1, 6, 7)
    a = R.reduced_solve(rom, om)
    Rt, I = R.tensors_mesh(fo, U, a, om, c.w, rom["N0"])
    Rm, Im = R.tensors_mm(rom, a, om, rom["N0"], fo.alpha)
    for k in range(om.size):
        Rf, If = R.tensors_fmm(fo, U @ a[k], om[k], c.w, rom["N0"])
        assert np.abs(Rf - Rt[k]).max() <= 1e-12 * np.abs(Rt[k]).max()
        scale_I = max(np.abs(I[k]).max(), 0.25 * fo.alpha ** 3 * om[k] * np.abs(rom["E"]).max())
        assert np.abs(If - I[k]).max() <= 1e-12 * scale_I
    assert np.abs(Rm - Rt).max() <= 1e-12 * np.abs(Rt).max()
    for k in range(om.size):
        scale_I = max(np.abs(I[k]).max(), 0.25 * fo.alpha ** 3 * om[k] * np.abs(rom["E"]).max())
        assert np.abs(Im[k] - I[k]).max() <= 1e-12 * scale_I


def test_untruncated_pod_reproduces_full_order_at_snapshots():
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 3 * c.snap.size)
    a = R.reduced_solve(rom, c.snap)
    Rt, I = R.tensors_mesh(fo, U, a, c.snap, c.w, rom["N0"])
    K = c.snap.size
    for k in range(K):
        q = c.D[:, [k, K + k, 2 * K + k]]
        Rf, If = R.tensors_fmm(fo, q, c.snap[k], c.w, rom["N0"])
        assert np.abs(Rf - Rt[k]).max() <= 1e-10 * np.abs(Rf).max()
        assert np.abs(If - I[k]).max() <= 1e-10 * np.abs(If).max()


def test_sphere_tensor_is_isotropic():
    p = _cases.sphere12()
    fo = FullOrder(p.ops.grid.n, p.ops.sigma_e, p.ops.mu_f, p.ops.alpha, p.ops.eps)
    U, s, M = R.pod_basis(p.D, p.wl.tol_sigma, p.M_cap)
    rom = R.project(fo.K, fo.c, fo.eps_h, p.w, U)
    rom["N0"] = R.static_tensor_mesh(fo, p.o)
    om = p.omega[::25]
    a = R.reduced_solve(rom, om)
    Rt, I = R.tensors_mesh(fo, U, a, om, p.w, rom["N0"])
    for T in (Rt, I):
        sc = np.abs(T).max()
        off = T - np.einsum("kii->ki", T)[:, :, None] * np.eye(3)
        assert np.abs(off).max() <= 1e-12 * sc
        d = np.einsum("kii->ki", T)
        assert np.abs(d - d[:, :1]).max() <= 1e-12 * sc


# full-order (R~11, I11) of the 12^3 sphere from an independent FEM-free
# computation of the same stand-in: the snapshot frequencies 10^(1 + 4k/15),
# k = 0, 5, 10, 15, and a separate solve at 1e3 rad/s
PROBES_SPHERE12 = (
    (1e1, -7.6801807e-10, 5.85715825e-08),
    (10.0 ** (1.0 + 4.0 * 5 / 15), -3.30192365e-07, 1.16882425e-06),
    (1e3, -2.824737e-06, 2.154237e-06),
    (10.0 ** (1.0 + 4.0 * 10 / 15), -4.35019211e-06, 7.14755144e-07),
    (1e5, -4.4673696e-06, 3.40696291e-08),
)


@pytest.mark.parametrize("omega,r11,i11", PROBES_SPHERE12)
def test_probe_values_sphere12(omega, r11, i11):
    """Full-order R~11 and I11 of the tiny sphere against the probe values
    (given to 7-9 significant digits)."""
    p = _cases.sphere12()
    fo = FullOrder(p.ops.grid.n, p.ops.sigma_e, p.ops.mu_f, p.ops.alpha, p.ops.eps)
    q = fo.full_solve(omega, p.w)
    Rf, If = R.tensors_fmm(fo, q, omega, p.w, np.zeros((3, 3)))
    assert abs(Rf[0, 0] - r11) <= 2e-7 * abs(r11)
    assert abs(If[0, 0] - i11) <= 2e-7 * abs(i11)


def test_definiteness_and_limits():
    """I is PSD, R = R~ - N0 is NSD; R ~ w^2 and I ~ w at low w; I ~ 1/w at high w."""
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    N0 = R.static_tensor_mesh(fo, c.o)

    def tens(om):
        q = fo.full_solve(om, c.w)
        return R.tensors_fmm(fo, q, om, c.w, N0)

    for om in (1e2, 1e4):
        Rt, I = tens(om)
        assert np.linalg.eigvalsh(I).min() >= -1e-12 * np.abs(I).max()
        assert np.linalg.eigvalsh(Rt - N0).max() <= 1e-12 * np.abs(Rt - N0).max()
    R1, I1 = tens(1e-3)
    R2, I2 = tens(2e-3)
    assert np.allclose(np.diag(R2 - N0) / np.diag(R1 - N0), 4.0, rtol=1e-4)
    assert np.allclose(np.diag(I2) / np.diag(I1), 2.0, rtol=1e-4)
    R3, I3 = tens(1e10)
    R4, I4 = tens(2e10)
    d = np.diag(I4) / np.diag(I3)
    assert np.all(np.abs(d - 0.5) < 0.02)


def test_scaling_law_and_omega_sigma_dependence():
    """Remark 6.2: M[s alpha B, w] = s^3 M[alpha B, s^2 w] on the same grid."""
    c = _cases.cube10_mu()
    o = c.ops
    s = 1.7
    fo1 = FullOrder(c.grid.n, o.sigma_e, o.mu_f, o.alpha, o.eps)
    fo2 = FullOrder(c.grid.n, o.sigma_e, o.mu_f, s * o.alpha, o.eps)
    fo3 = FullOrder(c.grid.n, 2.0 * o.sigma_e, o.mu_f, o.alpha, o.eps)
    w = c.w  # theta0 does not depend on alpha or sigma
    om = 3e3
    N0a = R.static_tensor_mesh(fo1, c.o)
    N0b = R.static_tensor_mesh(fo2, c.o)
    Ra, Ia = R.tensors_fmm(fo1, fo1.full_solve(s * s * om, w), s * s * om, w, N0a)
    Rb, Ib = R.tensors_fmm(fo2, fo2.full_solve(om, w), om, w, N0b)
    assert np.abs(Rb - s ** 3 * Ra).max() <= 1e-9 * np.abs(Rb).max()
    assert np.abs(Ib - s ** 3 * Ia).max() <= 1e-9 * np.abs(Ib).max()
    Rc, Ic = R.tensors_fmm(fo3, fo3.full_solve(om, w), om, w, N0a)
    Rd, Id = R.tensors_fmm(fo1, fo1.full_solve(2 * om, w), 2 * om, w, N0a)
    assert np.abs(Rc - Rd).max() <= 1e-9 * np.abs(Rc).max()
    assert np.abs(Ic - Id).max() <= 1e-9 * np.abs(Ic).max()


def test_static_tensor_two_forms_and_sphere_symmetry():
    c = _cases.magnetic10()
    fo = c.oracle_fo()
    N0 = R.static_tensor_mesh(fo, c.o)
    a3 = fo.alpha ** 3
    N0x = 0.25 * a3 * (c.ops.x.T @ ((fo.K1 - fo.K) @ c.ops.x) + c.o.T @ (fo.K @ c.o))
    assert np.abs(N0 - N0x).max() <= 1e-12 * np.abs(N0).max()
    assert np.abs(N0 - N0[0, 0] * np.eye(3)).max() <= 1e-10 * abs(N0[0, 0])
    assert N0[0, 0] > 0
    # magnetic ball of radius r_in: 3 V (mu-1)/(mu+2) alpha^3 within staircase error
    V = 4.0 / 3.0 * np.pi * 1.0 ** 3
    assert 0.5 < N0[0, 0] / (a3 * 3 * V * 49.0 / 52.0) < 1.5


# --------------------------------------------------------- certificates
S_REF16 = np.r_[0.0, 10.0 ** np.arange(1.0, 6.01, 0.5)]  # reference shifts, 2 per decade


def _spectral_lu(c, fo):
    """Conductor block of X^{-1} by SuperLU and its scaled eigenpairs."""
    cond = c.ops.cond_idx
    E = np.zeros((fo.grid.N, cond.size))
    E[cond, np.arange(cond.size)] = 1.0
    S = fo.X_solve(E)[cond]
    S = 0.5 * (S + S.T)
    d = np.sqrt(fo.c[cond])
    lam, V = np.linalg.eigh(d[:, None] * S * d[None, :])
    return lam, V, d


def test_residual_gram_spectral_equals_direct():
    """G_s = Z^H (X + s C)^{-1} Z from the conductor block's eigenpairs
    (Woodbury) equals the one from a SuperLU factorisation of X + s C, block
    by block; with the input generator's conductor block at s = 0 as well."""
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 8)
    M = 8
    A0 = rom["KM"] + fo.eps_h * rom["UhU"]
    cond = c.ops.cond_idx
    blocks = [(slice(0, 3), slice(0, 3)), (slice(0, 3), slice(3, 3 + M)),
              (slice(0, 3), slice(3 + M, None)), (slice(3, 3 + M), slice(3, 3 + M)),
              (slice(3, 3 + M), slice(3 + M, None)), (slice(3 + M, None), slice(3 + M, None))]
    lam, V, d = _spectral_lu(c, fo)
    for s in (0.0, 10.0, 1e3, 1e5):
        Gd = R.residual_gram_direct(fo, U, c.w, s)
        Gs = R.residual_gram_spectral(lam, V, d, cond, c.w, U, A0, s)
        assert np.abs(Gs - Gs.conj().T).max() == 0.0
        # X + s C has cond ~ 1e12: the two backward-stable routes agree to a
        # few eps * cond per block, a wrong weight, sign or block at O(1)
        for b in blocks:
            assert np.abs(Gs[b] - Gd[b]).max() <= 1e-3 * np.abs(Gd[b]).max()
    lam_h, V_h, d_h = c.fs._eig()
    Gh = R.residual_gram_spectral(lam_h, V_h, d_h, cond, c.w, U, A0, 0.0)
    assert np.abs(Gh - R.residual_gram_direct(fo, U, c.w, 0.0)).max() <= 1e-5 * np.abs(Gh).max()


def test_conj_defect_vanishes_for_conjugation_closed_span():
    """The linear term of the certificate measures how far conj(U a) is from
    span(U): zero for a real basis, positive for the complex POD basis, and
    equal to the full-order distance."""
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 6)
    Ur, _ = np.linalg.qr(np.concatenate([c.D.real[:, :3], c.D.imag[:, 5:8]], 1))
    romr = R.project(fo.K, fo.c, fo.eps_h, c.w, Ur.astype(np.complex128))
    for s in (0.0, 1e3):
        D = R.conj_defect_matrix(romr, s) - 4.0 * fo.eps_h * romr["UhU"]
        A = romr["KM"] + s * romr["CM"]
        assert np.abs(D).max() <= 1e-10 * np.abs(A).max()
        Dc = R.conj_defect_matrix(rom, s)
        assert np.linalg.eigvalsh(Dc).min() > -1e-12 * np.abs(Dc).max()
        # a^H D_s a against ||conj(q) - Pi conj(q)||^2 formed at full order
        import scipy.sparse as sps
        Xs = fo.X + s * sps.diags(fo.c)
        a = np.exp(1j * np.arange(6)) * np.linspace(1.0, 2.0, 6)
        q = U @ a
        cq = q.conj()
        cc = np.linalg.solve(U.conj().T @ (Xs @ U), U.conj().T @ (Xs @ cq))
        dv = cq - U @ cc
        d2 = np.real(np.vdot(dv, Xs @ dv))
        lhs = np.real(a.conj() @ (2.0 * (Dc - 4.0 * fo.eps_h * rom["UhU"])) @ a)
        assert d2 > 1e-6 * np.real(np.vdot(cq, Xs @ cq))
        assert abs(lhs - d2) <= 1e-6 * np.real(np.vdot(cq, Xs @ cq))


def test_certificate_gform_equals_direct_residual():
    """Lemma 4.1 evaluated from the Grams equals the same bound formed from
    full-order residuals, dual norms and the conjugation defect."""
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 4)
    A0 = rom["KM"] + fo.eps_h * rom["UhU"]
    om = np.array([3e1, 1e3, 3e4, 7e5])
    a = R.reduced_solve(rom, om)
    Dd = R.certificate_direct(fo, U, a, om, c.w, S_REF16)
    assert np.all(Dd >= 0)
    lam, V, d = _spectral_lu(c, fo)
    cert = R.certificate_data(rom, S_REF16, lambda s: R.residual_gram_spectral(
        lam, V, d, c.ops.cond_idx, c.w, U, A0, s))
    Dg = R.certificate_gform(cert["G"], cert["Dp"], S_REF16, a, om, fo.alpha)
    assert np.all(np.abs(Dg - Dd) <= 1e-3 * Dd)
    cert_lu = R.certificate_data(rom, S_REF16, lambda s: R.residual_gram_direct(fo, U, c.w, s))
    Dl = R.certificate_gform(cert_lu["G"], cert_lu["Dp"], S_REF16, a, om, fo.alpha)
    assert np.all(np.abs(Dl - Dd) <= 1e-8 * Dd)
    # with the input generator's conductor block (spectral X^{-1}, accurate to
    # ~1e-5 relative) the bound moves by at most a few percent
    lam_h, V_h, d_h = c.fs._eig()
    cert_h = R.certificate_data(rom, S_REF16, lambda s: R.residual_gram_spectral(
        lam_h, V_h, d_h, c.ops.cond_idx, c.w, U, A0, s))
    Dh = R.certificate_gform(cert_h["G"], cert_h["Dp"], S_REF16, a, om, fo.alpha)
    assert np.all(np.abs(Dh - Dd) <= 5e-2 * Dd)


@pytest.mark.parametrize("M", [3, 4, 6])
def test_lemma41_bounds_the_tensor_error(M):
    """Lemma 4.1: |R~ - R~^PODP|_ij <= Delta_ij and |I - I^PODP|_ij <= Delta_ij,
    against refined sparse-direct full-order solutions.  Effectivity
    Delta / error: at most 2e3 on every entry whose error stands above the
    full-order solve's accuracy, and at most 25 on the tightest entry of each
    frequency (measured: 2.0 - 23 on the tightest, up to 950 overall)."""
    import scipy.sparse.linalg as spla
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, M)
    om = np.array([30.0, 3e2, 3e3, 3e4, 3e5])
    a = R.reduced_solve(rom, om)
    Rt, It = R.tensors_mm(rom, a, om, rom["N0"], fo.alpha)
    Dd = R.certificate_direct(fo, U, a, om, c.w, S_REF16)
    for k, w in enumerate(om):
        A = fo.A(w)
        r = fo.rhs(w, c.w)
        lu = spla.splu(A)
        q = lu.solve(r)
        for _ in range(2):
            q = q + lu.solve(r - A @ q)
        Rf, If = R.tensors_fmm(fo, q, w, c.w, rom["N0"])
        tight = np.inf
        for T, Tp in ((Rf, Rt[k]), (If, It[k])):
            err = np.abs(T - Tp)
            assert np.all(err <= Dd[k]), (w, err / Dd[k])
            live = err > 1e-6 * np.abs(T).max()
            assert live.any()
            eff = Dd[k][live] / err[live]
            assert eff.max() <= 2e3, (w, eff)
            tight = min(tight, eff.min())
        # one Delta serves both parts: tight on the part with the larger error
        assert tight <= 25.0, (w, tight)


# ------------------------------------------------------------ selection
def test_select_snapshots_worked_example():
    om = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 10.0])
    snaps = np.array([1.0, 4.0, 7.0, 10.0])
    d = np.zeros((10, 6))
    d[1, 2] = 5.0  # interval 0 (1 < w < 4): max 5 at omega 2
    d[2, 0] = 5.0  # tie inside interval 0 -> smaller omega (2) wins
    d[4, 3] = 7.0  # interval 1 (4 < w < 7): 7 at omega 5
    d[8, 1] = 3.0  # interval 2 (7 < w < 10): 3 at omega 9
    d[9, 5] = 6.0  # omega 10 is the last snapshot: in no interval
    d[3, 4] = 9.0  # omega 4 is a snapshot: never selected again
    new, lam, lam_n = R.select_snapshots(om, d, snaps, 2)
    assert list(new) == [5.0, 2.0] and lam == 7.0
    assert list(lam_n) == [5.0, 7.0, 3.0]
    new1, _, _ = R.select_snapshots(om, d, snaps, 3)
    assert list(new1) == [5.0, 2.0, 9.0]


def test_select_never_returns_a_snapshot():
    """A certificate maximum sitting on a snapshot frequency (where the reduced
    model reproduces its own snapshot up to truncation) is passed over: the
    new frequencies are always new."""
    rng = np.random.default_rng(9)
    om = np.sort(rng.uniform(1.0, 1e3, 400))
    snaps = np.sort(rng.choice(om, 7, replace=False))
    d = rng.uniform(0.0, 1.0, (400, 6))
    d[np.isin(om, snaps)] = 10.0
    for n_star in (1, 2, 6):
        new, lam, lam_n = R.select_snapshots(om, d, snaps, n_star)
        assert not np.any(np.isin(new, snaps)) and lam < 10.0
    for theta in (1.0, 0.5, 1e-9):
        new, lam, _ = R.select_snapshots_threshold(om, d, snaps, theta)
        assert not np.any(np.isin(new, snaps)) and lam < 10.0


def test_select_snapshots_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(20):
        om = np.sort(rng.uniform(1, 100, 50))
        snaps = np.sort(rng.choice(om, 6, replace=False))
        d = rng.integers(0, 4, (50, 6)).astype(float)
        new, lam, lam_n = R.select_snapshots(om, d, snaps, 2)
        cands = []
        for n in range(5):
            lo, hi = snaps[n], snaps[n + 1]
            best = None
            for k in range(50):
                inside = lo < om[k] < hi
                if inside and (best is None or d[k].max() > d[best].max()):
                    best = k
            if best is not None:
                cands.append((-d[best].max(), n, om[best]))
        cands.sort()
        assert list(new) == [c[2] for c in cands[:2]]


# ---------------------------------------------------------- sensitivities
def test_forward_sensitivity_matches_central_differences():
    c = _cases.ellipsoid16()
    fo, U, rom = _rom(c, 10)
    om = np.array([50.0, 800.0, 2e4])
    rng = np.random.default_rng(1)
    wR = rng.standard_normal((3, 6)) * 1e6
    wI = rng.standard_normal((3, 6)) * 1e6

    def L(omega, scale=1.0):
        r2 = dict(rom)
        r2["CM"] = scale * rom["CM"]
        r2["g"] = scale * rom["g"]
        r2["E"] = scale * rom["E"]
        a = R.reduced_solve(r2, omega)
        Rt, I = R.tensors_mm(r2, a, omega, rom["N0"], fo.alpha)
        return np.sum(wR * R.pack(Rt) + wI * R.pack(I))

    dw, ds = R.forward_sensitivity(rom, om, fo.alpha, wR, wI)
    for k in range(3):
        h = 1e-6 * om[k]
        e = np.zeros(3); e[k] = h
        fd = (L(om + e) - L(om - e)) / (2 * h)
        assert abs(fd - dw[k]) <= 1e-6 * abs(dw[k]) + 1e-12
    fd_s = (L(om, 1 + 1e-6) - L(om, 1 - 1e-6)) / 2e-6
    assert abs(fd_s - ds) <= 1e-6 * abs(ds)
    assert abs(ds - np.sum(om * dw)) <= 1e-10 * abs(ds)


def test_material_sensitivities_pins():
    """sigma_m dL/dsigma_m per material of a two-material shell (core
    sigma 6e6, mu_r 50; shell sigma 3.5e7): one part holding the whole model
    gives sigma dL/dsigma; the parts sum to sum_k omega_k dL/domega_k (the
    model depends on sigma omega only); central differences in sigma_1."""
    c = _cases.shell16()
    fo, U, rom = _rom(c, 10)
    om = np.array([30.0, 2e3, 1e5])
    rng = np.random.default_rng(7)
    wR = rng.standard_normal((3, 6)) * 1e6
    wI = rng.standard_normal((3, 6)) * 1e6
    sig = c.ops.sigma_e
    parts = []
    for s_m in np.unique(sig[sig > 0]):
        cm = np.where(sig == s_m, fo.c, 0.0)
        pr = R.project(fo.K, cm, fo.eps_h, c.w, U)
        parts.append({"CM": pr["CM"], "g": pr["g"], "E": pr["E"]})
    assert len(parts) == 2
    whole = R.forward_sensitivity_materials(rom, [{"CM": rom["CM"], "g": rom["g"], "E": rom["E"]}],
                                            om, fo.alpha, wR, wI)
    dw, ds = R.forward_sensitivity(rom, om, fo.alpha, wR, wI)
    assert abs(whole[0] - ds) <= 1e-10 * abs(ds)
    per = R.forward_sensitivity_materials(rom, parts, om, fo.alpha, wR, wI)
    ident = np.sum(om * dw)
    assert abs(per.sum() - ident) <= 1e-8 * np.abs(per).max()
    assert np.all(np.abs(per) > 1e-3 * np.abs(per).max())  # both materials matter

    def L(h):
        r2 = dict(rom)
        r2["CM"] = rom["CM"] + h * parts[0]["CM"]
        r2["g"] = rom["g"] + h * parts[0]["g"]
        r2["E"] = rom["E"] + h * parts[0]["E"]
        a = R.reduced_solve(r2, om)
        Rt, I = R.tensors_mm(r2, a, om, rom["N0"], fo.alpha)
        return np.sum(wR * R.pack(Rt) + wI * R.pack(I))

    # step 1e-4: truncation ~1e-8 relative, rounding below that
    fd = (L(1e-4) - L(-1e-4)) / 2e-4
    assert abs(fd - per[0]) <= 1e-6 * abs(per[0])


def test_select_threshold_variant_limits():
    """theta = 1 keeps exactly the interval of the global maximum of Delta
    over all frequencies; theta -> 0 keeps every non-empty interval, in the
    rank order of the fixed-N_* selection with N_* = number of intervals;
    in between, the kept intervals are exactly those whose maximum reaches
    theta * Lambda (checked by brute force over the output frequencies)."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        om = np.sort(rng.uniform(1.0, 100.0, 60))
        d = rng.uniform(0.0, 1.0, (60, 6))
        snaps = np.sort(rng.uniform(0.5, 101.0, 6))
        dm = d.max(1)
        inside = (om >= snaps[0]) & (om <= snaps[-1])
        new1, L, lam_n = R.select_snapshots_threshold(om, d, snaps, 1.0)
        gk = np.flatnonzero(inside)[np.argmax(dm[inside])]
        assert new1.size == 1 and new1[0] == om[gk] and L == dm[gk]
        new0, _, _ = R.select_snapshots_threshold(om, d, snaps, 1e-300)
        nonempty = int(np.sum(np.isfinite(lam_n)))
        ref0, _, _ = R.select_snapshots(om, d, snaps, nonempty)
        assert np.array_equal(new0, ref0)
        theta = 0.8
        newt, _, _ = R.select_snapshots_threshold(om, d, snaps, theta)
        # brute force: for every interval, its maximum and whether it reaches theta * L
        expect = set()
        for n in range(snaps.size - 1):
            last = n == snaps.size - 2
            m = (om >= snaps[n]) & ((om <= snaps[n + 1]) if last else (om < snaps[n + 1]))
            if m.any() and dm[m].max() >= theta * L:
                expect.add(float(om[np.flatnonzero(m)[np.argmax(dm[m])]]))
        assert set(newt.tolist()) == expect
