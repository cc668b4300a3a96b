"""Pins of the per-direction oracle (one basis U_i per direction, Section 4.1,
with the cross-projected blocks of eqs. (podprealmpt), (podpimagmpt)) against
what the mathematics fixes: an untruncated basis reproduces the full-order
solution at its own snapshot frequencies; the matrix method equals explicit
sums over the grid; with the same basis in every direction everything is the
joint form; the certificate from Grams equals the one from full-order
residuals, and it bounds the tensor error (Lemma 4.1).  No GPU needed."""
import numpy as np
import pytest

from oracle import perdir as P
from oracle import rom as R
from tests import _cases

S_REF16 = np.r_[0.0, 10.0 ** np.arange(1.0, 6.01, 0.5)]


def _setup(c, tol, cap):
    fo = c.oracle_fo()
    K = c.snap.size
    Us = [b[0] for b in P.pod_bases(c.D, K, tol, cap)]
    pr = P.project(fo.K, fo.c, fo.eps_h, c.w, Us)
    pr["N0"] = R.static_tensor_mesh(fo, c.o)
    return fo, Us, pr


def _normwise(A, B):
    """max over frequencies of max_ij |A - B| / max_ij |B|."""
    return float(np.max(np.abs(A - B).max((1, 2)) / np.abs(B).max((1, 2))))


def test_untruncated_per_direction_reproduces_full_order_at_snapshots():
    c = _cases.ellipsoid16()
    fo, Us, pr = _setup(c, 0.0, 64)
    K = c.snap.size
    ks = [0, 5, 11, 15]
    om = c.snap[ks]
    a = P.reduced_solve(pr, om)
    for i in range(3):
        for t, k in enumerate(ks):
            q = c.D[:, i * K + k]
            err = np.linalg.norm(Us[i] @ a[i][t] - q) / np.linalg.norm(q)
            assert err <= 1e-9, (i, k, err)
    Rm, Im = P.tensors_mm(pr, a, om, pr["N0"], fo.alpha)
    for t, k in enumerate(ks):
        q = np.stack([c.D[:, i * K + k] for i in range(3)], 1)
        Rf, If = R.tensors_fmm(fo, q, om[t], c.w, pr["N0"])
        assert np.abs(Rm[t] - Rf).max() <= 1e-9 * np.abs(Rf).max()
        assert np.abs(Im[t] - If).max() <= 1e-9 * np.abs(If).max()


def test_per_direction_mm_equals_mesh_sums():
    c = _cases.shell16()
    fo, Us, pr = _setup(c, 1e-8, 5)
    om = np.logspace(1, 6, 9)
    a = P.reduced_solve(pr, om)
    Rm, Im = P.tensors_mm(pr, a, om, pr["N0"], fo.alpha)
    Rs, Is = P.tensors_mesh(fo, Us, a, om, c.w, pr["N0"])
    assert _normwise(Rm, Rs) <= 1e-11
    # I is a difference of terms of size omega a^3/4 |E| where the field is
    # expelled: rounding is relative to that scale
    for k in range(om.size):
        scale_I = max(np.abs(Is[k]).max(), 0.25 * fo.alpha ** 3 * om[k] * np.abs(pr["E"]).max())
        assert np.abs(Im[k] - Is[k]).max() <= 1e-12 * scale_I


def test_same_basis_in_every_direction_is_the_joint_form():
    c = _cases.ellipsoid16()
    fo = c.oracle_fo()
    U = np.linalg.svd(c.D, full_matrices=False)[0][:, :6]
    pr = P.project(fo.K, fo.c, fo.eps_h, c.w, [U, U, U])
    pr["N0"] = R.static_tensor_mesh(fo, c.o)
    rom = R.project(fo.K, fo.c, fo.eps_h, c.w, U)
    rom["N0"] = pr["N0"]
    om = np.array([30.0, 3e3, 3e5])
    gram = lambda s: R.residual_gram_direct(fo, U, c.w, s)
    out_j, _ = R.sweep(rom, om, R.certificate_data(rom, S_REF16, gram), fo.alpha)
    Ut = np.concatenate([U, U, U], 1)
    gram3 = lambda s: R.residual_gram_direct(fo, Ut, c.w, s)
    out_p, _ = P.sweep(pr, om, P.certificate_data(pr, S_REF16, gram3), fo.alpha)
    for part in range(3):  # R~, I, Delta: normwise per frequency
        sl = slice(6 * part, 6 * part + 6)
        d = np.abs(out_p[:, sl] - out_j[:, sl]).max(1) / np.abs(out_j[:, sl]).max(1)
        assert np.all(d <= 1e-9), (part, d)


def test_per_direction_certificate_gform_equals_direct():
    c = _cases.shell16()
    fo, Us, pr = _setup(c, 1e-8, 3)
    om = np.array([3e1, 1e3, 3e4, 7e5])
    a = P.reduced_solve(pr, om)
    Ut = np.concatenate(Us, 1)
    cert = P.certificate_data(pr, S_REF16, lambda s: R.residual_gram_direct(fo, Ut, c.w, s))
    Dg = P.certificate_gform(cert, a, om, fo.alpha)
    Dd = P.certificate_direct(fo, Us, a, om, c.w, S_REF16)
    assert np.all(Dd > 0)
    assert np.all(np.abs(Dg - Dd) <= 1e-7 * Dd)


@pytest.mark.parametrize("cap", [2, 5])
def test_lemma41_bounds_the_per_direction_error(cap):
    """|R~ - R~^PODP|_ij <= Delta_ij and |I - I^PODP|_ij <= Delta_ij with one
    basis per direction, against refined sparse-direct full-order solutions."""
    import scipy.sparse.linalg as spla
    c = _cases.shell16()
    fo, Us, pr = _setup(c, 1e-8, cap)
    om = np.array([30.0, 3e2, 3e3, 3e4, 3e5])
    a = P.reduced_solve(pr, om)
    Rt, It = P.tensors_mm(pr, a, om, pr["N0"], fo.alpha)
    Dd = P.certificate_direct(fo, Us, a, om, c.w, S_REF16)
    for k, w in enumerate(om):
        A = fo.A(w)
        r = fo.rhs(w, c.w)
        lu = spla.splu(A)
        q = lu.solve(r)
        for _ in range(2):
            q = q + lu.solve(r - A @ q)
        Rf, If = R.tensors_fmm(fo, q, w, c.w, pr["N0"])
        tight = np.inf
        for T, Tp in ((Rf, Rt[k]), (If, It[k])):
            err = np.abs(T - Tp)
            assert np.all(err <= Dd[k]), (w, err / Dd[k])
            live = err > 1e-6 * np.abs(T).max()
            if live.any():
                tight = min(tight, (Dd[k][live] / err[live]).min())
        print(f"cap {cap} omega {w:g}: tightest effectivity {tight:.3g}")
        assert tight <= 1e3, (w, tight)
