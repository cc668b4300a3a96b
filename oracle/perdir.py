"""Oracle for the per-direction form of the method: one truncated SVD per
snapshot matrix D_i (Section 4.1, eqs. (D), (SVD), (truncSVD) for i = 1, 2, 3),
the reduced system of each direction in its own basis (eq. (ReducedA) with
U_i^M), the tensors from the cross-projected blocks K^M_ij = U_i^H K U_j,
C^M_ij = U_i^H C U_j and t = U_i^H C w_j (eqs. (podprealmpt), (podpimagmpt)),
and the certificate of Lemma 4.1 for these reduced solutions.

Test infrastructure: plain numpy, only the tests, the entry's smoke check and
the benchmark's CPU baseline use it.

Certificate.  The residual of direction i is r_i - A U_i a_i = Z w^(i) with
Z = [C w_1..3 | X U_1 | X U_2 | X U_3 | C U_1 | C U_2 | C U_3] and w^(i)
holding i omega e_i, -a_i and i omega a_i in the slots of U_i (zeros in the
others), so the residual Grams are those of the joint form over the
concatenated basis [U_1 U_2 U_3].  The term linear in the residual norms
changes: Galerkin orthogonality of the error e_i holds against span(U_i)
only, so in the bound's term (U_j a_j)^T A e_i the part of conj(U_j a_j)
inside span(U_i) drops, leaving d_{j->i}, the distance (in the norm of
X + s C) from conj(U_j a_j) to span(U_i):
    Delta_ij = a^3/(8 alpha_LB) (n_i^2 + n_j^2 + ||r_i - r_j||^2)
               + a^3/4 (n_i e_{j->i} + n_j e_{i->j}),
    e_{j->i}^2 = d_{j->i}^2 / 2 + 4 eps h |U_j a_j|^2 = a_j^H D'_{i<-j} a_j,
    D'_{i<-j} = (A_s,jj - conj(T_ij^H A_s,ii^{-1} T_ij)) / 2 + 4 eps h U_j^H U_j,
with A_s,ii = U_i^H (X + s C) U_i and T_ij = U_i^H (X + s C) conj(U_j).  With
U_1 = U_2 = U_3 every piece is the joint form's.
"""
from __future__ import annotations

import numpy as np

from .rom import ALPHA_LB, pack, pod_basis, ref_index


def pod_bases(D, K, tol, m_cap):
    """U_i (truncated SVD of D_i = columns i K .. (i+1) K - 1 of D), i = 1..3."""
    out = []
    for i in range(3):
        U, s, M = pod_basis(D[:, i * K:(i + 1) * K], tol, m_cap)
        out.append((U, s, M))
    return out


def project(K, c, eps_h, w, Us):
    """Cross-projected blocks: KM[i][j] = U_i^H K U_j, CM, UU (U_i^H U_j),
    t[i][j] = U_i^H C w_j, E = w^T C w, and the pieces of the conjugation
    defects TX[i][j] = U_i^H X conj(U_j), TC[i][j] = U_i^H C conj(U_j)."""
    P = {"eps_h": float(eps_h), "M": [U.shape[1] for U in Us], "E": w.T @ (c[:, None] * w)}
    for key in ("KM", "CM", "UU", "t", "TX", "TC"):
        P[key] = [[None] * 3 for _ in range(3)]
    for i in range(3):
        Ui = Us[i]
        for j in range(3):
            Uj = Us[j]
            P["KM"][i][j] = Ui.conj().T @ (K @ Uj)
            P["CM"][i][j] = Ui.conj().T @ (c[:, None] * Uj)
            P["UU"][i][j] = Ui.conj().T @ Uj
            P["t"][i][j] = Ui.conj().T @ (c * w[:, j])
            P["TX"][i][j] = Ui.conj().T @ (K @ Uj.conj()) + float(eps_h) * (Ui.conj().T @ Uj.conj())
            P["TC"][i][j] = Ui.conj().T @ (c[:, None] * Uj.conj())
    return P


def reduced_solve(P, omega):
    """a_i(omega) of (K^M_ii + eps h U_i^H U_i - i omega C^M_ii) a_i = i omega t_ii,
    each direction in its own basis.  Returns a list of (n_omega, M_i)."""
    omega = np.atleast_1d(np.asarray(omega, float))
    out = []
    for i in range(3):
        A0 = P["KM"][i][i] + P["eps_h"] * P["UU"][i][i]
        A = A0[None] - 1j * omega[:, None, None] * P["CM"][i][i][None]
        r = 1j * omega[:, None] * P["t"][i][i][None]
        out.append(np.linalg.solve(A, r[..., None])[..., 0])
    return out


def tensors_mm(P, a, omega, N0, alpha):
    """R~_ij = N0_ij - a^3/4 Re a_i^H K^M_ij a_j,
    I_ij = omega a^3/4 (E_ij + Re(a_i^H C^M_ij a_j + a_i^H t_ij + t_ji^H a_j))."""
    a3 = alpha ** 3
    omega = np.atleast_1d(np.asarray(omega, float))
    nw = omega.size
    R = np.empty((nw, 3, 3))
    I = np.empty((nw, 3, 3))
    for i in range(3):
        for j in range(3):
            kq = np.einsum("ka,ab,kb->k", a[i].conj(), P["KM"][i][j], a[j])
            cq = np.einsum("ka,ab,kb->k", a[i].conj(), P["CM"][i][j], a[j])
            src = a[i].conj() @ P["t"][i][j] + a[j] @ P["t"][j][i].conj()
            R[:, i, j] = N0[i, j] - 0.25 * a3 * np.real(kq)
            I[:, i, j] = 0.25 * a3 * omega * (P["E"][i, j] + np.real(cq + src))
    return R, I


def tensors_mesh(fo, Us, a, omega, w, N0):
    """The same tensors by explicit sums over faces and conductor edges on the
    reconstructed fields q_i = U_i a_i."""
    a3 = fo.alpha ** 3
    omega = np.atleast_1d(np.asarray(omega, float))
    Rt = np.empty((omega.size, 3, 3))
    Im = np.empty((omega.size, 3, 3))
    for k in range(omega.size):
        q = np.stack([Us[i] @ a[i][k] for i in range(3)], 1)
        Cq = fo.Cf @ q
        Rt[k] = N0 - 0.25 * a3 * np.real(Cq.conj().T @ (fo.face_w[:, None] * Cq))
        v = q + w
        Im[k] = 0.25 * a3 * omega[k] * np.real(v.conj().T @ (fo.c[:, None] * v))
    return Rt, Im


def concat(a):
    """The per-direction solutions in the slots of the concatenated basis
    [U_1 U_2 U_3]: (n_omega, sum M_i, 3), block i of column i holding a_i."""
    Ms = [x.shape[1] for x in a]
    off = np.r_[0, np.cumsum(Ms)]
    out = np.zeros((a[0].shape[0], off[-1], 3), np.complex128)
    for i in range(3):
        out[:, off[i]:off[i + 1], i] = a[i]
    return out


def defect_forms(P, s):
    """D'_{i<-j} for all ordered pairs (a 3 x 3 list of M_j x M_j matrices)."""
    eh = P["eps_h"]
    out = [[None] * 3 for _ in range(3)]
    for i in range(3):
        Aii = P["KM"][i][i] + eh * P["UU"][i][i] + s * P["CM"][i][i]
        for j in range(3):
            Ajj = P["KM"][j][j] + eh * P["UU"][j][j] + s * P["CM"][j][j]
            T = P["TX"][i][j] + s * P["TC"][i][j]
            D = Ajj - (T.conj().T @ np.linalg.solve(Aii, T)).conj()
            Dp = 0.5 * D + 4.0 * eh * P["UU"][j][j]
            out[i][j] = 0.5 * (Dp + Dp.conj().T)
    return out


def _delta(n2, cross, e, alpha, alpha_lb):
    """Delta_ij from n_i^2, Re <r_i, r_j> and e[i][j] = e_{j->i}."""
    a3 = alpha ** 3
    n = np.sqrt(np.maximum(n2, 0.0))
    diff = n2[:, None] + n2[None, :] - 2.0 * cross
    quad = a3 / (8.0 * alpha_lb) * (n2[:, None] + n2[None, :] + diff)
    lin = 0.25 * a3 * (n[:, None] * e + n[None, :] * e.T)
    return quad + lin


def certificate_data(P, s_ref, gram):
    """Per-shift inputs: gram(s) -> G_s over the concatenated basis, and the
    defect forms."""
    return {"s_ref": np.asarray(s_ref, float), "G": [gram(s) for s in s_ref],
            "Dp": [defect_forms(P, s) for s in s_ref]}


def certificate_gform(cert, a, omega, alpha, alpha_lb=ALPHA_LB):
    """Delta (n_omega, 3, 3) from the concatenated residual Grams and the
    defect forms."""
    omega = np.atleast_1d(np.asarray(omega, float))
    ac = concat(a)
    nw, M, _ = ac.shape
    W = np.zeros((nw, 2 * M + 3, 3), np.complex128)
    for i in range(3):
        W[:, i, i] = 1j * omega
    W[:, 3:3 + M, :] = -ac
    W[:, 3 + M:, :] = 1j * omega[:, None, None] * ac
    ks = ref_index(cert["s_ref"], omega)
    out = np.empty((nw, 3, 3))
    for k in range(nw):
        Cm = W[k].conj().T @ cert["G"][ks[k]] @ W[k]
        Dp = cert["Dp"][ks[k]]
        e = np.empty((3, 3))
        for i in range(3):
            for j in range(3):
                e[i, j] = np.sqrt(max(np.real(a[j][k].conj() @ Dp[i][j] @ a[j][k]), 0.0))
        out[k] = _delta(np.real(np.diag(Cm)), np.real(Cm), e, alpha, alpha_lb)
    return out


def certificate_direct(fo, Us, a, omega, w, s_ref, alpha_lb=ALPHA_LB):
    """The same Delta from full-order residuals res_i = r_i - A U_i a_i, dual
    norms by SuperLU, and the distances d_{j->i} from conj(U_j a_j) to
    span(U_i) computed on the full-order vectors."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    omega = np.atleast_1d(np.asarray(omega, float))
    ks = ref_index(s_ref, omega)
    out = np.empty((omega.size, 3, 3))
    lus = {}
    for k in range(omega.size):
        s = float(np.asarray(s_ref)[ks[k]])
        Xs = (fo.X + s * sp.diags(fo.c)).tocsc()
        if s not in lus:
            lus[s] = spla.splu(Xs)
        lu = lus[s]
        solve = lambda B: lu.solve(np.ascontiguousarray(B.real)) + 1j * lu.solve(np.ascontiguousarray(B.imag))
        q = np.stack([Us[i] @ a[i][k] for i in range(3)], 1)
        res = fo.rhs(omega[k], w) - fo.A(omega[k]) @ q
        G = res.conj().T @ solve(res)
        e = np.empty((3, 3))
        for i in range(3):
            Ui = Us[i]
            for j in range(3):
                cb = q[:, j].conj()
                coef = np.linalg.solve(Ui.conj().T @ (Xs @ Ui), Ui.conj().T @ (Xs @ cb))
                dv = cb - Ui @ coef
                d2 = np.real(dv.conj() @ (Xs @ dv))
                e[i, j] = np.sqrt(0.5 * d2 + 4.0 * fo.eps_h * np.real(q[:, j].conj() @ q[:, j]))
        out[k] = _delta(np.real(np.diag(G)), np.real(G), e, fo.alpha, alpha_lb)
    return out


def sweep(P, omega, cert, alpha, alpha_lb=ALPHA_LB):
    """Per-direction solves, tensors and certificates: (n_omega, 18), a."""
    a = reduced_solve(P, omega)
    Rt, I = tensors_mm(P, a, omega, P["N0"], alpha)
    Dl = certificate_gform(cert, a, omega, alpha, alpha_lb)
    return np.concatenate([pack(Rt), pack(I), pack(Dl)], 1), a
