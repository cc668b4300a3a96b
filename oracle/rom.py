"""Oracle for the reduced-order steps: POD basis, projection, online sweep,
tensor post-processing, certificates, snapshot selection and sensitivities.

Notation follows Sections 3-4: snapshot matrix D (eq. (D)), TSVD basis U^M
(eqs. (SVD), (truncSVD)), reduced system A^M p = r^M (eq. (ReducedA)), tensors
R~ = N0 + R and I (eqs. (NRI), (Rmatrixmeth), (I_tensor_coeffs),
(podprealmpt), (podpimagmpt)), certificate Delta (Lemma 4.1).

Readings of points the paper leaves open (each listed in the design notes):
  * one joint basis U from D = [D_1 D_2 D_3] instead of one per direction;
    the paper's blocks K^M_ij, C^M_ij, C^(2),M_j, t_i^M collapse to K_M, C_M, g;
  * Remark 3.1 (same space for theta~^(0) and theta^(1)): C = C^(1) = C^(2),
    s_i = t_i, and o_i^T C o_j + c_ij + s_i^T o_j + s_j^T o_i = w_i^T C w_j;
  * truncation keeps M = #{s_m / s_1 >= TOL}, capped, and never splits a
    cluster of singular values that agree to 1e-8 relative;
  * the Y^(hp) norm is the energy norm of X = K + eps h I, so the residual dual
    norm is r^H X^{-1} r and alpha_LB = 1.
"""
from __future__ import annotations

import numpy as np

PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))  # stored order 11 12 13 22 23 33


# ---------------------------------------------------------------- POD (a1)
def truncation_rank(s, tol, m_cap, cluster=1e-8) -> int:
    """M from the singular values s (descending), Section 4.1 with the cap."""
    s = np.asarray(s, float)
    M = int(np.count_nonzero(s / s[0] >= tol))
    M = min(M, int(m_cap), s.size)
    while 0 < M < s.size and s[M] / s[M - 1] > 1.0 - cluster:
        M -= 1
    return M


def pod_basis(D, tol, m_cap):
    """Thin SVD of the snapshot matrix and its truncation (eqs. (SVD), (truncSVD))."""
    U, s, _ = np.linalg.svd(np.asarray(D), full_matrices=False)
    M = truncation_rank(s, tol, m_cap)
    return U[:, :M], s, M


# --------------------------------------------------------- projection (a2)
def project(K, c, eps_h, w, U):
    """Galerkin-projected pieces of A^M, r^M and the tensor forms.

    K_M = U^H K U, C_M = U^H C U, G_M = U^H U (for eps h U^H M U),
    g_i = U^H C w_i (the t^M / C^(2),M terms), E_ij = w_i^T C w_j.
    """
    U = np.asarray(U)
    KU = K @ U
    cU = c[:, None] * U
    cw = c[:, None] * w
    return {
        "KM": U.conj().T @ KU,
        "CM": U.conj().T @ cU,
        "UhU": U.conj().T @ U,
        "g": U.conj().T @ cw,
        "E": w.T @ cw,
        "eps_h": float(eps_h),
    }


def static_tensor_mesh(fo, o):
    """N0 by explicit sums over faces (eq. (NRI) first line, discrete):

    N0_ij = alpha^3 delta_ij sum_{f normal to e_i} h^3 (1 - 1/mu_f)
            + alpha^3/4 sum_f (1/(mu_f h)) (C o_i)_f (C o_j)_f
    Each face normal to e_i carries the dual volume h^3.
    """
    a3 = fo.alpha ** 3
    ax = fo.grid.face_normal_axis()
    vol = np.array([fo.h ** 3 * np.sum(1.0 - 1.0 / fo.mu_f[ax == i]) for i in range(3)])
    Co = fo.Cf @ o
    return a3 * np.diag(vol) + 0.25 * a3 * (Co.T @ (fo.face_w[:, None] * Co))


# --------------------------------------------------------------- sweep (a3)
def reduced_solve(rom, omega):
    """a_i(omega) from (K_M + eps h U^H U - i omega C_M) a_i = i omega g_i."""
    omega = np.atleast_1d(np.asarray(omega, float))
    A0 = rom["KM"] + rom["eps_h"] * rom["UhU"]
    A = A0[None] - 1j * omega[:, None, None] * rom["CM"][None]
    r = 1j * omega[:, None, None] * rom["g"][None]
    return np.linalg.solve(A, r)  # (n_omega, M, 3)


# ------------------------------------------------------- tensors (a4)
def tensors_mesh(fo, U, a, omega, w, N0):
    """R~ and I by explicit sums over faces and conductor edges (IM analogue).

    q_i = U a_i (eq. (solution:rebreakdown)),
    R_ij = -alpha^3/4 Re sum_f (1/(mu_f h)) conj((C q_i)_f) (C q_j)_f,
    I_ij = omega alpha^3/4 Re sum_e c_e conj(v_ie) v_je,  v_i = q_i + w_i.
    Returns (n_omega, 3, 3) arrays.
    """
    a3 = fo.alpha ** 3
    omega = np.atleast_1d(np.asarray(omega, float))
    Rt = np.empty((omega.size, 3, 3))
    Im = np.empty((omega.size, 3, 3))
    for k in range(omega.size):
        q = U @ a[k]
        Cq = fo.Cf @ q
        R = -0.25 * a3 * np.real(Cq.conj().T @ (fo.face_w[:, None] * Cq))
        v = q + w
        Im[k] = 0.25 * a3 * omega[k] * np.real(v.conj().T @ (fo.c[:, None] * v))
        Rt[k] = N0 + R
    return Rt, Im


def tensors_fmm(fo, q, omega, w, N0):
    """Full matrix method (eqs. (Rmatrixmeth), (I_tensor_coeffs)) for given q (N, 3)."""
    a3 = fo.alpha ** 3
    R = -0.25 * a3 * np.real(q.conj().T @ (fo.K @ q))
    v = q + w
    I = 0.25 * a3 * omega * np.real(v.conj().T @ (fo.c[:, None] * v))
    return N0 + R, I


def tensors_mm(rom, a, omega, N0, alpha):
    """Matrix method in the reduced space (eqs. (podprealmpt), (podpimagmpt))."""
    a3 = alpha ** 3
    omega = np.atleast_1d(np.asarray(omega, float))
    ah = np.conj(np.swapaxes(a, 1, 2))
    R = -0.25 * a3 * np.real(ah @ rom["KM"] @ a)
    gh = rom["g"].conj().T
    quad = ah @ rom["CM"] @ a + (gh @ a) + (ah @ rom["g"])
    I = 0.25 * a3 * omega[:, None, None] * (rom["E"][None] + np.real(quad))
    return N0[None] + R, I


# ------------------------------------------------------ certificates (a4)
def residual_gram_from(Z, XinvZ):
    """G = Z^H X^{-1} Z (Lemma 4.1) from the residual columns Z and X^{-1} Z;
    Hermitian by definition, so the two computed triangles are averaged."""
    G = np.asarray(Z).conj().T @ np.asarray(XinvZ)
    return 0.5 * (G + G.conj().T)


def residual_gram_direct(fo, U, w):
    """G = Z^H X^{-1} Z with Z = [C w_1, C w_2, C w_3, X U, C U] (SuperLU for X^{-1})."""
    Z = np.concatenate([fo.c[:, None] * w, fo.X @ U, fo.c[:, None] * U], 1).astype(np.complex128)
    return residual_gram_from(Z, fo.X_solve(Z))


def residual_gram_schur(S, cond_idx, c, w, U, KM, UhU, eps_h):
    """The same G using only the conductor block S = P^T X^{-1} P.

    C w_i and C U vanish off the conductor edges, and X^{-1} (X U) = U, so
    every block of Z^H X^{-1} Z is a product of S, U and the projected K.
    """
    M = U.shape[1]
    cc = c[cond_idx]
    Zc = np.concatenate([cc[:, None] * w[cond_idx], cc[:, None] * U[cond_idx]], 1).astype(np.complex128)
    G = np.zeros((2 * M + 3, 2 * M + 3), np.complex128)
    wc = np.r_[0:3, 3 + M:3 + 2 * M]  # positions of the conductor-supported columns
    xs = np.arange(3, 3 + M)
    Gc = Zc.conj().T @ (S @ Zc)
    G[np.ix_(wc, wc)] = 0.5 * (Gc + Gc.conj().T)  # Hermitian by definition
    ZU = Zc.conj().T @ U[cond_idx]
    G[np.ix_(wc, xs)] = ZU
    G[np.ix_(xs, wc)] = ZU.conj().T
    G[np.ix_(xs, xs)] = KM + eps_h * UhU
    return G


def certificate_gform(G, a, omega, alpha, alpha_lb=1.0):
    """Delta_ij (Lemma 4.1) with ||r_i||^2 = w^(i)H G w^(i) and the cross term
    -2 Re w^(i)H G w^(j);  w^(i) = [i w e_i ; -a_i ; i w a_i] so that the
    residual of the reduced solution is Z w^(i).  Returns (n_omega, 3, 3)."""
    omega = np.atleast_1d(np.asarray(omega, float))
    nw, M, _ = a.shape
    W = np.zeros((nw, 2 * M + 3, 3), np.complex128)
    for i in range(3):
        W[:, i, i] = 1j * omega
    W[:, 3:3 + M, :] = -a
    W[:, 3 + M:, :] = 1j * omega[:, None, None] * a
    Cm = np.conj(np.swapaxes(W, 1, 2)) @ G @ W  # (nw, 3, 3): c_ij
    n2 = np.real(np.diagonal(Cm, axis1=1, axis2=2))
    diff = n2[:, :, None] + n2[:, None, :] - 2.0 * np.real(Cm)
    return alpha ** 3 / (8.0 * alpha_lb) * (n2[:, :, None] + n2[:, None, :] + diff)


def certificate_direct(fo, U, a, omega, w, alpha_lb=1.0):
    """Delta_ij from full-order residuals res_i = r_i - A(omega) U a_i and X^{-1}."""
    omega = np.atleast_1d(np.asarray(omega, float))
    out = np.empty((omega.size, 3, 3))
    a3 = fo.alpha ** 3
    for k in range(omega.size):
        res = fo.rhs(omega[k], w) - fo.A(omega[k]) @ (U @ a[k])
        Xr = fo.X_solve(res)
        n2 = np.real(np.einsum("ni,ni->i", res.conj(), Xr))
        for i in range(3):
            for j in range(3):
                d = res[:, i] - res[:, j]
                dn = np.real(np.vdot(d, fo.X_solve(d)))
                out[k, i, j] = a3 / (8.0 * alpha_lb) * (n2[i] + n2[j] + dn)
    return out


def pack(T):
    """(n, 3, 3) symmetric -> (n, 6) in the order 11 12 13 22 23 33."""
    return np.stack([T[:, i, j] for i, j in PAIRS], 1)


def sweep(rom, omega, G, alpha, alpha_lb=1.0):
    """Reduced solves plus matrix-method tensors and certificates: (n_omega, 18)."""
    a = reduced_solve(rom, omega)
    Rt, I = tensors_mm(rom, a, omega, rom["N0"], alpha)
    Dl = certificate_gform(G, a, omega, alpha, alpha_lb)
    return np.concatenate([pack(Rt), pack(I), pack(Dl)], 1), a


# ------------------------------------------------------ selection (a5)
def select_snapshots(omega, delta, snap_omega, n_star):
    """Algorithm 1 selection step.

    Intervals [w_n, w_{n+1}) between consecutive sorted snapshot frequencies
    (the last one closed); Lambda_n = max over omega in the interval and over
    (i, j) of Delta_ij; Lambda = max_n Lambda_n; the N_* intervals with the
    largest Lambda_n (ties: lower n) each contribute one new snapshot at the
    omega attaining Lambda_n (ties: smaller omega).
    Returns (new omegas in rank order, Lambda, Lambda_n per interval).
    """
    omega = np.asarray(omega, float)
    dmax = np.max(np.asarray(delta, float).reshape(omega.size, -1), axis=1)
    sn = np.sort(np.asarray(snap_omega, float))
    nint = sn.size - 1
    lam = np.full(nint, -np.inf)
    arg = np.full(nint, -1)
    for n in range(nint):
        lo, hi = sn[n], sn[n + 1]
        inside = (omega >= lo) & ((omega < hi) if n < nint - 1 else (omega <= hi))
        idx = np.flatnonzero(inside)
        if idx.size == 0:
            continue
        best = idx[0]
        for t in idx[1:]:
            if dmax[t] > dmax[best] or (dmax[t] == dmax[best] and omega[t] < omega[best]):
                best = t
        lam[n] = dmax[best]
        arg[n] = best
    order = sorted(range(nint), key=lambda n: (-lam[n], n))
    chosen = [n for n in order if np.isfinite(lam[n])][:n_star]
    return omega[arg[chosen]], float(np.max(lam)), lam


def select_snapshots_threshold(omega, delta, snap_omega, theta):
    """Threshold variant of the selection step (§4.3, after Hesthaven et al.):
    instead of a fixed N_*, every interval whose maximum certificate reaches
    theta * Lambda (0 < theta <= 1) contributes one new snapshot at the omega
    attaining its maximum, at most one per interval as in Algorithm 1.  The
    intervals, ties and rank order are those of select_snapshots.
    Returns (new omegas in rank order, Lambda, Lambda_n per interval)."""
    omega = np.asarray(omega, float)
    _, lam_max, lam = select_snapshots(omega, delta, snap_omega, 0)
    keep = [n for n in range(lam.size) if np.isfinite(lam[n]) and lam[n] >= theta * lam_max]
    new, _, _ = select_snapshots(omega, delta, snap_omega, len(keep))
    return new, lam_max, lam


# ---------------------------------------------------- sensitivities (a7)
def forward_sensitivity(rom, omega, alpha, wR, wI):
    """dL/domega_k and dL/dsigma for L = sum_k sum_pairs wR R~ + wI I (weights per
    omega and stored pair, shape (n_omega, 6)), by forward differentiation:
    A da/dw = i g + i C_M a  (omega);  A da/ds = (i w/s)(g + C_M a)  (sigma,
    with C_M, g, E proportional to sigma and the basis frozen).
    Returns (dL/domega (n_omega,), sigma * dL/dsigma)."""
    omega = np.atleast_1d(np.asarray(omega, float))
    a3 = alpha ** 3
    A0 = rom["KM"] + rom["eps_h"] * rom["UhU"]
    KM, CM, g, E = rom["KM"], rom["CM"], rom["g"], rom["E"]
    dw = np.empty(omega.size)
    ds = 0.0
    for k, om in enumerate(omega):
        A = A0 - 1j * om * CM
        a = np.linalg.solve(A, 1j * om * g)
        rhs = 1j * (g + CM @ a)
        da = np.linalg.solve(A, rhs)  # d a / d omega
        das = om * da  # sigma * d a / d sigma
        I = 0.25 * a3 * om * (E + np.real(a.conj().T @ CM @ a + g.conj().T @ a + a.conj().T @ g))
        dR = -0.25 * a3 * np.real(da.conj().T @ KM @ a + a.conj().T @ KM @ da)
        dI = I / om + 0.25 * a3 * om * np.real(da.conj().T @ CM @ a + a.conj().T @ CM @ da
                                                + g.conj().T @ da + da.conj().T @ g)
        dRs = -0.25 * a3 * np.real(das.conj().T @ KM @ a + a.conj().T @ KM @ das)
        # sigma d/dsigma of I: explicit part I (C_M, g, E all scale with sigma)
        dIs = I + 0.25 * a3 * om * np.real(das.conj().T @ CM @ a + a.conj().T @ CM @ das
                                           + g.conj().T @ das + das.conj().T @ g)
        dw[k] = sum(wR[k, p] * dR[i, j] + wI[k, p] * dI[i, j] for p, (i, j) in enumerate(PAIRS))
        ds += sum(wR[k, p] * dRs[i, j] + wI[k, p] * dIs[i, j] for p, (i, j) in enumerate(PAIRS))
    return dw, ds


def forward_sensitivity_materials(rom, parts, omega, alpha, wR, wI):
    """sigma_m dL/dsigma_m for an object of several conducting materials (L as
    in forward_sensitivity).  C_sigma is the sum of one term per material,
    each proportional to that material's sigma, so C_M, g and E split into
    parts (C_M,m, g_m, E_m), each the projection of one material's edges
    alone; K_M and the basis do not depend on sigma.  Forward
    differentiation: A (sigma_m da/dsigma_m) = i w (g_m + C_M,m a), and I
    depends on sigma_m explicitly through C_M,m, g_m and E_m.
    parts: list of dicts with keys CM, g, E.  Returns one value per part."""
    omega = np.atleast_1d(np.asarray(omega, float))
    a3 = alpha ** 3
    A0 = rom["KM"] + rom["eps_h"] * rom["UhU"]
    KM, CM, g = rom["KM"], rom["CM"], rom["g"]
    out = np.zeros(len(parts))
    for k, om in enumerate(omega):
        A = A0 - 1j * om * CM
        a = np.linalg.solve(A, 1j * om * g)
        for m, pm in enumerate(parts):
            Cm, gm, Em = pm["CM"], pm["g"], pm["E"]
            dam = np.linalg.solve(A, 1j * om * (gm + Cm @ a))
            dR = -0.25 * a3 * np.real(dam.conj().T @ KM @ a + a.conj().T @ KM @ dam)
            dI = 0.25 * a3 * om * (Em + np.real(a.conj().T @ Cm @ a + gm.conj().T @ a
                                                + a.conj().T @ gm)
                                   + np.real(dam.conj().T @ CM @ a + a.conj().T @ CM @ dam
                                             + g.conj().T @ dam + dam.conj().T @ g))
            out[m] += sum(wR[k, p] * dR[i, j] + wI[k, p] * dI[i, j]
                          for p, (i, j) in enumerate(PAIRS))
    return out
