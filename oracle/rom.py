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
  * Lemma 4.1's norm and stability constant: at frequency omega the residual
    dual norm is taken in the energy norm of X + s C_sigma (X = K + eps h I),
    s = s(omega) the largest of a list of reference shifts s_0 = 0 < s_1 < ...
    that does not exceed omega (one residual Gram per shift, each independent
    of omega).  For s <= omega the Galerkin error e obeys
    ||e||^2_(X + omega C) <= 2 ||r||^2_(X + s C)^*, and the tensor errors are
    bounded by the Lemma's quadratic form with alpha_LB = 2 / (3 + sqrt 10)
    plus a term linear in the residual norms that vanishes when span(U) is
    closed under complex conjugation (see certificate_gform).
"""
from __future__ import annotations

import numpy as np

PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))  # stored order 11 12 13 22 23 33

# Stability constant of Lemma 4.1 in the reference norms: 1 / (3/2 + sqrt(5/2))
# (derivation in certificate_gform).
ALPHA_LB = 2.0 / (3.0 + np.sqrt(10.0))


# ---------------------------------------------------------------- POD (a1)
RANK_FLOOR = 1e-12  # relative singular values below this are rounding noise


def truncation_rank(s, tol, m_cap, cluster=1e-8) -> int:
    """M from the singular values s (descending), Section 4.1 with the cap.
    A tolerance below RANK_FLOOR counts as RANK_FLOOR: singular values under
    1e-12 s_1 carry no content of D in FP64 (a backward-stable SVD moves every
    one by ~1e-16 s_1), so even a fixed-rank request (tol = 0) stops at the
    numerical rank."""
    s = np.asarray(s, float)
    M = int(np.count_nonzero(s / s[0] >= max(tol, RANK_FLOOR)))
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
    Ub = U.conj()
    return {
        "KM": U.conj().T @ KU,
        "CM": U.conj().T @ cU,
        "UhU": U.conj().T @ U,
        "g": U.conj().T @ cw,
        "E": w.T @ cw,
        "eps_h": float(eps_h),
        # U^H X conj(U) and U^H C conj(U): how far span(U) is from being
        # closed under conjugation (enters the certificate's linear term)
        "TX": U.conj().T @ (K @ Ub) + float(eps_h) * (U.conj().T @ Ub),
        "TC": U.conj().T @ (c[:, None] * Ub),
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
def a0_of(rom):
    """A^M at w = 0: K_M + eps h U^H U (or the matrix supplied as rom["A0"])."""
    return rom["A0"] if "A0" in rom else rom["KM"] + rom["eps_h"] * rom["UhU"]


def reduced_solve(rom, omega):
    """a_i(omega) from (K_M + eps h U^H U - i omega C_M) a_i = i omega g_i."""
    omega = np.atleast_1d(np.asarray(omega, float))
    A0 = a0_of(rom)
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


def ref_index(s_ref, omega):
    """Index of the reference shift used at each omega: the largest s_k <= omega
    (s_ref ascending, s_ref[0] = 0)."""
    s_ref = np.asarray(s_ref, float)
    return np.searchsorted(s_ref, np.atleast_1d(np.asarray(omega, float)), side="right") - 1


def residual_columns(fo, U, w):
    """Z = [C w_1, C w_2, C w_3, X U, C U]: the reduced solution's residual is
    r_i - A(omega) U a_i = Z w^(i) with w^(i) = [i omega e_i; -a_i; i omega a_i]."""
    return np.concatenate([fo.c[:, None] * w, fo.X @ U, fo.c[:, None] * U], 1).astype(np.complex128)


def residual_gram_direct(fo, U, w, s=0.0):
    """G_s = Z^H (X + s C)^{-1} Z (Lemma 4.1's Gram in the reference norm of
    shift s) with a SuperLU factorisation of X + s C."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    Z = residual_columns(fo, U, w)
    if s == 0.0:
        return residual_gram_from(Z, fo.X_solve(Z))
    lu = spla.splu((fo.X + s * sp.diags(fo.c)).tocsc())
    Y = lu.solve(np.ascontiguousarray(Z.real)) + 1j * lu.solve(np.ascontiguousarray(Z.imag))
    return residual_gram_from(Z, Y)


def residual_gram_spectral(lam, V, dc, cond_idx, w, U, A0, s):
    """The same G_s from the conductor block alone.

    C_sigma = P Dc P^T is supported on the n_c conductor edges (P selects
    them, Dc = diag(c)).  With S = P^T X^{-1} P and the eigenpairs
    Dc^(1/2) S Dc^(1/2) = V diag(lam) V^T, the Sherman-Morrison-Woodbury
    identity gives Dc^(1/2) P^T (X + s C)^{-1} P Dc^(1/2) = V diag(phi) V^T,
    phi = lam / (1 + s lam).  With B = V^T Dc^(1/2) [w_c, U_c] (rows of w and
    U at the conductor edges) and chi = 1 / (1 + s lam), every block of G_s is
    a weighted Gram of B:
      [C w, C w]: B_w^H phi B_w     [C w, X U]: B_w^H chi B_U
      [C w, C U]: B_w^H phi B_U     [X U, X U]: A0 - B_U^H (s chi) B_U
      [X U, C U]: B_U^H chi B_U     [C U, C U]: B_U^H phi B_U
    ((X + s C)^{-1} X = I - s (X + s C)^{-1} C on the X U columns).
    lam, V: eigenpairs above; dc: sqrt(c) on the conductor edges."""
    M = U.shape[1]
    lam = np.asarray(lam, float)
    B = V.T @ (dc[:, None] * np.concatenate([w[cond_idx], U[cond_idx]], 1).astype(np.complex128))
    Bw, BU = B[:, :3], B[:, 3:]
    phi = lam / (1.0 + s * lam)
    chi = 1.0 / (1.0 + s * lam)
    gram = lambda X, f, Y: X.conj().T @ (f[:, None] * Y)
    G = np.zeros((2 * M + 3, 2 * M + 3), np.complex128)
    iw, ix, ic = slice(0, 3), slice(3, 3 + M), slice(3 + M, 3 + 2 * M)
    G[iw, iw] = gram(Bw, phi, Bw)
    G[iw, ix] = gram(Bw, chi, BU)
    G[iw, ic] = gram(Bw, phi, BU)
    G[ix, ix] = A0 - gram(BU, s * chi, BU)
    G[ix, ic] = gram(BU, chi, BU)
    G[ic, ic] = gram(BU, phi, BU)
    G[ix, iw] = G[iw, ix].conj().T
    G[ic, iw] = G[iw, ic].conj().T
    G[ic, ix] = G[ix, ic].conj().T
    return 0.5 * (G + G.conj().T)  # Hermitian by definition


def conj_defect_matrix(rom, s):
    """D'_s = D_s / 2 + 4 eps h U^H U with D_s the Hermitian form of the
    conjugation defect: for q = U a,
        a^H D_s a = min over v in span(U) of ||conj(q) - v||^2_(X + s C),
    i.e. ||conj q||^2 - ||Pi conj q||^2 with Pi the (X + s C)-orthogonal
    projector onto span(U):  D_s = A_s - conj(T_s^H A_s^{-1} T_s),
    A_s = U^H (X + s C) U, T_s = U^H (X + s C) conj(U).  a^H D'_s a bounds
    (d/2 + sqrt(2 eps h) |q|)^2 / 2 from above (see certificate_gform)."""
    A0 = a0_of(rom)
    As = A0 + s * rom["CM"]
    Ts = rom["TX"] + s * rom["TC"]
    Q = Ts.conj().T @ np.linalg.solve(As, Ts)
    D = As - Q.conj()
    Dp = 0.5 * D + 4.0 * rom["eps_h"] * rom["UhU"]
    return 0.5 * (Dp + Dp.conj().T)


def _delta(n2, cross, e, alpha, alpha_lb):
    """Delta_ij from n_i^2 = ||r_i||^2, cross_ij = Re <r_i, r_j> and e_i (the
    conjugation-defect weights); arrays (..., 3) and (..., 3, 3)."""
    a3 = alpha ** 3
    n = np.sqrt(np.maximum(n2, 0.0))
    diff = n2[..., :, None] + n2[..., None, :] - 2.0 * cross
    quad = a3 / (8.0 * alpha_lb) * (n2[..., :, None] + n2[..., None, :] + diff)
    lin = 0.25 * a3 * (n[..., :, None] * e[..., None, :] + n[..., None, :] * e[..., :, None])
    return quad + lin


def certificate_gform(Gs, Dps, s_ref, a, omega, alpha, alpha_lb=ALPHA_LB):
    """Delta_ij (Lemma 4.1) from the residual Grams, one per reference shift.

    At omega the shift s = s_k <= omega of ref_index is used:
      n_i^2 = w^(i)H G_s w^(i),  ||r_i - r_j||^2 = n_i^2 + n_j^2 - 2 Re w^(i)H G_s w^(j),
      w^(i) = [i omega e_i ; -a_i ; i omega a_i]  (residual Z w^(i)),
      e_i = (a_i^H D'_s a_i)^(1/2)  (conj_defect_matrix),
      Delta_ij = a^3/(8 alpha_LB) (n_i^2 + n_j^2 + ||r_i - r_j||^2)
                 + a^3/4 (n_i e_j + n_j e_i).
    Why this bounds |R~ - R~^PODP|_ij and |I - I^PODP|_ij.  Let e_i = q_i - U a_i
    (full-order minus reduced), r_i its residual A e_i, l_j(v) = w_j^T C v.
    The energy identities q_i^H A q_j = q_i^H r_j and q_j^H A q_i = q_j^H r_i
    hold for the full-order solution and, by Galerkin orthogonality, for the
    reduced one; they turn the Hermitian forms into
      Re q_i^H X q_j = omega/2 Im(l_j(q_i) + l_i(q_j)),
      I_ij = omega a^3/4 (E_ij + Re(l_j(q_i) + l_i(q_j)) / 2),
    and R_ij = -a^3/4 (Re q_i^H X q_j - eps h Re q_i^H q_j).  Since A is
    complex symmetric and A q_j = i omega C w_j,
      i omega l_j(e_i) = q_j^T A e_i = (U a_j)^T A e_i + e_j^T A e_i.
    The second term is bounded by ||e_i|| ||e_j|| in the norm of X + omega C,
    and ||e||^2 <= 2 n^2 there for s <= omega (|e^H r| <= ||e||_s n and
    e^H r = ||e||^2_X - i omega ||e||^2_C).  Maximising over what these
    constraints allow gives |quadratic part| <= kappa a^3/4 n_i n_j with
    kappa = 3/2 + sqrt(5/2) for R (the eps h term included) and 2 for I, so
    alpha_LB = 1/kappa.  The first term is not quadratic: Galerkin
    orthogonality removes only the part of conj(U a_j) inside span(U), leaving
    |(U a_j)^T A e_i| <= d_j n_i with d_j the distance (in the s-norm) from
    conj(U a_j) to span(U); with the eps h cross terms of R
    (<= sqrt(2 eps h) |U a_j| n_i) the linear part is at most
    a^3/4 (n_i e_j + n_j e_i), e_j >= d_j/2 + sqrt(2 eps h) |U a_j|.
    Gs, Dps: lists (one per shift) of (2M+3)^2 and M x M matrices.
    Returns (n_omega, 3, 3)."""
    omega = np.atleast_1d(np.asarray(omega, float))
    nw, M, _ = a.shape
    W = np.zeros((nw, 2 * M + 3, 3), np.complex128)
    for i in range(3):
        W[:, i, i] = 1j * omega
    W[:, 3:3 + M, :] = -a
    W[:, 3 + M:, :] = 1j * omega[:, None, None] * a
    ks = ref_index(s_ref, omega)
    out = np.empty((nw, 3, 3))
    for k in range(nw):
        Cm = W[k].conj().T @ Gs[ks[k]] @ W[k]  # c_ij
        n2 = np.real(np.diag(Cm))
        e = np.sqrt(np.maximum(np.real(np.einsum("mi,mn,ni->i", a[k].conj(), Dps[ks[k]], a[k])), 0.0))
        out[k] = _delta(n2, np.real(Cm), e, alpha, alpha_lb)
    return out


def certificate_direct(fo, U, a, omega, w, s_ref, alpha_lb=ALPHA_LB):
    """The same Delta_ij from full-order quantities: residuals
    res_i = r_i - A(omega) U a_i, dual norms with (X + s C)^{-1} by SuperLU, and
    the conjugation defect d_j = ||conj(q_j) - Pi conj(q_j)||_(X + s C)
    computed as the norm of the full-order difference.  e_j =
    (d_j^2 / 2 + 4 eps h |q_j|^2)^(1/2) as in conj_defect_matrix."""
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
        q = U @ a[k]
        res = fo.rhs(omega[k], w) - fo.A(omega[k]) @ q
        Yr = solve(res)
        G = res.conj().T @ Yr
        n2 = np.real(np.diag(G))
        cb = q.conj()
        c = np.linalg.solve(U.conj().T @ (Xs @ U), U.conj().T @ (Xs @ cb))
        dv = cb - U @ c
        d2 = np.real(np.einsum("ni,ni->i", dv.conj(), Xs @ dv))
        e = np.sqrt(0.5 * d2 + 4.0 * fo.eps_h * np.real(np.einsum("ni,ni->i", q.conj(), q)))
        out[k] = _delta(n2, np.real(G), e, fo.alpha, alpha_lb)
    return out


def pack(T):
    """(n, 3, 3) symmetric -> (n, 6) in the order 11 12 13 22 23 33."""
    return np.stack([T[:, i, j] for i, j in PAIRS], 1)


def certificate_data(rom, s_ref, gram):
    """Per-shift inputs of certificate_gform: gram(s) -> G_s for each s."""
    return {"s_ref": np.asarray(s_ref, float), "G": [gram(s) for s in s_ref],
            "Dp": [conj_defect_matrix(rom, s) for s in s_ref]}


def sweep(rom, omega, cert, alpha, alpha_lb=ALPHA_LB):
    """Reduced solves plus matrix-method tensors and certificates: (n_omega, 18).
    cert: certificate_data(...)."""
    a = reduced_solve(rom, omega)
    Rt, I = tensors_mm(rom, a, omega, rom["N0"], alpha)
    Dl = certificate_gform(cert["G"], cert["Dp"], cert["s_ref"], a, omega, alpha, alpha_lb)
    return np.concatenate([pack(Rt), pack(I), pack(Dl)], 1), a


# ------------------------------------------------------ selection (a5)
def select_snapshots(omega, delta, snap_omega, n_star):
    """Algorithm 1 selection step.

    Intervals w_n <= w < w_{n+1} between consecutive sorted snapshot
    frequencies, as in Algorithm 1, without their left end: w_n is a snapshot
    already, and a new snapshot there would repeat a column of D.  So
    Lambda_n = max over w_n < w < w_{n+1} and over (i, j) of Delta_ij;
    Lambda = max_n Lambda_n; the N_* intervals with the largest Lambda_n
    (ties: lower n) each contribute one new snapshot at the omega attaining
    Lambda_n (ties: smaller omega).
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
        inside = (omega > lo) & (omega < hi)
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
    """Threshold variant of the selection step (Section 4.4, after Hesthaven et al.):
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
    A0 = a0_of(rom)
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
    A0 = a0_of(rom)
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
