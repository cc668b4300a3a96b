"""Full-order solves of the Yee stand-in (the offline stage of Section 4.1).

A(omega) = K + eps h I - i omega C_sigma,   r_i = i omega C_sigma (x_i + o_i)
(eq. (Linear) with the sign pairing of the weak form in Section 3.1 and the
source i nu theta^(0) of (theta1transtrun)).

Method (exact up to rounding, then refined against the sparse operator):
  * X_1 = K_1 + eps h I (mu = 1 everywhere) is diagonalised by orthonormal
    DCT-II / DST-I transforms: on a mode with symbols s_a = 2 sin(pi k_a/2n) it
    acts as (|s|^2 I - s s^T)/h + eps h I, inverted in closed form.
  * Permeable faces F enter as a rank-|F| Woodbury correction
    X_mu = X_1 + C_F^T diag((1/mu_f - 1)/h) C_F.
  * C_sigma is supported on the n_c conductor edges, so
    q = X^{-1}(f + i omega P D_c P^T q) reduces to a dense n_c system with the
    conductor Schur block S = P^T X^{-1} P.
  * X^{-1} = T + G L^{-1} G^T / (eps h): a transverse part T (bounded) and
    the gradients G of nodal potentials, on which K vanishes (L = G^T G, the
    nodal Laplacian, inverted by DST-I).  The 1/(eps h) part makes S
    ill-conditioned (its transverse information sits ~1e-5 below its
    rounding), so the conductor system is solved in split form: with
    nu = (i omega / eps h) G_c^T D_c z,
        z - i omega S_T D_c z - G_c Y nu = f_c,   eps h nu - i omega G_c^T D_c z = 0,
    S_T = P^T T P, G_c = P^T G, Y the nodal Green's function on the nodes of
    conductor edges: no entry carries the 1/(eps h) factor.  One
    eigendecomposition of D_c^{1/2} S_T D_c^{1/2} reduces each frequency to a
    dense system on those nodes.
  * Iterative refinement with residuals of the sparse A(omega) brings the
    relative residual to ~1e-13.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp

from .yee import Operators, YeeGrid


def _workers():
    return -1


class SpectralX1:
    """Exact inverse of X_1 = C^T C / h + eps_h I on the interior edges."""

    def __init__(self, grid: YeeGrid, eps_h: float):
        n = grid.n
        self.g = grid
        s = 2.0 * np.sin(np.pi * np.arange(n) / (2.0 * n))
        SX, SY, SZ = np.meshgrid(s, s, s, indexing="ij")
        S2 = SX * SX + SY * SY + SZ * SZ
        S2[0, 0, 0] = 1.0
        self.SX, self.SY, self.SZ = SX[..., None], SY[..., None], SZ[..., None]
        self.S2 = S2[..., None]
        self.ia = 1.0 / (S2[..., None] / grid.h + eps_h)
        self.ib = 1.0 / eps_h

    def apply(self, V: np.ndarray, chunk: int = 24, transverse: bool = False) -> np.ndarray:
        """X_1^{-1} V.  transverse=True for V in the range of C^T (curls of
        face fields): the longitudinal part of such V vanishes exactly, so it
        is dropped instead of amplified by 1/(eps h) from rounding."""
        V = np.asarray(V)
        one = V.ndim == 1
        if one:
            V = V[:, None]
        out = np.empty(V.shape, dtype=np.result_type(V.dtype, np.float64))
        for c0 in range(0, V.shape[1], chunk):
            out[:, c0:c0 + chunk] = self._apply(V[:, c0:c0 + chunk], transverse)
        return out[:, 0] if one else out

    def _apply(self, V, transverse=False):
        g = self.g
        n, B = g.n, V.shape[1]
        nx = g.nx_edges
        w = _workers()
        vx = V[:nx].reshape(g.shape_x + (B,))
        vy = V[nx:2 * nx].reshape(g.shape_y + (B,))
        vz = V[2 * nx:].reshape(g.shape_z + (B,))
        tx = sfft.dst(sfft.dst(sfft.dct(vx, 2, axis=0, norm="ortho", workers=w), 1, axis=1, norm="ortho", workers=w), 1, axis=2, norm="ortho", workers=w)
        ty = sfft.dst(sfft.dst(sfft.dct(vy, 2, axis=1, norm="ortho", workers=w), 1, axis=0, norm="ortho", workers=w), 1, axis=2, norm="ortho", workers=w)
        tz = sfft.dst(sfft.dst(sfft.dct(vz, 2, axis=2, norm="ortho", workers=w), 1, axis=0, norm="ortho", workers=w), 1, axis=1, norm="ortho", workers=w)
        dt = tx.dtype
        Ax = np.zeros((n, n, n, B), dt)
        Ay = np.zeros((n, n, n, B), dt)
        Az = np.zeros((n, n, n, B), dt)
        Ax[:, 1:, 1:] = tx
        Ay[1:, :, 1:] = ty
        Az[1:, 1:, :] = tz
        lon = (0.0 - self.ia) if transverse else (self.ib - self.ia)
        coef = (self.SX * Ax + self.SY * Ay + self.SZ * Az) * (lon / self.S2)
        ox = self.ia * Ax + self.SX * coef
        oy = self.ia * Ay + self.SY * coef
        oz = self.ia * Az + self.SZ * coef
        ox = ox[:, 1:, 1:]
        oy = oy[1:, :, 1:]
        oz = oz[1:, 1:, :]
        rx = sfft.idct(sfft.dst(sfft.dst(ox, 1, axis=1, norm="ortho", workers=w), 1, axis=2, norm="ortho", workers=w), 2, axis=0, norm="ortho", workers=w)
        ry = sfft.idct(sfft.dst(sfft.dst(oy, 1, axis=0, norm="ortho", workers=w), 1, axis=2, norm="ortho", workers=w), 2, axis=1, norm="ortho", workers=w)
        rz = sfft.idct(sfft.dst(sfft.dst(oz, 1, axis=0, norm="ortho", workers=w), 1, axis=1, norm="ortho", workers=w), 2, axis=2, norm="ortho", workers=w)
        return np.concatenate([rx.reshape(nx, B), ry.reshape(nx, B), rz.reshape(nx, B)], 0)


class SpectralLaplacian:
    """Exact inverse of the interior-node Dirichlet Laplacian L = G^T G by
    orthonormal DST-I transforms (symbols |s|^2 with s_a = 2 sin(pi k_a/2n))."""

    def __init__(self, grid: YeeGrid):
        n, m = grid.n, grid.n - 1
        s2 = (2.0 * np.sin(np.pi * np.arange(1, n) / (2.0 * n))) ** 2
        self.m = m
        self.sym = (s2[:, None, None] + s2[None, :, None] + s2[None, None, :])[..., None]

    def solve(self, F: np.ndarray) -> np.ndarray:
        m = self.m
        one = F.ndim == 1
        F = F.reshape(m ** 3, -1)
        w = _workers()
        t = sfft.dstn(F.reshape(m, m, m, -1), type=1, axes=(0, 1, 2), norm="ortho", workers=w)
        out = sfft.idstn(t / self.sym, type=1, axes=(0, 1, 2), norm="ortho",
                         workers=w).reshape(m ** 3, -1)
        return out[:, 0] if one else out


class RegionGreen:
    """X_1^{-1} restricted to the interior edges inside a centred box.

    Computed once per grid (one spectral solve per edge of the box); every
    object inside the box then gets its conductor block and its permeability
    correction from dense sub-blocks instead of its own spectral solves."""

    def __init__(self, grid: YeeGrid, eps_h: float, half_width: float, chunk: int = 48,
                 verbose: bool = False):
        self.grid = grid
        mid = grid.edge_midpoints()
        self.idx = np.flatnonzero(np.all(np.abs(mid) <= half_width, axis=1)).astype(np.int64)
        sx = SpectralX1(grid, eps_h)
        n = self.idx.size
        self.G = np.empty((n, n))
        t0 = __import__("time").time()
        for c0 in range(0, n, chunk):
            cols = self.idx[c0:c0 + chunk]
            E = np.zeros((grid.N, cols.size))
            E[cols, np.arange(cols.size)] = 1.0
            self.G[:, c0:c0 + cols.size] = sx.apply(E, chunk)[self.idx]
            if verbose and (c0 // chunk) % 40 == 0:
                print(f"  region Green's function {c0}/{n} ({__import__('time').time() - t0:.0f} s)",
                      flush=True)
        self.G = 0.5 * (self.G + self.G.T)

    def positions(self, edges):
        pos = np.searchsorted(self.idx, edges)
        if np.any(pos >= self.idx.size) or np.any(self.idx[np.minimum(pos, self.idx.size - 1)] != edges):
            raise ValueError("object edges outside the region of the Green's function")
        return pos


class FullOrderSolver:
    """Snapshots q_i(omega), theta~^(0) DOFs o_i and the conductor block S."""

    def __init__(self, ops: Operators, C=None, chunk: int = 24, green: RegionGreen | None = None,
                 verbose: bool = False):
        self.ops = ops
        self.verbose = verbose
        g = ops.grid
        self.chunk = chunk
        self.sx = SpectralX1(g, ops.eps_h)
        self.cond = ops.cond_idx.astype(np.int64)
        self.green = green
        F = np.flatnonzero(ops.mu_f != 1.0)
        self.F = F
        self._S = None
        if F.size:
            if C is None:
                C = g.curl()
            self.CF = C[F].tocsr()
            self.CFT = self.CF.T.tocsc()
            delta = 1.0 / ops.mu_f[F] - 1.0
            nF = F.size
            if green is not None:
                CFc = self.CF.tocoo()
                pos = green.positions(np.unique(CFc.col))
                lut = np.full(g.N, -1, dtype=np.int64)
                lut[np.unique(CFc.col)] = pos
                import scipy.sparse as sp
                CFR = sp.csr_matrix((CFc.data, (CFc.row, lut[CFc.col])), shape=(nF, green.idx.size))
                GC = CFR @ green.G  # (nF, nR)
                Gam = np.asarray((CFR @ GC.T))
                cpos = green.positions(self.cond)
                Wc = np.asarray(GC[:, cpos].T)
            else:
                Gam = np.empty((nF, nF))
                Wc = np.empty((self.cond.size, nF))
                for c0 in range(0, nF, chunk):
                    cols = self.CFT[:, c0:c0 + chunk].toarray()
                    W = self.sx.apply(cols, chunk, transverse=True)
                    Gam[:, c0:c0 + chunk] = self.CF @ W
                    Wc[:, c0:c0 + chunk] = W[self.cond]
            Gam = 0.5 * (Gam + Gam.T)
            self.cap = sla.lu_factor(np.diag(g.h / delta) + Gam)
            self.Wc = Wc
            self.delta = delta

    # ---- X^{-1} with the permeability correction ----------------------
    def xinv(self, V):
        U = self.sx.apply(V, self.chunk)
        if self.F.size:
            z = sla.lu_solve(self.cap, self.CF @ U)
            U = U - self.sx.apply(self.CFT @ z, self.chunk, transverse=True)
        return U

    def apply_X(self, V):
        ops = self.ops
        return ops.K @ V + ops.eps_h * V

    def apply_A(self, V, omega):
        """A(omega) V for V (N, B) with one omega per column."""
        ops = self.ops
        return ops.K @ V + ops.eps_h * V - 1j * (ops.c[:, None] * V) * np.asarray(omega)[None, :]

    # ---- conductor Schur block ---------------------------------------
    def schur(self) -> np.ndarray:
        """S = P^T X^{-1} P over the conductor edges (n_c x n_c, symmetric)."""
        if self._S is None and self.green is not None:
            cpos = self.green.positions(self.cond)
            S = self.green.G[np.ix_(cpos, cpos)].copy()
            if self.F.size:
                S -= self.Wc @ sla.lu_solve(self.cap, self.Wc.T)
            self._S = 0.5 * (S + S.T)
        if self._S is None:
            # S = S_T + G_c Y G_c^T / (eps h) from the split data
            sp_ = self.split()
            S = sp_["ST"] + (sp_["GY"] @ sp_["Gc"].T) / self.ops.eps_h
            self._S = 0.5 * (S + S.T)
        return self._S

    def residual_columns(self, U, w):
        """Z = [C_sigma w_1..3 | X U | C_sigma U] (N x (2M+3), complex) and
        X^{-1} Z by this solver, column by column: the inputs of the residual
        Gram in its full form."""
        ops = self.ops
        Z = np.concatenate([ops.c[:, None] * w, self.apply_X(U), ops.c[:, None] * U],
                           1).astype(np.complex128)
        Y = self.xinv(np.ascontiguousarray(Z.real)) + 1j * self.xinv(np.ascontiguousarray(Z.imag))
        return np.ascontiguousarray(Z), np.ascontiguousarray(Y)

    # ---- transverse / longitudinal split -------------------------------
    def tmu(self, V):
        """T_mu V: the transverse part of X^{-1} V (permeability included).
        The Woodbury correction lives in the range of C^T, so it only
        changes the transverse part."""
        U = self.sx.apply(V, self.chunk, transverse=True)
        if self.F.size:
            z = sla.lu_solve(self.cap, self.CF @ U)
            U = U - self.sx.apply(self.CFT @ z, self.chunk, transverse=True)
        return U

    def split(self):
        """Conductor data of the split form (built once): S_T, G_c, G_c Y,
        the eigenpairs of D_c^{1/2} S_T D_c^{1/2} and the per-frequency
        reduction onto the nodes of conductor edges."""
        if getattr(self, "_sp", None) is not None:
            return self._sp
        from scipy.sparse.csgraph import connected_components

        ops = self.ops
        g = ops.grid
        cond = self.cond
        nc = cond.size
        G = g.gradient()
        lap = SpectralLaplacian(g)
        ST = np.empty((nc, nc))
        for c0 in range(0, nc, self.chunk):
            if self.verbose and c0 % (40 * self.chunk) == 0:
                print(f"  conductor block (transverse): {c0}/{nc} columns", flush=True)
            idx = cond[c0:c0 + self.chunk]
            E = np.zeros((ops.N, idx.size))
            E[idx, np.arange(idx.size)] = 1.0
            ST[:, c0:c0 + idx.size] = self.sx.apply(E, self.chunk, transverse=True)[cond]
        if self.F.size:  # the permeability correction is transverse
            ST -= self.Wc @ sla.lu_solve(self.cap, self.Wc.T)
        ST = 0.5 * (ST + ST.T)
        Gcond = G[cond].tocsc()
        cn = np.flatnonzero(np.diff(Gcond.indptr) > 0)  # nodes of conductor edges
        Gc = Gcond[:, cn].toarray()
        Gcond = Gcond.tocsr()
        GY = np.empty((nc, cn.size))  # G_c Y, Y = L^{-1} on those nodes
        for c0 in range(0, cn.size, 4 * self.chunk):
            nd = cn[c0:c0 + 4 * self.chunk]
            E = np.zeros((G.shape[1], nd.size))
            E[nd, np.arange(nd.size)] = 1.0
            GY[:, c0:c0 + nd.size] = Gcond @ lap.solve(E)
        ncomp, lab = connected_components(sp.csr_matrix(np.abs(Gc).T @ np.abs(Gc)), directed=False)
        Cc = np.zeros((cn.size, ncomp))
        Cc[np.arange(cn.size), lab] = 1.0
        Cc /= np.linalg.norm(Cc, axis=0)
        d = np.sqrt(ops.c[cond])
        lam, V = np.linalg.eigh(d[:, None] * ST * d[None, :])
        self._sp = {"G": G, "lap": lap, "ST": ST, "Gc": Gc, "GY": GY, "cn": cn, "Cc": Cc,
                    "d": d, "lam": lam, "V": V, "P1": (Gc.T * d[None, :]) @ V,
                    "P2": V.T @ (d[:, None] * GY)}
        return self._sp

    def _split_solve(self, fc, omega):
        """(z, nu) of  z - i w S_T D z - G_c Y nu = f_c,  eps_h nu - i w G_c^T D z = 0
        for each column of f_c (n_c, B) with its own omega; one dense
        factorisation per distinct omega on the nodes of conductor edges.
        Constant potentials on each connected conductor piece have no
        gradient there, so nu has no component along them: that direction of
        the reduced matrix (eigenvalue eps h) is lifted to its scale."""
        sp_ = self.split()
        lam, V, d, P1, P2, Cc = (sp_[k] for k in ("lam", "V", "d", "P1", "P2", "Cc"))
        omega = np.asarray(omega, dtype=np.float64)
        fh = V.T @ (d[:, None] * fc)
        Z = np.empty(fc.shape, dtype=np.complex128)
        NU = np.empty((P1.shape[0], fc.shape[1]), dtype=np.complex128)
        eye = np.eye(P1.shape[0])
        for om in np.unique(omega):
            cols = np.flatnonzero(omega == om)
            R = 1.0 / (1.0 - 1j * om * lam)
            Mw = -1j * om * ((P1 * R.real[None, :]) @ P2 + 1j * ((P1 * R.imag[None, :]) @ P2))
            gam = max(np.abs(Mw).sum(1).max(), self.ops.eps_h)
            Mw += self.ops.eps_h * eye + gam * (Cc @ Cc.T)
            rhs = 1j * om * (P1 @ (R[:, None] * fh[:, cols]))
            nu = sla.solve(Mw, rhs)
            Z[:, cols] = (V @ (R[:, None] * (fh[:, cols] + P2 @ nu))) / d[:, None]
            NU[:, cols] = nu
        return Z, NU

    def _split_field(self, Z, NU, omega, base=None):
        """base + i w T_mu(C z) + G L^{-1} E nu: the full field from the
        conductor unknowns."""
        sp_ = self.split()
        ops = self.ops
        CZ = np.zeros((ops.N, Z.shape[1]), dtype=np.complex128)
        CZ[self.cond] = ops.c[self.cond][:, None] * Z
        En = np.zeros((sp_["G"].shape[1], Z.shape[1]), dtype=np.complex128)
        En[sp_["cn"]] = NU
        out = 1j * np.asarray(omega)[None, :] * self.tmu(CZ) + sp_["G"] @ sp_["lap"].solve(En)
        return out if base is None else base + out

    def _split_correction(self, res, omega):
        """A(omega)^{-1} res in split form: u = X^{-1} res, then the conductor
        system with f_c = u_c and d = u + i w X^{-1} C z."""
        sp_ = self.split()
        u = self.tmu(res) + sp_["G"] @ sp_["lap"].solve(sp_["G"].T @ res) / self.ops.eps_h
        Z, NU = self._split_solve(u[self.cond], omega)
        return self._split_field(Z, NU, omega, base=u)

    def _eig(self):
        """Eigenpairs (lam, V, d) of D_c^{1/2} S D_c^{1/2}, d = sqrt(c) on the
        conductor edges."""
        if not hasattr(self, "_lam"):
            if self.green is None:
                lam, V = self._eig_split()
                d = self.split()["d"]
            else:
                S = self.schur()
                d = np.sqrt(self.ops.c[self.cond])
                lam, V = np.linalg.eigh(d[:, None] * S * d[None, :])
            self._lam, self._V, self._d = lam, V, d
        return self._lam, self._V, self._d

    def _eig_split(self):
        """Eigenpairs of M = M_T + H Y H^T / (eps h) (M_T = D^{1/2} S_T D^{1/2},
        H = D^{1/2} G_c) to the accuracy of each eigenvalue's own scale.

        A dense eigensolver on M perturbs every eigenvector by eps ||M|| / gap,
        which is ~1e-5 for the transverse pairs here.  Instead: in orthonormal
        bases of null(H^T) (divergence-free conductor currents) and range(H),
        M = [[A, B], [B^T, C + E / eps_h]].  The invariant subspace of the
        small eigenvalues is span [I; X] with X solving the Riccati equation
        (C + E/eps_h) X = -B^T + X A + X B X (a contraction by
        ||(C + E/eps_h)^{-1}|| ||A||, so a few fixed-point steps converge);
        [I; X] and [-X^T; I] are exactly orthogonal, and each block is
        diagonalised on its own scale."""
        sp_ = self.split()
        d, ST, Gc, GY = sp_["d"], sp_["ST"], sp_["Gc"], sp_["GY"]
        eh = self.ops.eps_h
        MT = d[:, None] * ST * d[None, :]
        H = d[:, None] * Gc
        Uh, sv, _ = np.linalg.svd(H, full_matrices=True)
        r = Gc.shape[1] - sp_["Cc"].shape[1]  # rank: one constant per conductor piece
        QR, QN = Uh[:, :r], Uh[:, r:]
        E = QR.T @ ((d[:, None] * GY) @ (H.T @ QR))
        E = 0.5 * (E + E.T)
        A = QN.T @ MT @ QN
        Bm = QN.T @ MT @ QR
        Cbig = QR.T @ MT @ QR + E / eh
        Cbig = 0.5 * (Cbig + Cbig.T)
        cf = sla.cho_factor(Cbig)
        X = np.zeros((r, QN.shape[1]))
        for _ in range(8):
            Xn = sla.cho_solve(cf, -Bm.T + X @ A + X @ (Bm @ X))
            done = np.abs(Xn - X).max() <= 1e-15 * max(np.abs(Xn).max(), 1e-300)
            X = Xn
            if done:
                break

        def isqrt(Nm):
            w, Q = np.linalg.eigh(Nm)
            return (Q / np.sqrt(w)[None, :]) @ Q.T

        N1 = isqrt(np.eye(X.shape[1]) + X.T @ X)
        N2 = isqrt(np.eye(r) + X @ X.T)
        A1 = N1 @ (A + Bm @ X + X.T @ Bm.T + X.T @ (Cbig @ X)) @ N1
        A2 = N2 @ (Cbig - X @ Bm - Bm.T @ X.T + X @ (A @ X.T)) @ N2
        l1, W1 = np.linalg.eigh(0.5 * (A1 + A1.T))
        l2, W2 = np.linalg.eigh(0.5 * (A2 + A2.T))
        V1 = (QN + QR @ X) @ (N1 @ W1)
        V2 = (QR - QN @ X.T) @ (N2 @ W2)
        lam = np.r_[l1, l2]
        V = np.concatenate([V1, V2], 1)
        order = np.argsort(lam)
        return lam[order], np.ascontiguousarray(V[:, order])

    def _csolve(self, u_c, omega):
        """Solve (I - i w S D_c) q_c = u_c for each column (own omega)."""
        lam, V, d = self._eig()
        y = V.T @ (d[:, None] * u_c)
        y = y / (1.0 - 1j * lam[:, None] * np.asarray(omega)[None, :])
        return (V @ y) / d[:, None]

    def _solve_general(self, f, omega):
        u = self.xinv(f)
        qc = self._csolve(u[self.cond], omega)
        g = np.zeros_like(u)
        g[self.cond] = self.ops.c[self.cond][:, None] * qc
        return u + 1j * np.asarray(omega)[None, :] * self.xinv(g)

    def snapshots(self, omegas, w, tol=1e-13, max_iter=8, verbose=False, gmres_cycles=8):
        """Full-order q_i(omega_k); returns D (N, 3K) = [q_1(w_1..K)|q_2|q_3] and residuals."""
        if self.green is None:
            return self._snapshots_split(omegas, w, tol, max_iter, verbose)
        ops = self.ops
        omegas = np.asarray(omegas, dtype=np.float64)
        K = omegas.size
        om = np.tile(omegas, 3)  # column j -> direction j // K, frequency j % K
        W = np.repeat(w, K, axis=1)  # (N, 3K)
        cond = self.cond
        c_c = ops.c[cond]
        r = 1j * om[None, :] * (ops.c[:, None] * W)
        S = self.schur()
        u_c = 1j * om[None, :] * (S @ (c_c[:, None] * W[cond]))
        qc = self._csolve(u_c, om)
        g = np.zeros((ops.N, 3 * K), dtype=np.complex128)
        g[cond] = c_c[:, None] * (W[cond] + qc)
        Q = 1j * om[None, :] * self.xinv(g)
        rn = np.linalg.norm(r, axis=0)
        hist = []
        prev, Qprev = np.inf, None
        for it in range(max_iter):
            res = r - self.apply_A(Q, om)
            rel = np.linalg.norm(res, axis=0) / rn
            hist.append(float(rel.max()))
            if verbose:
                print(f"  refine {it}: max rel residual {rel.max():.3e}", flush=True)
            if rel.max() <= tol:
                return Q, hist
            if rel.max() > 0.5 * prev:  # refinement stalls or diverges
                if rel.max() > prev:  # keep the better iterate
                    Q = Qprev
                    hist.append(float(prev))
                break
            prev, Qprev = rel.max(), Q
            Q = Q + self._solve_general(res, om)
        else:
            res = r - self.apply_A(Q, om)
            hist.append(float((np.linalg.norm(res, axis=0) / rn).max()))
            return Q, hist
        # the preconditioner is too far from A^{-1} for a stationary
        # iteration (high sigma omega): restarted GMRES on the same operator,
        # within the given number of cycles (0: keep the best iterate)
        if gmres_cycles <= 0:
            return Q, hist
        for c0 in range(0, Q.shape[1], self.chunk):
            sl = slice(c0, c0 + self.chunk)
            Q[:, sl], h2 = self._gmres(r[:, sl], Q[:, sl], om[sl], tol, cycles=gmres_cycles,
                                       verbose=verbose)
            hist.append(h2)
        return Q, hist

    def _snapshots_split(self, omegas, w, tol, max_iter, verbose):
        """Snapshots by the split conductor system.  With z = w_c + q_c the
        equation q = i w X^{-1} C (w + q) becomes z - i w S D z = w_c on the
        conductor and q = i w X^{-1} C z, free of the 1/(eps h) cancellation
        that the right-hand side i w C w would carry; refinement steps solve
        A d = residual in the same split form."""
        ops = self.ops
        omegas = np.asarray(omegas, dtype=np.float64)
        K = omegas.size
        om = np.tile(omegas, 3)  # column j -> direction j // K, frequency j % K
        W = np.repeat(w, K, axis=1)
        r = 1j * om[None, :] * (ops.c[:, None] * W)
        Z, NU = self._split_solve(W[self.cond].astype(np.complex128), om)
        Q = self._split_field(Z, NU, om)
        rn = np.linalg.norm(r, axis=0)
        hist = []
        prev, Qprev = np.inf, None
        for it in range(max_iter):
            res = r - self.apply_A(Q, om)
            rel = np.linalg.norm(res, axis=0) / rn
            hist.append(float(rel.max()))
            if verbose:
                print(f"  refine {it}: max rel residual {rel.max():.3e}", flush=True)
            if rel.max() <= tol:
                break
            if rel.max() > 0.5 * prev:  # at the rounding floor
                if rel.max() > prev:
                    Q = Qprev
                    hist.append(float(prev))
                break
            prev, Qprev = rel.max(), Q
            Q = Q + self._split_correction(res, om)
        return Q, hist

    def _gmres(self, b, x, om, tol, m=30, cycles=8, verbose=False):
        """Right-preconditioned restarted GMRES(m) for A(om) x = b, one
        independent Krylov space per column (the columns advance in lockstep);
        the preconditioner is the spectral / Woodbury / Schur solve."""
        bn = np.linalg.norm(b, axis=0)
        B = b.shape[1]
        rel = None
        for cyc in range(cycles):
            r = b - self.apply_A(x, om)
            beta = np.linalg.norm(r, axis=0)
            rel = beta / bn
            if verbose:
                print(f"  gmres cycle {cyc}: max rel residual {rel.max():.3e}", flush=True)
            if rel.max() <= tol:
                break
            V = np.empty((m + 1,) + r.shape, dtype=np.complex128)
            H = np.zeros((B, m + 1, m), dtype=np.complex128)
            V[0] = r / beta
            k = m
            for j in range(m):
                w = self.apply_A(self._solve_general(V[j], om), om)
                for i in range(j + 1):
                    hij = np.einsum("nb,nb->b", V[i].conj(), w)
                    H[:, i, j] = hij
                    w = w - V[i] * hij
                hn = np.linalg.norm(w, axis=0)
                H[:, j + 1, j] = hn
                V[j + 1] = w / np.where(hn > 0, hn, 1.0)
                # residual estimate from the small least-squares problems
                e1 = np.zeros((B, j + 2), dtype=np.complex128)
                e1[:, 0] = beta
                est = np.array([np.linalg.norm(e1[c] - H[c, :j + 2, :j + 1] @ np.linalg.lstsq(
                    H[c, :j + 2, :j + 1], e1[c], rcond=None)[0]) for c in range(B)]) / bn
                if est.max() <= 0.5 * tol:
                    k = j + 1
                    break
            e1 = np.zeros((B, k + 1), dtype=np.complex128)
            e1[:, 0] = beta
            Y = np.stack([np.linalg.lstsq(H[c, :k + 1, :k], e1[c], rcond=None)[0] for c in range(B)], 1)
            x = x + self._solve_general(np.einsum("jnb,jb->nb", V[:k], Y), om)
        r = b - self.apply_A(x, om)
        return x, float((np.linalg.norm(r, axis=0) / bn).max())

    def theta0(self, tol=1e-13, max_iter=8):
        """theta~^(0) DOFs o_i: X_mu o_i = -(K_mu - K_1) x_i, zero on the boundary.

        Discrete form of the nu = 0 transmission problem for
        theta~^(0) = theta^(0) - e_i x xi (Section 3); zero when mu_r = 1.
        """
        ops = self.ops
        N = ops.N
        if not self.F.size:
            return np.zeros((N, 3)), [0.0]
        h = ops.grid.h
        Cx = self.CF @ ops.x  # face circulation of e_i x xi on F
        b = -(self.CFT @ ((self.delta / h)[:, None] * Cx))
        o = -self.sx.apply(self.CFT @ sla.lu_solve(self.cap, Cx), transverse=True)
        bn = np.linalg.norm(b, axis=0)
        hist = []
        for _ in range(max_iter):
            res = b - self.apply_X(o)
            rel = np.linalg.norm(res, axis=0) / bn
            hist.append(float(rel.max()))
            if rel.max() <= tol:
                break
            o = o + self.xinv(res)
        return o, hist
