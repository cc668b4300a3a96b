"""Oracle's own Yee-grid bookkeeping and full-order operators (FP64, SciPy).

Stand-in for the discretisation of Section 3.1 (weak form a = k - i w c + eps m,
matrices (kmatrix), (cmatrix)).  Built independently of the input generator:
unknowns are found from a node-indexed lookup table, and the face circulation
follows the right-hand rule for each cyclic axis triple.

Conventions (the interface shared with the data):
  * box [-L, L]^3, n cells per side, h = 2L/n; node p = (i,j,k) at -L + h p;
  * an a-edge starts at node p and ends at p + e_a; it is an unknown iff the two
    other coordinates of p lie in [1, n-1] (n x theta = 0 on the boundary);
  * unknowns are numbered x-edges, then y-edges, then z-edges, each block in
    C order of the start node;
  * faces with normal a sit at node planes p_a in [1, n-1] with p_b, p_c in
    [0, n-1] (C order), x-faces then y-faces then z-faces.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MU0 = 4.0e-7 * np.pi


class Grid:
    def __init__(self, n: int, L: float = 5.0):
        self.n, self.L = int(n), float(L)
        self.h = 2.0 * self.L / self.n
        P = np.indices((n + 1,) * 3)
        self.table = []
        start = []
        count = 0
        for a in range(3):
            ok = P[a] <= n - 1
            for b in range(3):
                if b != a:
                    ok &= (P[b] >= 1) & (P[b] <= n - 1)
            t = np.full((n + 1,) * 3, -1, dtype=np.int64)
            t[ok] = count + np.arange(int(ok.sum()))
            count += int(ok.sum())
            self.table.append(t)
            start.append(np.argwhere(ok))
        self.N = count
        self.edge_start = start  # per axis: (N_a, 3) start nodes in numbering order
        fstart = []
        for a in range(3):
            ok = (P[a] >= 1) & (P[a] <= n - 1)
            for b in range(3):
                if b != a:
                    ok &= P[b] <= n - 1
            fstart.append(np.argwhere(ok))
        self.face_start = fstart
        self.n_faces = sum(f.shape[0] for f in fstart)

    def _edge(self, a, nodes):
        n = self.n
        ok = np.all((nodes >= 0) & (nodes <= n), axis=1)
        out = np.full(nodes.shape[0], -1, dtype=np.int64)
        nn = nodes[ok]
        out[ok] = self.table[a][nn[:, 0], nn[:, 1], nn[:, 2]]
        return out

    def curl(self) -> sp.csr_matrix:
        rows, cols, vals = [], [], []
        f0 = 0
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            p = self.face_start[a]
            fid = f0 + np.arange(p.shape[0])
            eb = np.zeros(3, dtype=np.int64)
            ec = np.zeros(3, dtype=np.int64)
            eb[b] = 1
            ec[c] = 1
            for axis, off, s in ((b, 0 * eb, 1.0), (c, eb, 1.0), (b, ec, -1.0), (c, 0 * eb, -1.0)):
                e = self._edge(axis, p + off)
                keep = e >= 0
                rows.append(fid[keep])
                cols.append(e[keep])
                vals.append(np.full(int(keep.sum()), s))
            f0 += p.shape[0]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(f0, self.N))

    def face_normal_axis(self) -> np.ndarray:
        return np.concatenate([np.full(f.shape[0], a) for a, f in enumerate(self.face_start)])

    def source_dofs(self) -> np.ndarray:
        """(N, 3): h (e_m x xi)(midpoint) . t_e, the edge DOFs of e_m x xi."""
        out = np.zeros((self.N, 3))
        r = 0
        for a in range(3):
            mid = -self.L + self.h * (self.edge_start[a] + 0.5 * np.eye(3)[a])
            for m in range(3):
                out[r:r + mid.shape[0], m] = self.h * np.cross(np.eye(3)[m], mid)[:, a]
            r += mid.shape[0]
        return out


class FullOrder:
    """A(omega) = K + eps h I - i omega C_sigma and its pieces, assembled here."""

    def __init__(self, n, sigma_e, mu_f, alpha, eps, L=5.0):
        self.grid = Grid(n, L)
        g = self.grid
        self.alpha, self.eps = float(alpha), float(eps)
        self.h = g.h
        self.Cf = g.curl()
        self.mu_f = np.asarray(mu_f, float)
        self.face_w = 1.0 / (self.mu_f * g.h)  # 1/(mu_f h)
        self.K = (self.Cf.T @ sp.diags(self.face_w) @ self.Cf).tocsr()
        self.K1 = (self.Cf.T @ sp.diags(np.full(self.mu_f.size, 1.0 / g.h)) @ self.Cf).tocsr()
        self.c = alpha * alpha * MU0 * g.h * np.asarray(sigma_e, float)
        self.eps_h = self.eps * g.h
        self.X = (self.K + self.eps_h * sp.eye(g.N)).tocsc()
        self.x = g.source_dofs()
        self._Xlu = None

    def A(self, omega):
        return (self.X - 1j * omega * sp.diags(self.c)).tocsc()

    def rhs(self, omega, w):
        """r_i = i omega C_sigma w_i (source i nu theta^(0) of (theta1transtrun))."""
        return 1j * omega * (self.c[:, None] * w)

    def X_solve(self, B):
        """X^{-1} B by SuperLU (real factorisation, reused)."""
        if self._Xlu is None:
            import scipy.sparse.linalg as spla
            self._Xlu = spla.splu(self.X)
        B = np.asarray(B)
        if np.iscomplexobj(B):
            return self._Xlu.solve(np.ascontiguousarray(B.real)) + 1j * self._Xlu.solve(np.ascontiguousarray(B.imag))
        return self._Xlu.solve(B)

    def full_solve(self, omega, w):
        """Full-order q_i(omega), i = 1..3, by sparse direct solve (eq. (Linear))."""
        import scipy.sparse.linalg as spla
        return spla.splu(self.A(omega)).solve(self.rhs(omega, w))
