"""Lowest-order edge (Yee) grid on the box [-L, L]^3 with n^3 cells.

Stand-in for the hp H(curl) discretisation of Section 3.1: degrees of freedom
are line integrals of the field along grid edges, the curl maps them to face
fluxes, and the bilinear forms k, c, m of the weak form become
    K   = C^T diag(1/(mu_f h)) C          (curl-curl, mu~_r^{-1} weighted)
    C_s = alpha^2 mu_0 h diag(sigma_e)    (conductivity mass on B)
    eps M = eps h I                       (regularisation, applied everywhere)
The tangential trace n x theta = 0 on the outer boundary removes the edges that
lie in the boundary, so the unknowns are the 3 n (n-1)^2 interior edges.

Interior-edge numbering (the row order of every N-vector in this project):
    x-edges  (i, j, k), i in [0,n-1], j,k in [1,n-1]:  ((i)(n-1) + j-1)(n-1) + k-1
    y-edges  (i, j, k), i in [1,n-1], j in [0,n-1], k in [1,n-1]:
             n(n-1)^2 + ((i-1) n + j)(n-1) + k-1
    z-edges  (i, j, k), i,j in [1,n-1], k in [0,n-1]:
             2n(n-1)^2 + ((i-1)(n-1) + j-1) n + k
An a-edge (i,j,k) runs from node (i,j,k) one step along axis a; node (i,j,k)
sits at (-L + i h, -L + j h, -L + k h).

Faces that touch an interior edge, each oriented by the right-hand rule about
its +axis normal:
    x-faces at node plane i in [1,n-1], cell (j,k) in [0,n-1]^2
    y-faces at j in [1,n-1], cell (i,k);  z-faces at k in [1,n-1], cell (i,j)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

MU0 = 4e-7 * np.pi  # H/m; the paper's mu_0 (exact pre-2019 definition)


class YeeGrid:
    def __init__(self, n: int, L: float = 5.0):
        if n < 3:
            raise ValueError("need n >= 3 cells per side")
        self.n = int(n)
        self.L = float(L)
        self.h = 2.0 * self.L / self.n
        m = self.n - 1
        self.nx_edges = self.n * m * m
        self.N = 3 * self.nx_edges
        self.shape_x = (self.n, m, m)
        self.shape_y = (m, self.n, m)
        self.shape_z = (m, m, self.n)
        self.shape_fx = (m, self.n, self.n)
        self.shape_fy = (self.n, m, self.n)
        self.shape_fz = (self.n, self.n, m)
        self.n_faces = 3 * m * self.n * self.n

    # ---- coordinates -------------------------------------------------
    def coord(self, idx):
        return -self.L + np.asarray(idx, dtype=np.float64) * self.h

    def edge_midpoints(self) -> np.ndarray:
        """(N, 3) midpoints of the interior edges in numbering order."""
        n, m = self.n, self.n - 1
        out = np.empty((self.N, 3))
        i, j, k = np.meshgrid(np.arange(n), np.arange(1, n), np.arange(1, n), indexing="ij")
        blk = slice(0, self.nx_edges)
        out[blk, 0] = self.coord(i + 0.5).ravel()
        out[blk, 1] = self.coord(j).ravel()
        out[blk, 2] = self.coord(k).ravel()
        i, j, k = np.meshgrid(np.arange(1, n), np.arange(n), np.arange(1, n), indexing="ij")
        blk = slice(self.nx_edges, 2 * self.nx_edges)
        out[blk, 0] = self.coord(i).ravel()
        out[blk, 1] = self.coord(j + 0.5).ravel()
        out[blk, 2] = self.coord(k).ravel()
        i, j, k = np.meshgrid(np.arange(1, n), np.arange(1, n), np.arange(n), indexing="ij")
        blk = slice(2 * self.nx_edges, 3 * self.nx_edges)
        out[blk, 0] = self.coord(i).ravel()
        out[blk, 1] = self.coord(j).ravel()
        out[blk, 2] = self.coord(k + 0.5).ravel()
        del m
        return out

    def edge_axis(self) -> np.ndarray:
        return np.repeat(np.arange(3), self.nx_edges)

    def face_centres(self) -> np.ndarray:
        """(n_faces, 3) centres of x-, y-, z-faces in that order."""
        n = self.n
        parts = []
        i, j, k = np.meshgrid(np.arange(1, n), np.arange(n), np.arange(n), indexing="ij")
        parts.append(np.stack([self.coord(i), self.coord(j + 0.5), self.coord(k + 0.5)], -1).reshape(-1, 3))
        i, j, k = np.meshgrid(np.arange(n), np.arange(1, n), np.arange(n), indexing="ij")
        parts.append(np.stack([self.coord(i + 0.5), self.coord(j), self.coord(k + 0.5)], -1).reshape(-1, 3))
        i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(1, n), indexing="ij")
        parts.append(np.stack([self.coord(i + 0.5), self.coord(j + 0.5), self.coord(k)], -1).reshape(-1, 3))
        return np.concatenate(parts, 0)

    def face_axis(self) -> np.ndarray:
        return np.repeat(np.arange(3), self.n_faces // 3)

    def cell_centres(self) -> np.ndarray:
        c = self.coord(np.arange(self.n) + 0.5)
        X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
        return np.stack([X, Y, Z], -1).reshape(-1, 3)

    # ---- edge index helpers (return -1 for boundary edges) -----------
    def ex(self, i, j, k):
        n = self.n
        ok = (j >= 1) & (j <= n - 1) & (k >= 1) & (k <= n - 1) & (i >= 0) & (i <= n - 1)
        idx = (i * (n - 1) + (j - 1)) * (n - 1) + (k - 1)
        return np.where(ok, idx, -1)

    def ey(self, i, j, k):
        n = self.n
        ok = (i >= 1) & (i <= n - 1) & (k >= 1) & (k <= n - 1) & (j >= 0) & (j <= n - 1)
        idx = self.nx_edges + ((i - 1) * n + j) * (n - 1) + (k - 1)
        return np.where(ok, idx, -1)

    def ez(self, i, j, k):
        n = self.n
        ok = (i >= 1) & (i <= n - 1) & (j >= 1) & (j <= n - 1) & (k >= 0) & (k <= n - 1)
        idx = 2 * self.nx_edges + ((i - 1) * (n - 1) + (j - 1)) * n + k
        return np.where(ok, idx, -1)

    def curl(self) -> sp.csr_matrix:
        """Face-by-interior-edge incidence C with entries +-1 (circulation)."""
        n = self.n
        rows, cols, vals = [], [], []
        base = 0

        def add(face_ids, edge_ids, sign):
            keep = edge_ids >= 0
            rows.append(face_ids[keep])
            cols.append(edge_ids[keep])
            vals.append(np.full(keep.sum(), sign, dtype=np.float64))

        # x-faces: e_y(i,j,k) + e_z(i,j+1,k) - e_y(i,j,k+1) - e_z(i,j,k)
        i, j, k = [a.ravel() for a in np.meshgrid(np.arange(1, n), np.arange(n), np.arange(n), indexing="ij")]
        f = base + np.arange(i.size)
        add(f, self.ey(i, j, k), 1.0)
        add(f, self.ez(i, j + 1, k), 1.0)
        add(f, self.ey(i, j, k + 1), -1.0)
        add(f, self.ez(i, j, k), -1.0)
        base += i.size
        # y-faces: e_z(i,j,k) + e_x(i,j,k+1) - e_z(i+1,j,k) - e_x(i,j,k)
        i, j, k = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(1, n), np.arange(n), indexing="ij")]
        f = base + np.arange(i.size)
        add(f, self.ez(i, j, k), 1.0)
        add(f, self.ex(i, j, k + 1), 1.0)
        add(f, self.ez(i + 1, j, k), -1.0)
        add(f, self.ex(i, j, k), -1.0)
        base += i.size
        # z-faces: e_x(i,j,k) + e_y(i+1,j,k) - e_x(i,j+1,k) - e_y(i,j,k)
        i, j, k = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n), np.arange(1, n), indexing="ij")]
        f = base + np.arange(i.size)
        add(f, self.ex(i, j, k), 1.0)
        add(f, self.ey(i + 1, j, k), 1.0)
        add(f, self.ex(i, j + 1, k), -1.0)
        add(f, self.ey(i, j, k), -1.0)
        base += i.size
        C = sp.csr_matrix(
            (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
            shape=(base, self.N),
        )
        C.sum_duplicates()
        return C

    def gradient(self) -> sp.csr_matrix:
        """Interior-edge-by-interior-node incidence G (entries +-1): the edge
        line integrals of the gradient of a nodal potential that vanishes on
        the boundary.  Interior node (i,j,k), i,j,k in [1,n-1], has index
        ((i-1)(n-1) + j-1)(n-1) + k-1.  C G = 0 and G^T G is the 7-point
        Dirichlet Laplacian."""
        n, m = self.n, self.n - 1

        def node(i, j, k):
            ok = (i >= 1) & (i <= m) & (j >= 1) & (j <= m) & (k >= 1) & (k <= m)
            return np.where(ok, ((i - 1) * m + (j - 1)) * m + (k - 1), -1)

        rows, cols, vals = [], [], []
        ranges = [(self.ex, (np.arange(n), np.arange(1, n), np.arange(1, n))),
                  (self.ey, (np.arange(1, n), np.arange(n), np.arange(1, n))),
                  (self.ez, (np.arange(1, n), np.arange(1, n), np.arange(n)))]
        for ax, (index, axes) in enumerate(ranges):
            i, j, k = [a.ravel() for a in np.meshgrid(*axes, indexing="ij")]
            e = index(i, j, k)
            d = np.eye(3, dtype=np.int64)[ax]
            for sign, nd in ((1.0, node(i + d[0], j + d[1], k + d[2])), (-1.0, node(i, j, k))):
                keep = nd >= 0
                rows.append(e[keep])
                cols.append(nd[keep])
                vals.append(np.full(keep.sum(), sign))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.N, m ** 3))

    def rotation_field_dofs(self) -> np.ndarray:
        """(N, 3): column m holds the edge line integrals of e_m x xi.

        e_m x xi is linear and its a-component does not depend on xi_a, so the
        midpoint rule h (e_m x xi_mid)_a is exact on every a-edge.
        """
        P = self.edge_midpoints()
        ax = self.edge_axis()
        out = np.empty((self.N, 3))
        for m in range(3):
            e = np.zeros(3)
            e[m] = 1.0
            field = np.cross(np.broadcast_to(e, P.shape), P)
            out[:, m] = self.h * field[np.arange(self.N), ax]
        return out


@dataclass
class Operators:
    """Full-order operators of one object on one grid (all FP64)."""

    grid: YeeGrid
    alpha: float
    eps: float
    sigma_e: np.ndarray  # (N,) conductivity per interior edge [S/m]
    mu_f: np.ndarray  # (n_faces,) relative permeability per face
    K: sp.csr_matrix  # (N, N) curl-curl with 1/(mu_f h) weights, sorted columns
    c: np.ndarray  # (N,) diagonal of C_sigma = alpha^2 mu0 h sigma_e
    x: np.ndarray  # (N, 3) DOFs of e_i x xi
    cond_idx: np.ndarray  # (n_c,) int32 sorted indices of edges with c > 0
    vol: np.ndarray  # (3,) h^3 * sum over faces normal to e_i of (1 - 1/mu_f)
    cell_count: int  # number of cells whose centre is inside B

    @property
    def N(self) -> int:
        return self.grid.N

    @property
    def eps_h(self) -> float:
        return self.eps * self.grid.h

    @property
    def volume(self) -> float:
        """|B_alpha| on the staircase: alpha^3 h^3 #cells inside B."""
        return self.alpha ** 3 * self.grid.h ** 3 * self.cell_count


def build_operators(grid: YeeGrid, sigma_e, mu_f, alpha: float, eps: float, C=None, cell_count=0) -> Operators:
    if C is None:
        C = grid.curl()
    h = grid.h
    w = 1.0 / (np.asarray(mu_f, dtype=np.float64) * h)
    K = (C.T @ sp.diags(w) @ C).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    sigma_e = np.asarray(sigma_e, dtype=np.float64)
    c = alpha * alpha * MU0 * h * sigma_e
    cond_idx = np.flatnonzero(c > 0).astype(np.int32)
    fa = grid.face_axis()
    vol = np.array([h ** 3 * np.sum((1.0 - 1.0 / mu_f)[fa == a]) for a in range(3)])
    return Operators(grid=grid, alpha=float(alpha), eps=float(eps), sigma_e=sigma_e,
                     mu_f=np.asarray(mu_f, dtype=np.float64), K=K, c=c,
                     x=grid.rotation_field_dofs(), cond_idx=cond_idx, vol=vol,
                     cell_count=int(cell_count))
