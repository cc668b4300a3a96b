"""The five seeded synthetic workloads (Yee-grid stand-ins for the paper's objects).

Seeds: numpy SeedSequence(230705590, spawn_key=(workload_id, object_id)).
Draw order per object: shape type, dimensions, rotation, sigma_*, mu_r, M, n_omega.

  1 sphere12      12^3 grid, unit sphere, sigma 5.8e7, mu_r 1; 16 snapshots on
                  [1e1,1e5]; TOL_Sigma 1e-6, M <= 16; 200 output omegas.
  2 ellipsoid48   48^3 grid, axis-aligned ellipsoid with semi-axes U[0.5,1.5],
                  sigma 1.5e7, mu_r 1; 32 snapshots on [1e1,1e6]; TOL 1e-8,
                  M <= 48; 1e4 output omegas on [1e1,1e6].
  3 dictionary32  32^3 grid, 256 objects: ellipsoid / cuboid / torus with
                  random dimensions and SO(3) orientation, sigma log-U[1e6,6e7],
                  mu_r in {1,8,32}; 16 snapshots on [1e1,1e6]; M ~ U{8..48};
                  n_omega ~ U{500..4000} on [1e1,1e6].
  4 adjoint48     64 ellipsoids as in 2; M ~ U{8..32}; 16 snapshots; 2000
                  omegas on [1e1,1e6].
  5 shell64       64^3 grid, steel core r < 0.6 (mu_r 50, sigma 6e6) in an
                  aluminium shell r < 1 (sigma 3.5e7); 48 initial snapshots on
                  [1e1,1e7] + 3 adaptive rounds x 2; TOL 1e-8, M <= 96; 1e5
                  output omegas on [1e1,1e7].
Snapshots of objects with their own spectral solves (1, 2, 5) are solved in
the split transverse/longitudinal form to a relative residual of 1e-12 or
better at every frequency; the largest is recorded in Problem.snap_residual.
All use alpha = 1e-2 m, eps = 1e-10 and the box [-5,5]^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fullorder import FullOrderSolver, RegionGreen
from .shapes import Shape, cuboid, ellipsoid, random_rotation, shell_sphere, sphere, torus
from .yee import Operators, YeeGrid, build_operators

SEED = 230705590


@dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    n: int
    n_objects: int
    n_snap: int
    snap_range: tuple
    tol_sigma: float
    m_cap: int
    n_omega: int
    omega_range: tuple
    alpha: float = 1e-2
    eps: float = 1e-10
    m_range: tuple | None = None  # fixed-rank M ~ U{lo..hi} per object
    n_omega_range: tuple | None = None
    adapt_rounds: int = 0
    n_star: int = 2
    gmres_cycles: int = 8  # GMRES budget of the shared-Green path once refinement stalls


WORKLOADS = {
    "sphere12": Workload(1, "sphere12", 12, 1, 16, (1e1, 1e5), 1e-6, 16, 200, (1e1, 1e5)),
    "ellipsoid48": Workload(2, "ellipsoid48", 48, 1, 32, (1e1, 1e6), 1e-8, 48, 10_000, (1e1, 1e6)),
    "dictionary32": Workload(3, "dictionary32", 32, 256, 16, (1e1, 1e6), 1e-8, 48, 0, (1e1, 1e6),
                             m_range=(8, 48), n_omega_range=(500, 4000)),
    "adjoint48": Workload(4, "adjoint48", 48, 64, 16, (1e1, 1e6), 1e-8, 32, 2000, (1e1, 1e6),
                          m_range=(8, 32)),
    "shell64": Workload(5, "shell64", 64, 1, 48, (1e1, 1e7), 1e-8, 96, 100_000, (1e1, 1e7),
                        adapt_rounds=3),
}


def rng_for(wid: int, obj: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(SEED, spawn_key=(wid, obj)))


@dataclass
class ObjectDraw:
    shape: Shape
    M_fixed: int | None
    n_omega: int


def draw_object(wl: Workload, obj: int) -> ObjectDraw:
    rng = rng_for(wl.wid, obj)
    if wl.name == "sphere12":
        shp = sphere(1.0, 5.8e7)
    elif wl.name in ("ellipsoid48", "adjoint48"):
        a, b, c = rng.uniform(0.5, 1.5, 3)
        shp = ellipsoid(a, b, c, 1.5e7)
    elif wl.name == "dictionary32":
        kind = ["ellipsoid", "cuboid", "torus"][rng.integers(0, 3)]
        if kind == "ellipsoid":
            dims = rng.uniform(0.4, 1.3, 3)
        elif kind == "cuboid":
            dims = rng.uniform(0.3, 0.8, 3)
        else:
            dims = np.array([rng.uniform(0.6, 1.0), rng.uniform(0.3, 0.45)])
        Rot = random_rotation(rng)
        sigma = float(np.exp(rng.uniform(np.log(1e6), np.log(6e7))))
        mu_r = float([1.0, 8.0, 32.0][rng.integers(0, 3)])
        if kind == "ellipsoid":
            shp = ellipsoid(*dims, sigma, mu_r, Rot)
        elif kind == "cuboid":
            shp = cuboid(*dims, sigma, mu_r, Rot)
        else:
            shp = torus(dims[0], dims[1], sigma, mu_r, Rot)
    elif wl.name == "shell64":
        shp = shell_sphere(0.6, 1.0, (6e6, 50.0), (3.5e7, 1.0))
    else:
        raise KeyError(wl.name)
    M_fixed = None
    if wl.m_range is not None:
        M_fixed = int(rng.integers(wl.m_range[0], wl.m_range[1] + 1))
    n_omega = wl.n_omega
    if wl.n_omega_range is not None:
        n_omega = int(rng.integers(wl.n_omega_range[0], wl.n_omega_range[1] + 1))
    return ObjectDraw(shp, M_fixed, n_omega)


def log_grid(lo, hi, n):
    return np.logspace(np.log10(lo), np.log10(hi), int(n))


def reference_shifts(lo, hi, per_decade=2):
    """Reference shifts of the certificate's norms X + s C_sigma: 0, then
    lo * 10^(k / per_decade) up to hi (the frequency band of the outputs)."""
    n = int(np.floor(per_decade * np.log10(hi / lo) + 1e-9)) + 1
    return np.r_[0.0, lo * 10.0 ** (np.arange(n) / per_decade)]


@dataclass
class Problem:
    """Everything the hot path consumes for one object (host arrays, FP64)."""

    wl: Workload
    obj: int
    draw: ObjectDraw
    ops: Operators
    snap_omega: np.ndarray  # (K,)
    omega: np.ndarray  # (n_omega,) output frequencies
    D: np.ndarray  # (N, 3K) complex, column block i holds q_i(snap_omega)
    o: np.ndarray  # (N, 3) theta~^(0) DOFs
    S: np.ndarray  # (n_c, n_c) conductor block of (K + eps h I)^{-1}
    snap_residual: float
    solver: FullOrderSolver = field(repr=False, default=None)

    @property
    def w(self) -> np.ndarray:
        return self.ops.x + self.o

    @property
    def s_ref(self) -> np.ndarray:
        return reference_shifts(*self.wl.omega_range)

    def cond_spectrum(self):
        """(lam, Vt): eigenvalues and eigenvectors (rows) of sqrt(c) S sqrt(c)
        on the conductor edges, S the conductor block of X^{-1}."""
        lam, V, _ = self.solver._eig()
        return lam, np.ascontiguousarray(V.T)

    @property
    def M_cap(self) -> int:
        return self.draw.M_fixed if self.draw.M_fixed is not None else self.wl.m_cap

    def add_snapshots(self, new_omega, tol=1e-12):
        """Full-order solves at new frequencies; appends to D (Alg. 1 update
        step) and returns the new columns [q_1(new) | q_2(new) | q_3(new)]."""
        Q, hist = self.solver.snapshots(np.asarray(new_omega, float), self.w, tol=tol, max_iter=12,
                                        gmres_cycles=self.wl.gmres_cycles)
        K0 = self.snap_omega.size
        k_new = len(new_omega)
        blocks = []
        for i in range(3):
            blocks.append(self.D[:, i * K0:(i + 1) * K0])
            blocks.append(Q[:, i * k_new:(i + 1) * k_new])
        self.D = np.ascontiguousarray(np.concatenate(blocks, 1))
        self.snap_omega = np.concatenate([self.snap_omega, np.asarray(new_omega, float)])
        self.snap_residual = max(self.snap_residual, hist[-1])
        return Q


# half-width of the box that contains every object of a dictionary workload
REGION_HALF_WIDTH = {"dictionary32": 1.5, "adjoint48": 1.5}


def region_green(name: str, grid: YeeGrid, verbose: bool = False) -> RegionGreen:
    """Shared X_1^{-1} block for the objects of a dictionary workload (mu_r
    corrections are applied per object)."""
    wl = WORKLOADS[name]
    return RegionGreen(grid, wl.eps * grid.h, REGION_HALF_WIDTH[name] + 1.01 * grid.h,
                       verbose=verbose)


def make_problem(name: str, obj: int = 0, n: int | None = None, n_snap: int | None = None,
                 n_omega: int | None = None, tol: float = 1e-12, grid: YeeGrid | None = None,
                 curl=None, verbose: bool = False, green: RegionGreen | None = None) -> Problem:
    """Build one object's full-order data.  n / n_snap / n_omega override sizes (tests)."""
    wl = WORKLOADS[name]
    draw = draw_object(wl, obj)
    nn = wl.n if n is None else n
    g = grid if grid is not None else YeeGrid(nn)
    C = curl if curl is not None else g.curl()
    sig, mu, ncell = draw.shape.assign(g)
    ops = build_operators(g, sig, mu, wl.alpha, wl.eps, C=C, cell_count=ncell)
    fo = FullOrderSolver(ops, C=C, green=green, verbose=verbose)
    o, _ = fo.theta0()
    K = wl.n_snap if n_snap is None else n_snap
    snap = log_grid(*wl.snap_range, K)
    D, hist = fo.snapshots(snap, ops.x + o, tol=tol, max_iter=12, verbose=verbose,
                           gmres_cycles=wl.gmres_cycles)
    no = draw.n_omega if n_omega is None else n_omega
    om = log_grid(*wl.omega_range, no)
    return Problem(wl, obj, draw, ops, snap, om, np.ascontiguousarray(D), o, fo.schur(), hist[-1], fo)
