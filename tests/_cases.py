"""Small seeded cases shared by the tests (built once per session)."""
import functools

import numpy as np

from synth.fullorder import FullOrderSolver
from synth.shapes import ellipsoid, shell_sphere, sphere, cuboid
from synth.workloads import reference_shifts
from synth.yee import YeeGrid, build_operators


class Case:
    def __init__(self, n, shape, snap, alpha=1e-2, eps=1e-10):
        self.grid = YeeGrid(n)
        sig, mu, nc = shape.assign(self.grid)
        self.ops = build_operators(self.grid, sig, mu, alpha, eps, cell_count=nc)
        self.fs = FullOrderSolver(self.ops)
        self.o, self.theta0_hist = self.fs.theta0()
        self.w = self.ops.x + self.o
        self.snap = np.asarray(snap, float)
        self.D, hist = self.fs.snapshots(self.snap, self.w, tol=1e-13, max_iter=12)
        self.snap_res = hist[-1]
        self.S = self.fs.schur()
        self.shape = shape
        # conductor block's eigenpairs (lam, V, sqrt(c)) and the reference
        # shifts of the certificate over the test band [1e1, 1e6]
        self.spec = self.fs._eig()
        self.lam = self.spec[0]
        self.Vt = np.ascontiguousarray(self.spec[1].T)
        self.s_ref = reference_shifts(1e1, 1e6)

    def oracle_fo(self):
        from oracle.grid import FullOrder
        o = self.ops
        return FullOrder(self.grid.n, o.sigma_e, o.mu_f, o.alpha, o.eps)


@functools.lru_cache(maxsize=None)
def sphere12():
    from synth import make_problem
    return make_problem("sphere12")


@functools.lru_cache(maxsize=None)
def ellipsoid16():
    return Case(16, ellipsoid(1.6, 1.2, 0.9, 5.8e7), np.logspace(1, 5, 16))


@functools.lru_cache(maxsize=None)
def shell16():
    """Two conducting materials that both carry eddy currents: a magnetic
    core (sigma 6e6, mu_r 50, r < 1.2) in a non-magnetic shell (sigma 3.5e7)."""
    return Case(16, shell_sphere(1.2, 2.0, (6e6, 50.0), (3.5e7, 1.0)), np.logspace(1, 6, 8))


@functools.lru_cache(maxsize=None)
def magnetic10():
    return Case(10, shell_sphere(1.0, 2.0, (6e6, 50.0), (3.5e7, 1.0)), np.logspace(1, 6, 8))


@functools.lru_cache(maxsize=None)
def cube10_mu():
    return Case(10, cuboid(1.5, 1.0, 1.5, 1e7, 8.0), np.logspace(1, 6, 6))


@functools.lru_cache(maxsize=None)
def ellipsoid16_k32():
    """The 16^3 ellipsoid with 32 snapshots (96 columns): room for M = 64."""
    return Case(16, ellipsoid(1.6, 1.2, 0.9, 5.8e7), np.logspace(1, 6, 32))
