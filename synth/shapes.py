"""Seeded object shapes B (dimensionless, centred at the origin) and materials.

Material assignment on the Yee grid: an edge carries sigma_* when its midpoint
is strictly inside a conducting region; a face carries mu_r when its centre is
inside a region.  Shapes are point-membership tests in the object frame; an
optional rotation maps world points into that frame (xi_obj = R^T xi).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Shape:
    kind: str
    params: dict
    materials: list  # [(sigma_*, mu_r)] for region labels 1, 2, ...
    R: np.ndarray = field(default_factory=lambda: np.eye(3))

    def region(self, pts: np.ndarray) -> np.ndarray:
        """Region label per point: 0 outside B, k >= 1 for material k-1."""
        p = np.asarray(pts, dtype=np.float64) @ self.R  # rows: R^T xi
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        k = self.kind
        P = self.params
        lab = np.zeros(p.shape[0], dtype=np.int64)
        if k == "sphere":
            lab[x * x + y * y + z * z < P["r"] ** 2] = 1
        elif k == "ellipsoid":
            a, b, c = P["a"], P["b"], P["c"]
            lab[(x / a) ** 2 + (y / b) ** 2 + (z / c) ** 2 < 1.0] = 1
        elif k == "cuboid":
            a, b, c = P["a"], P["b"], P["c"]
            lab[(np.abs(x) < a) & (np.abs(y) < b) & (np.abs(z) < c)] = 1
        elif k == "torus":
            Rm, rm = P["R"], P["r"]
            rho = np.sqrt(x * x + y * y)
            lab[(rho - Rm) ** 2 + z * z < rm * rm] = 1
        elif k == "shell_sphere":
            r2 = x * x + y * y + z * z
            lab[r2 < P["r_out"] ** 2] = 2
            lab[r2 < P["r_in"] ** 2] = 1
        else:
            raise ValueError(f"unknown shape {k}")
        return lab

    def assign(self, grid):
        """(sigma_e per interior edge, mu_f per face, #cells with centre in B)."""
        sig = np.array([0.0] + [m[0] for m in self.materials])
        mu = np.array([1.0] + [m[1] for m in self.materials])
        sigma_e = sig[self.region(grid.edge_midpoints())]
        mu_f = mu[self.region(grid.face_centres())]
        ncell = int(np.count_nonzero(self.region(grid.cell_centres())))
        return sigma_e, mu_f, ncell


def sphere(r, sigma, mu_r=1.0):
    return Shape("sphere", {"r": float(r)}, [(float(sigma), float(mu_r))])


def ellipsoid(a, b, c, sigma, mu_r=1.0, R=None):
    return Shape("ellipsoid", {"a": float(a), "b": float(b), "c": float(c)},
                 [(float(sigma), float(mu_r))], np.eye(3) if R is None else np.asarray(R))


def cuboid(a, b, c, sigma, mu_r=1.0, R=None):
    return Shape("cuboid", {"a": float(a), "b": float(b), "c": float(c)},
                 [(float(sigma), float(mu_r))], np.eye(3) if R is None else np.asarray(R))


def torus(Rmaj, rmin, sigma, mu_r=1.0, R=None):
    return Shape("torus", {"R": float(Rmaj), "r": float(rmin)},
                 [(float(sigma), float(mu_r))], np.eye(3) if R is None else np.asarray(R))


def shell_sphere(r_in, r_out, core, shell):
    """Two materials: core (sigma, mu_r) for r < r_in, shell for r_in <= r < r_out."""
    return Shape("shell_sphere", {"r_in": float(r_in), "r_out": float(r_out)},
                 [tuple(map(float, core)), tuple(map(float, shell))])


def random_rotation(rng) -> np.ndarray:
    """Uniform rotation in SO(3) from a QR of a Gaussian matrix (sign-fixed)."""
    A = rng.standard_normal((3, 3))
    Q, Rr = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(Rr))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q
