"""Seeded synthetic inputs for the MPT reduced-order hot path.

This package builds the full-order model that the paper delegates to an hp-FEM
code: a lowest-order edge (Yee) discretisation of the regularised eddy-current
problem for theta^(1) (Section 3, problem (theta1transtrun) and the weak form in
Section 3.1) on a Cartesian box, seeded objects and materials, the magnetostatic
theta~^(0) DOFs, and full-order snapshot solves (eq. (Linear)).

It holds none of the reduced-order method's arithmetic (POD, Galerkin
projection, reduced solves, tensor post-processing, certificates, snapshot
selection).  Both the CPU oracle tests and the GPU path consume its outputs.
"""
from .yee import YeeGrid, Operators, build_operators  # noqa: F401
from .shapes import Shape, sphere, ellipsoid, cuboid, torus, shell_sphere  # noqa: F401
from .fullorder import FullOrderSolver  # noqa: F401

from .workloads import WORKLOADS, Workload, Problem, make_problem, draw_object, log_grid  # noqa: F401
