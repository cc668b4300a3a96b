"""Benchmark of the MPT reduced-order hot path on one MI355X.

A step is one pass of the whole hot path over the 48^3 single-object workload
(seeded ellipsoid, sigma 1.5e7, N = 318,096 edge unknowns, 32 snapshots x 3
directions, TOL 1e-8, M <= 48, 10^4 output frequencies on [1e1, 1e6]):
  a1 POD basis of D (318,096 x 96 complex)      mpt_pod_basis
  a2 Galerkin projection + residual Gram         mpt_project
  a3+a4 sweep: reduced solves, tensors, certificates for 10^4 omegas   mpt_sweep
  a5 adaptive snapshot selection                 mpt_select_snapshots
Inputs (snapshots, operator, conductor block) are generated on the host before
timing and are resident in HBM.  value = output frequencies (tensor +
certificate each) per second of step time.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--forms]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TF = 78.6
FP64_MFMA_PEAK_TF = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_flops(M):
    """Algorithmic FP64 flops per (object, omega): complex LU 8/3 M^3, forming A
    4 M^2, three solves 24 M^2, four reduced mat-vecs on three vectors 96 M^2,
    quadratic forms and certificate dots O(M)."""
    return 8.0 / 3.0 * M ** 3 + 4 * M ** 2 + 24 * M ** 2 + 96 * M ** 2 + 200 * M


def spmm_bytes(N, nnz, M):
    """Algorithmic bytes of Y = K U: CSR (8 B value + 4 B index per nonzero,
    4 B per row pointer), U read once and Y written once (16 B per complex)."""
    return 12 * nnz + 4 * (N + 1) + 16 * M * N * 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2307_05590_amd import mpt
    from synth import make_problem

    mpt.lib()
    dev = torch.device("cuda:0")
    t0 = time.time()
    log("generating the ellipsoid48 workload (full-order snapshots on the host) ...")
    p = make_problem("ellipsoid48", verbose=True)
    ops = p.ops
    log(f"generated in {time.time() - t0:.1f} s: N={ops.N} nnz={ops.K.nnz} n_c={ops.cond_idx.size} "
        f"D={p.D.shape} residual={p.snap_residual:.1e}")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    D = T(p.D, torch.complex128)
    K = mpt.Csr.from_scipy(ops.K, dev)
    c = T(ops.c, torch.float64)
    w = T(p.w, torch.float64)
    o = T(p.o, torch.float64) if np.any(p.o) else None
    vol = T(ops.vol, torch.float64)
    cond = T(ops.cond_idx, torch.int32)
    S = T(p.S, torch.float64)
    omega = T(p.omega, torch.float64)
    snap = T(np.sort(p.snap_omega), torch.float64)
    tol, cap = p.wl.tol_sigma, p.wl.m_cap
    torch.cuda.synchronize()

    stages = ["pod", "project", "sweep", "select"]
    ev = {s: [] for s in stages}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        U, sig, M = mpt.mpt_pod_basis(D, tol, cap)
        e[1].record()
        rom = mpt.mpt_project(K, c, ops.eps_h, w, o, vol, ops.alpha, U, cond, S)
        e[2].record()
        out, st = mpt.mpt_sweep(rom, omega)
        e[3].record()
        new, lam, Lmax = mpt.mpt_select_snapshots(omega, out, snap, 2)
        e[4].record()
        if record:
            for i, s in enumerate(stages):
                ev[s].append((e[i], e[i + 1]))
        return M, out, st, new

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        M, out, st, new = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms = {s: float(np.mean([a.elapsed_time(b) for a, b in ev[s]])) for s in stages}
    assert int(st.abs().max()) == 0, "singular reduced system"
    n_omega = omega.numel()
    ms_step = 1e3 * elapsed / args.steps
    value = n_omega / (elapsed / args.steps)
    log(f"M={M}; ms/step {ms_step:.3f}; stages {ms}")

    # sweep kernel roofline (FP64 vector ALU) and the SpMM on its own (HBM)
    sweep_tf = sweep_flops(M) * n_omega / (ms["sweep"] * 1e-3) / 1e12
    U, _, _ = mpt.mpt_pod_basis(D, tol, cap)
    for _ in range(3):
        mpt.mpt_spmm(K, U)
    torch.cuda.synchronize()
    es, ee = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    es.record()
    for _ in range(reps):
        mpt.mpt_spmm(K, U)
    ee.record()
    torch.cuda.synchronize()
    spmm_ms = es.elapsed_time(ee) / reps
    spmm_gbs = spmm_bytes(ops.N, ops.K.nnz, M) / (spmm_ms * 1e-3) / 1e9

    dominant = max(stages, key=lambda s: ms[s])
    roofline = {"kernel": "sweep (k_sweep: reduced LU + solves + tensors + certificates)",
                "bound": "alu", "achieved": round(sweep_tf, 3), "peak": FP64_VALU_PEAK_TF,
                "unit": "TFLOP/s", "frac": round(sweep_tf / FP64_VALU_PEAK_TF, 4), "traffic": None,
                "flops_per_unit": sweep_flops(M), "units_per_launch": n_omega,
                "launch_ms": round(ms["sweep"], 4)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(p, args.cpu_seconds)

    line = {
        "metric": "MPT tensors/sec (3x3 + error cert per omega per object)",
        "value": round(value, 1),
        "unit": "tensors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ellipsoid48: one seeded ellipsoid on a 48^3 Yee grid, N=318096, "
                               "32 snapshots x 3 directions, TOL 1e-8, M<=48, 1e4 omegas",
                   "N": int(ops.N), "nnz": int(ops.K.nnz), "n_snap": int(p.snap_omega.size),
                   "M": int(M), "n_omega": int(n_omega), "n_c": int(ops.cond_idx.size)},
        "stages_ms": {k: round(v, 4) for k, v in ms.items()},
        "dominant_stage": dominant,
        "roofline": roofline,
        "spmm": {"bound": "hbm", "achieved": round(spmm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(spmm_gbs / HBM_PEAK_GBS, 4), "launch_ms": round(spmm_ms, 4),
                 "bytes_per_launch": spmm_bytes(ops.N, ops.K.nnz, M)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(p, budget_s):
    """The CPU oracle (LAPACK SVD, plain projection, per-omega LAPACK solves,
    matrix-method tensors and G-form certificates, selection) on a bounded
    frequency sample of the same workload."""
    from threadpoolctl import threadpool_info

    from oracle import rom as R
    from oracle.grid import FullOrder

    ops = p.ops
    t0 = time.perf_counter()
    fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
    U, s, M = R.pod_basis(p.D, p.wl.tol_sigma, p.wl.m_cap)
    rom = R.project(fo.K, fo.c, fo.eps_h, p.w, U)
    rom["N0"] = R.static_tensor_mesh(fo, p.o)
    G = R.residual_gram_schur(p.S, ops.cond_idx, fo.c, p.w, U, rom["KM"], rom["UhU"], fo.eps_h)
    t_off = time.perf_counter() - t0
    # sweep a growing sample until the budget is spent
    n = 250
    t_sw, done = 0.0, 0
    rng = np.random.default_rng(0)
    while t_sw < budget_s - t_off and done < p.omega.size:
        sel = np.sort(rng.choice(p.omega.size, min(n, p.omega.size), replace=False))
        t1 = time.perf_counter()
        out, _ = R.sweep(rom, p.omega[sel], G, ops.alpha)
        R.select_snapshots(p.omega[sel], out[:, 12:], p.snap_omega, 2)
        t_sw += time.perf_counter() - t1
        done += sel.size
        n *= 2
    # per-step rate: offline part once plus the sweep scaled to 1e4 omegas
    per_omega = t_sw / done
    step_s = t_off + per_omega * p.omega.size
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": round(p.omega.size / step_s, 2), "unit": "tensors/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"oracle POD+projection once ({t_off:.1f} s) and {done} sampled omegas "
                      f"({t_sw:.1f} s), step time = offline + per-omega x 1e4"}


if __name__ == "__main__":
    main()
