"""Benchmark of the MPT reduced-order hot path on one MI355X.

Default line: the 64^3 two-material sphere (shell64; steel core mu_r 50,
sigma 6e6 in an aluminium shell sigma 3.5e7; N = 762,048 edge unknowns; 48
initial snapshots x 3 directions, TOL 1e-8, M <= 96, 10^5 output frequencies
on [1e1, 1e7]).  Three adaptive rounds (Algorithm 1) add two frequencies each
from the certificates (host full-order solves at the chosen frequencies,
untimed; Lambda / |B_alpha| reported per round against TOL_Delta = 1e-3); then
a step is one pass of the whole hot path at the final snapshot set:
  a1 POD basis of D (762,048 x 162 complex)      mpt_pod_basis
  a2 Galerkin projection + certificate data      mpt_project
  a3+a4 sweep: reduced solves, tensors, certificates for 10^5 omegas
        (Hessenberg-triangular pencil form)      mpt_pencil_reduce + mpt_sweep_pencil
  a5 adaptive snapshot selection                 mpt_select_snapshots
Inputs are generated on the host before timing and are resident in HBM.
value = output frequencies (tensor + certificate each) per second of step
time.  The 48^3 single-object step (ellipsoid48, 10^4 omegas, LU sweep) is
measured after it and reported under "extra".

Other forms, each printing its own line:
  --form plain     the 48^3 single-object step alone
  --form batched   256-object dictionary on 32^3 grids (M ~ U{8..48}, 500-4000
                   omegas each): batched pencil sweep (or the persistent,
                   graph-captured, autotuned LU launch) against per-object calls
  --form adjoint   64 ellipsoids on 48^3 (M ~ U{8..32}, 2000 omegas): forward
                   sweep + adjoint sweep (dJ/domega, dJ/dsigma) of
                   J = sum |I_ij|^2 + |R~_ij - N0_ij|^2, batched and per object
  --form fmm       full matrix and integration methods on q = U a (48^3)
  --extras         with the default form: also the batched and adjoint lines
                   under "extra"
For the dictionaries the snapshots are refined to 1e-6 relative residual (the
reduced models stay Galerkin projections of the full operator).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--form adaptive|plain|batched|adjoint|fmm] [--objects N]
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



def cert_inputs(p, T):
    """Certificate inputs of mpt_project for a problem: the conductor block's
    eigenvectors (rows) and eigenvalues, and the reference shifts."""
    import torch
    lam, Vt = p.cond_spectrum()
    return T(Vt, torch.float64), T(lam, torch.float64), T(p.s_ref, torch.float64)


def oracle_cert(p, fo, U, rom):
    """The oracle's certificate data for a problem (the same conductor-block
    eigenpairs as the GPU path)."""
    from oracle import rom as R
    lam, Vt = p.cond_spectrum()
    A0 = rom["KM"] + fo.eps_h * rom["UhU"]
    dc = np.sqrt(fo.c[p.ops.cond_idx])
    return R.certificate_data(rom, p.s_ref, lambda s: R.residual_gram_spectral(
        lam, Vt.T, dc, p.ops.cond_idx, p.w, U, A0, s))

def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_ellipsoid48.md")
COUNTERS_SHELL = os.path.join(ROOT, "profiles", "counters_shell64_ellipsoid48.md")
KERNEL_SOURCES = {
    "sweep": ["paper_2307_05590_amd/csrc/sweep_impl.h", "paper_2307_05590_amd/csrc/sweep.hip",
              "paper_2307_05590_amd/csrc/device_util.h"],
    "spmm": ["paper_2307_05590_amd/csrc/spmm.hip", "paper_2307_05590_amd/csrc/device_util.h"],
    "sweep_pencil": ["paper_2307_05590_amd/csrc/pencil.hip",
                     "paper_2307_05590_amd/csrc/device_util.h"],
    "pencil_stage": ["paper_2307_05590_amd/csrc/pencil.hip",
                     "paper_2307_05590_amd/csrc/device_util.h"],
    "spmm64": ["paper_2307_05590_amd/csrc/spmm.hip", "paper_2307_05590_amd/csrc/device_util.h"],
    "sweep_e48": ["paper_2307_05590_amd/csrc/sweep_impl.h", "paper_2307_05590_amd/csrc/sweep.hip",
                  "paper_2307_05590_amd/csrc/device_util.h"],
}


def source_digest(kind):
    import hashlib
    h = hashlib.sha1()
    for rel in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, path=COUNTERS_FILE):
    """HBM bytes per launch of the kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, each scaled by what
    the counter reads for a plain 1 GiB copy), or None when the summary is
    missing or the kernel's sources changed since the counters were taken."""
    try:
        with open(path) as f:
            text = f.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    k = blob.get("kernels", {}).get(kind)
    cal = blob.get("calibration", {})
    if not k or k.get("source_sha1") != source_digest(kind):
        return None
    return 1024.0 * (k["fetch_kib"] * cal["fetch_factor"] + k["write_kib"] * cal["write_factor"])


def sweep_flops(M):
    """The per-omega flop count of the sweep as the method states it: complex
    LU 8/3 M^3, forming A 4 M^2, three solves 24 M^2, K_M a and C_M a 48 M^2,
    the certificate's mat-vecs with the (2M+3)-square residual Gram 24 (2M+3)^2,
    i.e. F(M) = 8/3 M^3 + 76 M^2 + 96 (M + 1.5)^2."""
    return 8.0 / 3.0 * M ** 3 + 76 * M ** 2 + 96 * (M + 1.5) ** 2


def pencil_sweep_flops(M):
    """Algorithmic FP64 flops per (object, omega) of the sweep on the
    Hessenberg-triangular pencil: column elimination with the interleaved back
    substitution on three right-hand sides 16 M^2, the transformed reduced
    products (four M x M matrices and six rows) on three vectors 96 M^2 +
    144 M, the quadratic-form contractions 96 M, the column transforms of the
    solution and the final formulas O(M)."""
    return 16 * M ** 2 + 96 * M ** 2 + 144 * M + 96 * M + 24 * M + 200


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
    ap.add_argument("--form", choices=["plain", "batched", "adjoint", "adaptive", "fmm"],
                    default="adaptive")
    ap.add_argument("--objects", type=int, default=0, help="dictionary size (default: the workload's)")
    ap.add_argument("--sweep", choices=["lu", "pencil"], default=None,
                    help="per-frequency LU of the reduced system, or the Hessenberg-triangular "
                         "pencil form (reduced once per step); default: lu for the 48^3 object, "
                         "pencil for the 64^3 object and the dictionary")
    ap.add_argument("--no-extras", action="store_true",
                    help="adaptive form only: skip the 48^3 plain step reported beside it")
    ap.add_argument("--extras", action="store_true",
                    help="adaptive form: also run the batched and adjoint dictionaries")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    sweep_arg = args.sweep
    if args.sweep is None:
        args.sweep = "pencil" if args.form in ("batched", "adaptive") else "lu"

    import torch

    from paper_2307_05590_amd import mpt

    mpt.lib()
    dev = torch.device("cuda:0")
    if args.calibrate:
        copy_calibration(dev)
    if args.form == "fmm":
        line = bench_fmm(args)
    elif args.form == "plain":
        line = bench_plain(args)
    elif args.form in ("batched", "adjoint"):
        line = bench_dictionary(args)
    else:
        line = bench_adaptive(args)
        extra = {}
        if not args.no_extras:
            torch.cuda.empty_cache()
            sub = argparse.Namespace(**vars(args))
            sub.form, sub.no_cpu = "plain", True
            sub.sweep = sweep_arg or "lu"
            extra["ellipsoid48_plain"] = summary(bench_plain(sub))
        if args.extras:
            for form in ("batched", "adjoint"):
                torch.cuda.empty_cache()
                sub = argparse.Namespace(**vars(args))
                sub.form, sub.no_cpu = form, True
                sub.sweep = sweep_arg or ("pencil" if form == "batched" else "lu")
                extra[("dictionary32_" if form == "batched" else "adjoint48_") + form] = \
                    summary(bench_dictionary(sub))
        if extra:
            line["extra"] = extra
    print(json.dumps(line), flush=True)


def summary(line):
    """The figures of another form's line, to sit under the headline's extra key."""
    keep = ("metric", "value", "unit", "ms_per_step", "config", "stages_ms", "roofline", "spmm",
            "plain_path", "alt_path", "snap_residual", "per_direction")
    return {k: line[k] for k in keep if k in line}


def bench_plain(args):
    """The 48^3 single-object step (ellipsoid48): POD, projection, sweep and
    selection over 10^4 omegas."""
    import torch

    from paper_2307_05590_amd import mpt
    from synth import make_problem

    dev = torch.device("cuda:0")
    t0 = time.time()
    log("generating the ellipsoid48 workload (full-order snapshots on the host) ...")
    p = make_problem("ellipsoid48", verbose=True)
    ops = p.ops
    log(f"generated in {time.time() - t0:.1f} s: N={ops.N} nnz={ops.K.nnz} n_c={ops.cond_idx.size} "
        f"D={p.D.shape} residual={p.snap_residual:.1e}")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    D = T(p.D, torch.complex128)
    K = mpt.Csr.from_scipy(ops.K, dev, row_blocks=3)
    c = T(ops.c, torch.float64)
    w = T(p.w, torch.float64)
    o = T(p.o, torch.float64) if np.any(p.o) else None
    vol = T(ops.vol, torch.float64)
    cond = T(ops.cond_idx, torch.int32)
    S = cert_inputs(p, T)
    omega = T(p.omega, torch.float64)
    snap = T(np.sort(p.snap_omega), torch.float64)
    tol, cap = p.wl.tol_sigma, p.wl.m_cap
    torch.cuda.synchronize()

    pencil = args.sweep == "pencil"
    stages = ["pod", "project", "pencil", "sweep", "select"] if pencil else \
        ["pod", "project", "sweep", "select"]
    ev = {s: [] for s in stages}

    def step(record):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
        e[0].record()
        U, sig, M = mpt.mpt_pod_basis(D, tol, cap)
        e[1].record()
        rom = mpt.mpt_project(K, c, ops.eps_h, w, o, vol, ops.alpha, U, cond, *S)
        e[2].record()
        if pencil:
            pen = mpt.mpt_pencil_reduce(rom)
            e[3].record()
            out, st = mpt.mpt_sweep_pencil(pen, omega)
        else:
            out, st = mpt.mpt_sweep(rom, omega)
        e[len(stages) - 1].record()
        new, lam, Lmax = mpt.mpt_select_snapshots(omega, out, snap, 2)
        e[len(stages)].record()
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
    fpu = pencil_sweep_flops(M) if pencil else sweep_flops(M)
    sweep_tf = fpu * n_omega / (ms["sweep"] * 1e-3) / 1e12
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

    # the paper's per-direction form on the same snapshots: one basis per
    # direction (POD of each D_i), projection onto [U_1 U_2 U_3], sweep with
    # each direction in its own basis
    Kd = p.snap_omega.size

    def perdir_step(record=None):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        Us = []
        for i in range(3):
            Ui, _, Mi = mpt.mpt_pod_basis(D[:, i * Kd:(i + 1) * Kd].contiguous(), tol, cap // 3)
            Us.append(Ui[:, :Mi])
        e[1].record()
        rom_d, _ = mpt.mpt_project_dirs(K, c, ops.eps_h, w, o, vol, ops.alpha, Us, cond, *S)
        e[2].record()
        out_d, st_d = mpt.mpt_sweep(rom_d, omega)
        e[3].record()
        if record is not None:
            record.append(e)
        return rom_d, st_d

    perdir_step()
    torch.cuda.synchronize()
    prec = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        rom_d, st_d = perdir_step(prec)
    torch.cuda.synchronize()
    pd_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    assert int(st_d.abs().max()) == 0, "singular reduced system (per-direction form)"
    pd_stage = {k: round(float(np.mean([e[i].elapsed_time(e[i + 1]) for e in prec])), 4)
                for i, k in enumerate(["pod", "project", "sweep"])}
    per_direction = {"form": "one POD basis per direction (M_i <= M_cap / 3), cross blocks, "
                             "each direction solved in its own basis",
                     "dirs": [int(x) for x in rom_d.dirs], "ms_per_step": round(pd_ms, 4),
                     "value": round(n_omega / (pd_ms * 1e-3), 1), "stages_ms": pd_stage}
    log(f"per-direction form: dirs {rom_d.dirs}, ms/step {pd_ms:.3f}, {pd_stage}")

    dominant = max(stages, key=lambda s: ms[s])
    if pencil:
        roofline = {"kernel": "sweep on the Hessenberg-triangular pencil (k_sweep_pencil: "
                              "Hessenberg solves + MFMA quadratic forms + tensors + certificates)",
                    "bound": "mfma", "achieved": round(sweep_tf, 3), "peak": FP64_VALU_PEAK_TF,
                    "unit": "TFLOP/s", "frac": round(sweep_tf / FP64_VALU_PEAK_TF, 4),
                    "traffic": measured_traffic("sweep_pencil"),
                    "flops_per_unit": fpu, "units_per_launch": n_omega,
                    "launch_ms": round(ms["sweep"], 4)}
    else:
        roofline = {"kernel": "sweep (k_sweep: reduced LU + solves + tensors + certificates)",
                    "bound": "alu", "achieved": round(sweep_tf, 3), "peak": FP64_VALU_PEAK_TF,
                    "unit": "TFLOP/s", "frac": round(sweep_tf / FP64_VALU_PEAK_TF, 4),
                    # counters of the 48^3 step (k_sweep<32, false> at M = 31)
                    "traffic": measured_traffic("sweep_e48", COUNTERS_SHELL) if M <= 32 else None,
                    "flops_per_unit": fpu, "units_per_launch": n_omega,
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
                 "bytes_per_launch": spmm_bytes(ops.N, ops.K.nnz, M),
                 "traffic": measured_traffic("spmm")},
        "snap_residual": float(p.snap_residual),
        "per_direction": per_direction,
        "cpu_baseline": cpu,
    }
    return line


COPY_BYTES = 1 << 30


def copy_calibration(dev):
    """Three plain device-to-device copies of 1 GiB (read 1 GiB, write 1 GiB):
    the per-dispatch FETCH_SIZE / WRITE_SIZE they report calibrate the HBM
    counters of the other kernels."""
    import torch

    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x {COPY_BYTES} bytes")
    del a, b


def build_dictionary(name, n_obj, dev, keep=2, tol_snap=1e-6):
    """Full-order data per object on the host (shared region Green's function),
    then the GPU POD basis (fixed rank) and projection per object."""
    import torch

    from paper_2307_05590_amd import mpt
    from synth import WORKLOADS, make_problem
    from synth.workloads import region_green
    from synth.yee import YeeGrid

    wl = WORKLOADS[name]
    g = YeeGrid(wl.n)
    C = g.curl()
    t0 = time.time()
    log(f"{name}: region Green's function on the {wl.n}^3 grid ...")
    gr = region_green(name, g, verbose=True)
    log(f"  {gr.idx.size} edges in {time.time() - t0:.0f} s")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    roms, omegas, sigmas, kept = [], [], [], []
    for o in range(n_obj):
        p = make_problem(name, o, grid=g, curl=C, tol=tol_snap, green=gr)
        ops = p.ops
        U, sig, M = mpt.mpt_pod_basis(T(p.D, torch.complex128), 0.0, p.M_cap)
        rom = mpt.mpt_project(mpt.Csr.from_scipy(ops.K, dev, row_blocks=3), T(ops.c, torch.float64), ops.eps_h,
                              T(p.w, torch.float64), T(p.o, torch.float64) if np.any(p.o) else None,
                              T(ops.vol, torch.float64), ops.alpha, U, T(ops.cond_idx, torch.int32),
                              *cert_inputs(p, T))
        roms.append(rom)
        omegas.append(T(p.omega, torch.float64))
        sigmas.append(p.draw.shape.materials[0][0])
        if len(kept) < keep:
            kept.append(p)
        if o % 16 == 15 or o == n_obj - 1:
            torch.cuda.synchronize()
            log(f"  {o + 1}/{n_obj} objects ({time.time() - t0:.0f} s)")
    return roms, omegas, sigmas, kept


def bench_dictionary(args):
    import torch

    from paper_2307_05590_amd import autotune, mpt

    dev = torch.device("cuda:0")
    name = "dictionary32" if args.form == "batched" else "adjoint48"
    from synth import WORKLOADS
    n_obj = args.objects or WORKLOADS[name].n_objects
    roms, omegas, sigmas, kept = build_dictionary(name, n_obj, dev)
    dic = mpt.Dictionary(roms, omegas)
    n_units = int(dic.omega.numel())
    Ms = np.array([r.M for r in roms])
    flops = float(sum(sweep_flops(r.M) * w.numel() for r, w in zip(roms, omegas)))
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res = {"plain_ms": None}
    if args.form == "batched":
        best, best_ms, cached = autotune.tune(dic, verbose=True)
        log(f"autotuned schedule {best} ({best_ms:.3f} ms, cached={cached})")
        out = torch.empty((n_units, 18), dtype=torch.float64, device=dev)
        st = torch.empty(n_units, dtype=torch.int32, device=dev)

        def lu_step():
            mpt.mpt_sweep_batched(dic, tune=best, use_graph=True, out=out, status=st)

        pbuf = [None]

        def pencil_step():
            # every object's pencil reduction, then the batched pencil sweep
            _, _, pbuf[0] = mpt.mpt_sweep_pencil_batched(dic, out=out, status=st, buf=pbuf[0])

        step, alt_step = (pencil_step, lu_step) if args.sweep == "pencil" else (lu_step, pencil_step)

        def plain():
            for r, w in zip(roms, omegas):
                mpt.mpt_sweep(r, w)
        tune_info = {"omegas_per_item": best[0], "waves_per_group": best[1], "groups_per_cu": best[2]}
    else:
        mult = torch.tensor([1.0, 2.0, 2.0, 1.0, 2.0, 2.0], dtype=torch.float64, device=dev)
        n0 = torch.cat([torch.stack([r.N0[0, 0], r.N0[0, 1], r.N0[0, 2], r.N0[1, 1], r.N0[1, 2],
                                     r.N0[2, 2]])[None].expand(w.numel(), 6)
                        for r, w in zip(roms, omegas)])
        dout = torch.zeros((n_units, 18), dtype=torch.float64, device=dev)
        out = torch.empty((n_units, 18), dtype=torch.float64, device=dev)
        st = torch.empty(n_units, dtype=torch.int32, device=dev)
        best = (8, 2, 2)
        alt_step = None

        def step():
            mpt.mpt_sweep_batched(dic, tune=best, use_graph=True, out=out, status=st)
            # dJ/dout of J = sum_omega sum_ij I_ij^2 + (R~_ij - N0_ij)^2 (caller's objective)
            dout[:, :6] = 2.0 * (out[:, :6] - n0) * mult
            dout[:, 6:12] = 2.0 * out[:, 6:12] * mult
            mpt.mpt_sweep_adjoint_batched(dic, dout)

        def plain():
            for o, (r, w) in enumerate(zip(roms, omegas)):
                a, b = dic.offsets[o], dic.offsets[o + 1]
                o1, _ = mpt.mpt_sweep(r, w)
                d = torch.zeros((w.numel(), 18), dtype=torch.float64, device=dev)
                d[:, :6] = 2.0 * (o1[:, :6] - n0[a:b]) * mult
                d[:, 6:12] = 2.0 * o1[:, 6:12] * mult
                mpt.mpt_sweep_adjoint(r, w, d)
        tune_info = {"omegas_per_item": best[0], "waves_per_group": best[1], "groups_per_cu": best[2]}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    t1 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_step = 1e3 * elapsed / args.steps
    assert int(st.abs().max()) == 0, "singular reduced system"
    plain()
    torch.cuda.synchronize()
    p0, p1 = ev(), ev()
    p0.record()
    plain()
    p1.record()
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1)
    value = n_units / (elapsed / args.steps)
    kernel_ms = e0.elapsed_time(e1) / args.steps
    alt = None
    if alt_step is not None:
        for _ in range(args.warmup):
            alt_step()
        torch.cuda.synchronize()
        a0, a1 = ev(), ev()
        a0.record()
        for _ in range(args.steps):
            alt_step()
        a1.record()
        torch.cuda.synchronize()
        alt_ms = a0.elapsed_time(a1) / args.steps
        alt = {"path": "lu batched" if args.sweep == "pencil" else "pencil batched",
               "value": round(n_units / (alt_ms * 1e-3), 1), "ms": round(alt_ms, 4)}
    # the adjoint kernel recomputes the forward work and adds the three A^H
    # solves (24 M^2) and the gradient dots (~24 M^2)
    pencil_form = args.form == "batched" and args.sweep == "pencil"
    if pencil_form:
        flops = float(sum(pencil_sweep_flops(r.M) * w.numel() for r, w in zip(roms, omegas)))
    fl = flops if args.form == "batched" else float(
        sum((2 * sweep_flops(r.M) + 48 * r.M ** 2) * w.numel() for r, w in zip(roms, omegas)))
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    cpu = None if args.no_cpu else cpu_baseline_dictionary(kept, args.form, args.cpu_seconds)
    line = {
        "metric": "MPT tensors/sec (3x3 + error cert per omega per object)" if args.form == "batched"
                  else "MPT tensors/sec with adjoint gradients (dJ/domega, dJ/dsigma) per omega per object",
        "value": round(value, 1), "unit": "tensors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"{name}: {n_obj} seeded objects" +
                                (" (ellipsoids/cuboids/tori, random SO(3), sigma log-U[1e6,6e7], "
                                 "mu_r in {1,8,32}) on 32^3 grids" if args.form == "batched"
                                 else " (ellipsoids as ellipsoid48) on 48^3 grids")),
                   "n_objects": n_obj, "n_units": n_units, "M_min": int(Ms.min()),
                   "M_max": int(Ms.max()), "M_mean": round(float(Ms.mean()), 2),
                   "schedule": tune_info},
        "plain_path": {"value": round(n_units / (plain_ms * 1e-3), 1), "ms": round(plain_ms, 4),
                       "speedup": round(plain_ms / kernel_ms, 3)},
        "alt_path": alt,
        "roofline": {"kernel": ("pencil reductions + batched pencil sweep" if pencil_form else
                                "persistent batched sweep" + (" + adjoint" if args.form == "adjoint"
                                                              else "")),
                     "bound": "mfma" if pencil_form else "alu", "achieved": round(achieved, 3),
                     "peak": FP64_VALU_PEAK_TF,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TF, 4),
                     "traffic": None, "launch_ms": round(kernel_ms, 4)},
        "cpu_baseline": cpu,
    }
    return line


def fmm_bytes(N, nnz, M, n_omega):
    """Algorithmic HBM bytes of the full matrix method over n_omega frequencies
    in batches of 16: per batch U read once (16 N M), the CSR once, the N x 48
    panels Q = U A and Y = K Q each written once and read once by the SpMM /
    the dot pass (Q twice)."""
    batches = (n_omega + 15) // 16
    return batches * (16 * N * M + 12 * nnz + 4 * (N + 1) + 5 * 16 * N * 48)


def bench_fmm(args):
    """Full matrix method (tensors from the reconstructed field q = U a with
    the full-order K and C_sigma) on the 48^3 workload, next to the reduced
    matrix method (the sweep) on the same frequencies: the comparison of
    methods the paper makes, on the stand-in."""
    import torch

    from paper_2307_05590_amd import mpt
    from synth import make_problem

    dev = torch.device("cuda:0")
    log("generating the ellipsoid48 workload (full-order snapshots on the host) ...")
    p = make_problem("ellipsoid48", verbose=True)
    ops = p.ops
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    K = mpt.Csr.from_scipy(ops.K, dev, row_blocks=3)
    c = T(ops.c, torch.float64)
    w = T(p.w, torch.float64)
    o = T(p.o, torch.float64) if np.any(p.o) else None
    cond = T(ops.cond_idx, torch.int32)
    n_fmm = 2000
    omega = T(p.omega[:: p.omega.size // n_fmm][:n_fmm], torch.float64)
    U, sig, M = mpt.mpt_pod_basis(T(p.D, torch.complex128), p.wl.tol_sigma, p.wl.m_cap)
    rom = mpt.mpt_project(K, c, ops.eps_h, w, o, T(ops.vol, torch.float64), ops.alpha, U, cond,
                          *cert_inputs(p, T))
    out_mm, st, a = mpt.mpt_sweep(rom, omega, want_a=True)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    ws = None
    for _ in range(args.warmup):
        out, ws = mpt.mpt_tensors_fmm(K, c, w, U, cond, a, omega, rom.N0, ops.alpha, ws)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1 = ev(), ev()
    t1 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        out, ws = mpt.mpt_tensors_fmm(K, c, w, U, cond, a, omega, rom.N0, ops.alpha, ws)
    e1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms = e0.elapsed_time(e1) / args.steps
    m0, m1 = ev(), ev()
    m0.record()
    for _ in range(args.steps):
        mpt.mpt_sweep(rom, omega)
    m1.record()
    torch.cuda.synchronize()
    mm_ms = m0.elapsed_time(m1) / args.steps
    # the integration-method analogue: sums over faces of the curl of q
    curl = mpt.Csr.from_scipy(ops.grid.curl(), dev)
    fw = T(1.0 / (ops.mu_f * ops.grid.h), torch.float64)
    wsi = None
    for _ in range(args.warmup):
        out_im, wsi = mpt.mpt_tensors_im(curl, fw, c, w, U, cond, a, omega, rom.N0, ops.alpha, wsi)
    torch.cuda.synchronize()
    i0, i1 = ev(), ev()
    i0.record()
    for _ in range(args.steps):
        out_im, wsi = mpt.mpt_tensors_im(curl, fw, c, w, U, cond, a, omega, rom.N0, ops.alpha, wsi)
    i1.record()
    torch.cuda.synchronize()
    im_ms = i0.elapsed_time(i1) / args.steps
    # the two methods agree (normwise, per frequency and part)
    o1, o2 = out.cpu().numpy(), out_mm.cpu().numpy()[:, :12]
    agree = max(float(np.max(np.abs(o1[:, 6 * q:6 * q + 6] - o2[:, 6 * q:6 * q + 6]) /
                             np.abs(o2[:, 6 * q:6 * q + 6]).max(1, keepdims=True))) for q in range(2))
    n = omega.numel()
    nbytes = fmm_bytes(ops.N, ops.K.nnz, M, n)
    gbs = nbytes / (ms * 1e-3) / 1e9
    line = {
        "metric": "MPT tensors/sec, full matrix method on q = U a (comparison method)",
        "value": round(n / (elapsed / args.steps), 1), "unit": "tensors/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ellipsoid48: N={ops.N}, M={M}, {n} of the 1e4 output frequencies",
                   "N": int(ops.N), "M": int(M), "n_omega": int(n)},
        "reduced_matrix_method": {"ms": round(mm_ms, 4), "value": round(n / (mm_ms * 1e-3), 1),
                                  "fmm_over_mm_time": round(ms / mm_ms, 1),
                                  "max_rel_difference": agree},
        "integration_method": {"ms": round(im_ms, 4), "value": round(n / (im_ms * 1e-3), 1),
                               "im_over_mm_time": round(im_ms / mm_ms, 1),
                               "max_rel_difference_vs_mm": max(float(np.max(np.abs(
                                   out_im.cpu().numpy()[:, 6 * q:6 * q + 6] - o2[:, 6 * q:6 * q + 6]) /
                                   np.abs(o2[:, 6 * q:6 * q + 6]).max(1, keepdims=True)))
                                   for q in range(2))},
        "roofline": {"kernel": "full matrix method (U A on MFMA, K Q SpMM, row reductions)",
                     "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(nbytes), "launch_ms": round(ms, 4)},
    }
    return line


def cpu_baseline_dictionary(kept, form, budget_s):
    """The CPU oracle on a bounded sample: POD, projection, residual Gram and the
    sweep (or the forward sensitivities) of the first objects."""
    from threadpoolctl import threadpool_info

    from oracle import rom as R
    from oracle.grid import FullOrder

    done, t = 0, 0.0
    for p in kept:
        ops = p.ops
        t0 = time.perf_counter()
        fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
        U, s, M = R.pod_basis(p.D, 0.0, p.M_cap)
        rom = R.project(fo.K, fo.c, fo.eps_h, p.w, U)
        rom["N0"] = R.static_tensor_mesh(fo, p.o)
        G = oracle_cert(p, fo, U, rom)
        t += time.perf_counter() - t0
        om = p.omega[: max(1, int(len(p.omega) * min(1.0, budget_s / 20.0)))]
        t0 = time.perf_counter()
        out, _ = R.sweep(rom, om, G, ops.alpha)
        if form == "adjoint":
            w6 = np.ones((om.size, 6))
            R.forward_sensitivity(rom, om, ops.alpha, w6, w6)
        t += time.perf_counter() - t0
        done += om.size
        if t > budget_s:
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": round(done / t, 2), "unit": "tensors/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(kept)} objects: oracle POD + projection + residual Gram + "
                      f"{'sweep + forward sensitivities' if form == 'adjoint' else 'sweep'} "
                      f"over {done} frequencies in {t:.1f} s"}


TOL_DELTA = 1e-3  # Algorithm 1's stopping tolerance in the adaptive sphere study


def pod_flops(N, m, M):
    """Flops of the two-pass POD on MFMA: two Hermitian Grams 4 m^2 N each, the
    rotation D V 8 m^2 N and the basis U = Q W 8 m M N (complex multiply-add =
    8 real flops; a Hermitian output counts half)."""
    return 2 * 4.0 * m * m * N + 8.0 * m * m * N + 8.0 * m * M * N


def bench_adaptive(args):
    """Adaptive POD (Algorithm 1) on the 64^3 two-material sphere (steel core
    mu_r 50, sigma 6e6 in an aluminium shell sigma 3.5e7): 48 initial
    snapshots, three rounds of POD + projection + sweep with certificates over
    10^5 omegas + selection of two new frequencies, each followed by host
    full-order solves at those frequencies (untimed), then the timed step: one
    pass of the hot path at the final snapshot set (M <= 96).  Each round
    reports Lambda / |B_alpha| against TOL_Delta = 1e-3; the rounds run to
    the workload's count whatever the rule says, so that the timed work is
    fixed."""
    import torch

    from paper_2307_05590_amd import mpt
    from paper_2307_05590_amd.adaptive import adaptive_pod
    from synth import make_problem

    dev = torch.device("cuda:0")
    t0 = time.time()
    log("shell64: 48 initial snapshots on the 64^3 grid (host) ...")
    p = make_problem("shell64", verbose=True)
    ops = p.ops
    t_gen = time.time() - t0
    log(f"generated in {t_gen:.0f} s: N={ops.N} nnz={ops.K.nnz} n_c={ops.cond_idx.size} "
        f"D={p.D.shape} max snapshot residual {p.snap_residual:.1e}")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    K = mpt.Csr.from_scipy(ops.K, dev, row_blocks=3)
    c = T(ops.c, torch.float64)
    w = T(p.w, torch.float64)
    o = T(p.o, torch.float64) if np.any(p.o) else None
    vol = T(ops.vol, torch.float64)
    cond = T(ops.cond_idx, torch.int32)
    S = cert_inputs(p, T)
    omega = T(p.omega, torch.float64)
    tol, cap, nstar = p.wl.tol_sigma, p.wl.m_cap, p.wl.n_star
    pencil = args.sweep == "pencil"

    def project(U):
        return mpt.mpt_project(K, c, ops.eps_h, w, o, vol, ops.alpha, U, cond, *S)

    def solve(new):
        t1 = time.time()
        Q = p.add_snapshots(new)
        log(f"  host snapshots at {new} in {time.time() - t1:.0f} s "
            f"(max residual so far {p.snap_residual:.1e})")
        return T(Q, torch.complex128)

    D, snap_h, rounds, _ = adaptive_pod(
        T(p.D, torch.complex128), p.snap_omega, omega, solve, project, tol_sigma=tol, m_cap=cap,
        n_star=nstar, volume=ops.volume, tol_delta=TOL_DELTA, max_rounds=p.wl.adapt_rounds,
        stop=False, sweep=args.sweep, log=log)
    torch.cuda.synchronize()
    snap = T(np.sort(snap_h), torch.float64)
    # pencil form: the projection and the pencil reduction are one call, the
    # reduction running beside the certificate data (project_reduce)
    stages = ["pod", "project_reduce" if pencil else "project", "sweep", "select"]
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(record=None, form=None):
        e = [ev() for _ in range(5)]
        e[0].record()
        U, sig, M = mpt.mpt_pod_basis(D, tol, cap)
        e[1].record()
        if (form or args.sweep) == "pencil":
            rom, pen = mpt.mpt_project_pencil(K, c, ops.eps_h, w, o, vol, ops.alpha, U, cond, *S)
            e[2].record()
            out, st = mpt.mpt_sweep_pencil(pen, omega)
        else:
            rom = project(U)
            e[2].record()
            out, st = mpt.mpt_sweep(rom, omega)
        e[3].record()
        new, lam, Lmax = mpt.mpt_select_snapshots(omega, out, snap, nstar)
        e[4].record()
        if record is not None:
            record.append(e)
        return M, out, st, U, rom

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rec = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        M, out, st, U, rom = step(rec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    assert int(st.abs().max()) == 0, "singular reduced system"
    ms = {s_: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in rec])) for i, s_ in
          enumerate(stages)}
    n_omega = omega.numel()
    ms_step = 1e3 * elapsed / args.steps
    value = n_omega / (elapsed / args.steps)
    log(f"final: {D.shape[1]} columns, M={M}, ms/step {ms_step:.3f}, {ms}")
    # the other sweep form on the same final snapshot set, for comparison
    alt_form = "lu" if pencil else "pencil"
    step(form=alt_form)
    torch.cuda.synchronize()
    arec = []
    for _ in range(args.steps):
        step(arec, form=alt_form)
    torch.cuda.synchronize()
    alt_sweep = float(np.mean([e[2].elapsed_time(e[3]) for e in arec]))
    alt_step = float(np.mean([e[0].elapsed_time(e[4]) for e in arec]))
    # the pencil reduction on its own (inside the step it runs beside the
    # certificate data), for the sweep stage's roofline
    reduce_ms = None
    if pencil:
        for _ in range(3):
            mpt.mpt_pencil_reduce(rom)
        torch.cuda.synchronize()
        er, ef = ev(), ev()
        er.record()
        for _ in range(10):
            mpt.mpt_pencil_reduce(rom)
        ef.record()
        torch.cuda.synchronize()
        reduce_ms = er.elapsed_time(ef) / 10
    # the SpMM of the projection on its own (HBM roofline)
    for _ in range(3):
        mpt.mpt_spmm(K, U)
    torch.cuda.synchronize()
    es, ee = ev(), ev()
    es.record()
    for _ in range(10):
        mpt.mpt_spmm(K, U)
    ee.record()
    torch.cuda.synchronize()
    spmm_ms = es.elapsed_time(ee) / 10
    spmm_gbs = spmm_bytes(ops.N, ops.K.nnz, M) / (spmm_ms * 1e-3) / 1e9

    sweep_ms = reduce_ms + ms["sweep"] if pencil else ms["sweep"]
    F = sweep_flops(M)
    stage_tf = F * n_omega / (sweep_ms * 1e-3) / 1e12
    m_cols = int(D.shape[1])
    pod_tf = pod_flops(ops.N, m_cols, M) / (ms["pod"] * 1e-3) / 1e12
    kern = {"kernel": "k_sweep_pencil (Hessenberg-triangular solves, MFMA quadratic forms, "
                      "tensors, certificates)",
            "flops_per_unit": pencil_sweep_flops(M), "launch_ms": round(ms["sweep"], 4)} if pencil \
        else {"kernel": "k_sweep_big" if M > 64 else "k_sweep", "flops_per_unit": sweep_flops(M),
              "launch_ms": round(ms["sweep"], 4)}
    kern["achieved"] = round(kern["flops_per_unit"] * n_omega / (ms["sweep"] * 1e-3) / 1e12, 3)
    kern["frac"] = round(kern["achieved"] / FP64_MFMA_PEAK_TF, 4)
    kern["unit"] = "TFLOP/s"
    cpu = None if args.no_cpu else cpu_baselines(p, args.cpu_seconds)
    line = {
        "metric": "MPT tensors/sec (3x3 + error cert per omega per object)",
        "value": round(value, 1), "unit": "tensors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "shell64: steel core (mu_r 50, sigma 6e6) in an aluminium shell "
                               "(sigma 3.5e7) on a 64^3 Yee grid, 48 + 3x2 adaptive snapshots, "
                               "TOL 1e-8, M<=96, 1e5 omegas",
                   "N": int(ops.N), "nnz": int(ops.K.nnz), "n_c": int(ops.cond_idx.size),
                   "n_snap": int(snap_h.size), "columns": m_cols, "M": int(M),
                   "n_omega": int(n_omega), "volume_B_alpha": ops.volume, "rounds": rounds},
        "snap_residual": float(p.snap_residual),
        "host_generation_s": round(t_gen, 1),
        "stages_ms": {k: round(v, 4) for k, v in ms.items()},
        "reduce_alone_ms": round(reduce_ms, 4) if pencil else None,
        "dominant_stage": max(ms, key=ms.get),
        "sweep_form": args.sweep,
        "alt_path": {"sweep_form": alt_form, "sweep_ms": round(alt_sweep, 4),
                     "step_ms_gpu": round(alt_step, 4)},
        "roofline": {"kernel": ("sweep stage a3+a4: k_pencil_reduce + k_pencil_z + k_sweep_pencil "
                                "(the reduction timed on its own)" if pencil else kern["kernel"]),
                     "bound": "mfma", "achieved": round(stage_tf, 3), "peak": FP64_MFMA_PEAK_TF,
                     "unit": "TFLOP/s", "frac": round(stage_tf / FP64_MFMA_PEAK_TF, 4),
                     "traffic": measured_traffic("pencil_stage", COUNTERS_SHELL) if pencil else None,
                     "flops_per_unit": round(F),
                     "flops_basis": "F(M) = 8/3 M^3 + 76 M^2 + 96 (M+1.5)^2 per omega",
                     "units_per_launch": int(n_omega), "launch_ms": round(sweep_ms, 4)},
        "stage_rooflines": {
            "sweep_kernel": kern,
            "pod": {"kernels": "k_gram_chunk x2, eigen chain, k_rotate x2", "bound": "mfma",
                    "flops": pod_flops(ops.N, m_cols, M), "achieved": round(pod_tf, 3),
                    "unit": "TFLOP/s", "frac": round(pod_tf / FP64_MFMA_PEAK_TF, 4),
                    "ms": round(ms["pod"], 4)},
            "spmm": {"kernel": "k_spmm (Y = K U)", "bound": "hbm", "achieved": round(spmm_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(spmm_gbs / HBM_PEAK_GBS, 4),
                     "launch_ms": round(spmm_ms, 4),
                     "bytes_per_launch": spmm_bytes(ops.N, ops.K.nnz, M),
                     "traffic": measured_traffic("spmm64", COUNTERS_SHELL)}},
        "cpu_baseline": cpu,
    }
    return line


def cpu_model():
    """The host CPU's model name (lscpu), and the number of CPUs it reports."""
    import subprocess
    name = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                name = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return name, os.cpu_count()


def cpu_baselines(p, budget_s):
    """The oracle's step on the host at every thread the BLAS pool has and at
    one thread (each with its own budget), with the CPU model."""
    from threadpoolctl import threadpool_limits

    log("CPU oracle baseline (all threads) ...")
    many = cpu_baseline(p, budget_s)
    log(f"  {many['value']} tensors/s on {many['cores']} threads; one thread ...")
    with threadpool_limits(limits=1):
        one = cpu_baseline(p, budget_s)
    log(f"  {one['value']} tensors/s on one thread")
    name, ncpu = cpu_model()
    many["one_thread"] = {"value": one["value"], "cores": one["cores"], "sample": one["sample"]}
    many["cpu_model"] = name
    many["nproc"] = ncpu
    return many


def cpu_baseline(p, budget_s):
    """The CPU oracle (LAPACK SVD, plain projection, per-omega LAPACK solves,
    matrix-method tensors and G-form certificates, selection) on the same
    workload: whole steps repeated until the budget is spent when one fits
    well inside it, else the offline part once and a bounded frequency
    sample scaled to the workload's frequency count."""
    from threadpoolctl import threadpool_info

    from oracle import rom as R
    from oracle.grid import FullOrder

    ops = p.ops
    n_om = p.omega.size

    def offline():
        fo = FullOrder(ops.grid.n, ops.sigma_e, ops.mu_f, ops.alpha, ops.eps)
        U, s, M = R.pod_basis(p.D, p.wl.tol_sigma, p.wl.m_cap)
        rom = R.project(fo.K, fo.c, fo.eps_h, p.w, U)
        rom["N0"] = R.static_tensor_mesh(fo, p.o)
        G = oracle_cert(p, fo, U, rom)
        return rom, G

    def sweep_select(rom, G, om):
        out, _ = R.sweep(rom, om, G, ops.alpha)
        R.select_snapshots(om, out[:, 12:], p.snap_omega, 2)

    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    rom, G = offline()
    t_off = time.perf_counter() - t0
    sel = np.sort(rng.choice(n_om, min(250, n_om), replace=False))
    t1 = time.perf_counter()
    sweep_select(rom, G, p.omega[sel])
    per_omega = (time.perf_counter() - t1) / sel.size
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    if t_off + per_omega * n_om <= 0.5 * budget_s:
        # whole steps: the offline part and every frequency, repeated
        steps, t_tot = 0, 0.0
        while steps == 0 or t_tot < budget_s:
            t1 = time.perf_counter()
            rom_k, G_k = offline()
            sweep_select(rom_k, G_k, p.omega)
            t_tot += time.perf_counter() - t1
            steps += 1
        return {"value": round(n_om * steps / t_tot, 2), "unit": "tensors/s", "cores": int(threads),
                "kind": "oracle",
                "sample": f"{steps} whole oracle steps (POD, projection, residual Gram, sweep and "
                          f"selection over all {n_om} omegas) in {t_tot:.1f} s"}
    # sweep a growing sample until the budget is spent
    n = 250
    t_sw, done = 0.0, 0
    while t_sw < budget_s - t_off and done < n_om:
        sel = np.sort(rng.choice(n_om, min(n, n_om), replace=False))
        t1 = time.perf_counter()
        sweep_select(rom, G, p.omega[sel])
        t_sw += time.perf_counter() - t1
        done += sel.size
        n *= 2
    # per-step rate: offline part once plus the sweep scaled to the frequency count
    step_s = t_off + t_sw / done * n_om
    return {"value": round(n_om / step_s, 2), "unit": "tensors/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"oracle POD+projection once ({t_off:.1f} s) and {done} sampled omegas "
                      f"({t_sw:.1f} s), step time = offline + per-omega x {n_om}"}


if __name__ == "__main__":
    main()
