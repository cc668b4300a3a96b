"""Host logic of the benchmark's roofline accounting (no GPU): the per-unit
counts it divides by, and the link between the committed counter summaries
and the kernel sources they were taken on."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_sweep_flop_count_terms():
    # F(M) = 8/3 M^3 (LU) + 4 M^2 (forming A) + 24 M^2 (three solves) + 48 M^2
    # (K_M a, C_M a on three vectors) + 24 (2M+3)^2 (residual Gram mat-vecs)
    for M in (1, 16, 31, 45, 96):
        direct = 8.0 / 3.0 * M ** 3 + 4 * M ** 2 + 24 * M ** 2 + 48 * M ** 2 + 24 * (2 * M + 3) ** 2
        assert abs(bench.sweep_flops(M) - direct) <= 1e-9 * direct


def test_spmm_bytes_counts_each_array_once():
    N, nnz, M = 1000, 12750, 45
    # CSR values + column indices (12 B per nonzero), row pointers, U read
    # once and Y written once (16 B per complex entry each)
    assert bench.spmm_bytes(N, nnz, M) == 12 * nnz + 4 * (N + 1) + 32 * M * N


def test_counters_are_tied_to_the_sources():
    """Every per-launch HBM figure in the shell64 summary carries the digest
    of the sources it was measured on: the bench reports it (scaled by the
    copy calibration) exactly when the sources still have that digest."""
    text = open(bench.COUNTERS_SHELL).read()
    blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    cal = blob["calibration"]
    for kind, k in blob["kernels"].items():
        t = bench.measured_traffic(kind, bench.COUNTERS_SHELL)
        if k["source_sha1"] == bench.source_digest(kind):
            ref = 1024.0 * (k["fetch_kib"] * cal["fetch_factor"] + k["write_kib"] * cal["write_factor"])
            assert t == ref and t > 0, kind
        else:
            assert t is None, kind


def test_traffic_is_null_for_changed_sources(monkeypatch):
    monkeypatch.setitem(bench.KERNEL_SOURCES, "pencil_stage",
                        ["paper_2307_05590_amd/csrc/spmm.hip"])
    assert bench.measured_traffic("pencil_stage", bench.COUNTERS_SHELL) is None
