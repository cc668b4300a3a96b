"""Autotuner of the persistent batched sweep.

Searches the launch schedule of mpt_sweep_batched (frequencies per work item,
waves per workgroup, persistent workgroups per compute unit) on the actual
dictionary, timing each candidate with HIP events on the stream the graph is
launched on, and caches the best schedule in a JSON file keyed by a summary of
the dictionary (histograms of M and of the frequency counts)."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

from . import mpt

CANDIDATES = [(opi, wpg, gpc) for opi in (2, 4, 8, 16, 32) for wpg in (1, 2, 4) for gpc in (1, 2, 4)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mpt_autotune.json")


def dictionary_key(dic: "mpt.Dictionary") -> str:
    Ms = np.array([r.M for r in dic.roms])
    counts = np.diff(np.array(dic.offsets))
    hM = np.bincount(np.minimum(Ms // 8, 8), minlength=9)
    hn = np.bincount(np.minimum(counts // 500, 20), minlength=21)
    dev = torch.cuda.get_device_name(dic.omega.device)
    blob = json.dumps([dev, int(dic.n_obj), hM.tolist(), hn.tolist()])
    return hashlib.sha1(blob.encode()).hexdigest()[:16]


def time_schedule(dic, tune, reps=5):
    out = torch.empty((dic.omega.numel(), 18), dtype=torch.float64, device=dic.omega.device)
    st = torch.empty(dic.omega.numel(), dtype=torch.int32, device=dic.omega.device)
    mpt.mpt_sweep_batched(dic, tune=tune, use_graph=True, out=out, status=st)  # build + warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mpt.mpt_sweep_batched(dic, tune=tune, use_graph=True, out=out, status=st)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(dic, cache_path: str | None = DEFAULT_CACHE, candidates=CANDIDATES, verbose=False):
    """Best (omegas_per_item, waves_per_group, groups_per_cu) and its time in ms."""
    key = dictionary_key(dic)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        t = tuple(cache[key]["tune"])
        return t, time_schedule(dic, t), True
    best, best_ms = None, float("inf")
    for cand in candidates:
        ms = time_schedule(dic, cand)
        if verbose:
            print(f"  autotune {cand}: {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = cand, ms
    if cache_path:
        cache[key] = {"tune": list(best), "ms": best_ms}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, best_ms, False
