"""Algorithm 1 (Section 4.4): the adaptive POD loop around the hot path.

Each round runs the whole path on the device (POD basis of the current
snapshot matrix, projection with the certificate data, the sweep with
certificates over the output frequencies, the selection) and then tests
Algorithm 1's stopping rule: the largest certificate over the open intervals
between snapshot frequencies, Lambda, relative to the object's volume |B_alpha|.
While Lambda / |B_alpha| > TOL_Delta, the caller's full-order solver supplies
the snapshots at the selected frequencies and the loop goes on.  Every step of
the path runs in the library; this module only sequences the calls and moves
the chosen frequencies to the host.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mpt


def adaptive_pod(D, snap_omega, omega, solve, project, *, tol_sigma, m_cap, n_star, volume,
                 tol_delta=1e-3, max_rounds=3, stop=True, sweep="pencil", log=None):
    """Run Algorithm 1's rounds.

    D: (N, 3K) complex128 snapshot matrix on the device; snap_omega: (K,)
    host frequencies of its columns; omega: output frequencies (device).
    solve(new_omega) -> (N, 3k) complex128 device columns of the full-order
    solutions at the k new frequencies; project(U) -> mpt.Rom (the Galerkin
    projection and certificate data for a basis).  tol_delta is TOL_Delta of
    the stopping rule; max_rounds caps the number of enrichments.  With
    stop=False the rounds run to max_rounds whatever the rule says (a fixed
    amount of work, for measurement), and each round still records whether
    the rule had been met.

    Returns (D, snap_omega, rounds, last): rounds is a list of dicts with the
    round's column count, M, Lambda, Lambda/|B_alpha|, whether
    Lambda/|B_alpha| <= tol_delta, and the frequencies it added; last holds
    the final round's basis, reduced model and sweep output."""
    snap_omega = np.asarray(snap_omega, dtype=np.float64)
    rounds = []
    r = 0
    while True:
        snap = torch.as_tensor(np.sort(snap_omega), dtype=torch.float64, device=omega.device)
        U, sig, M = mpt.mpt_pod_basis(D, tol_sigma, m_cap)
        rom = project(U)
        if sweep == "pencil":
            out, st = mpt.mpt_sweep_pencil(mpt.mpt_pencil_reduce(rom), omega)
        else:
            out, st = mpt.mpt_sweep(rom, omega)
        new, _, Lmax = mpt.mpt_select_snapshots(omega, out, snap, n_star)
        if int(st.abs().max()) != 0:
            raise mpt.MptError("singular reduced system in an adaptive round")
        lam = float(Lmax.item())
        rel = lam / volume
        met = rel <= tol_delta
        rec = {"columns": int(D.shape[1]), "M": int(M), "Lambda": lam, "Lambda_rel": rel,
               "tol_delta": tol_delta, "converged": bool(met), "new_omega": []}
        rounds.append(rec)
        if (stop and met) or r >= max_rounds:
            if log:
                log(f"round {r}: {D.shape[1]} columns, M={M}, Lambda/|B|={rel:.3e} "
                    f"({'met' if met else 'not met'} at TOL {tol_delta:g}); done")
            return D, snap_omega, rounds, {"U": U, "sigma": sig, "M": M, "rom": rom, "out": out}
        new_h = new.cpu().numpy()
        new_h = new_h[np.isfinite(new_h)]
        if new_h.size == 0:  # no interval holds an output frequency
            return D, snap_omega, rounds, {"U": U, "sigma": sig, "M": M, "rom": rom, "out": out}
        rec["new_omega"] = [float(x) for x in new_h]
        if log:
            log(f"round {r}: {D.shape[1]} columns, M={M}, Lambda/|B|={rel:.3e} "
                f"({'met' if met else 'not met'} at TOL {tol_delta:g}); adding {new_h}")
        D = torch.cat([D, solve(new_h)], 1)
        snap_omega = np.concatenate([snap_omega, new_h])
        r += 1
