"""Algorithm 1's rounds on the GPU against the oracle, round by round.

The 16^3 two-material sphere (magnetic core mu_r 50, sigma 6e6, in a shell
sigma 3.5e7) with 4 initial snapshots on [1e1, 1e6] and M <= 12: the
certificates start well above TOL_Delta (Lambda / |B_alpha| ~ 1e-2), so the
rounds make real enrichments.  Each round's basis rank M must equal the
oracle's POD on the same snapshot matrix; the oracle's reduced model on the
GPU's basis gives the certificates (G-form, the same conductor eigenpairs),
its Lambda must match the GPU's to 1e-8 plus the certificate's rounding
floor, and the selected frequencies must be the oracle's (or, at a near
tie, attain the oracle's Lambda_n within that floor)."""
import numpy as np
import pytest

from oracle import rom as R
from tests._gpu_helpers import delta_floor, oracle_rom

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_adaptive_rounds_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_05590_amd import mpt
    from paper_2307_05590_amd.adaptive import adaptive_pod
    from synth.shapes import shell_sphere
    from tests._cases import Case

    mpt.lib()
    c = Case(16, shell_sphere(1.2, 2.0, (6e6, 50.0), (3.5e7, 1.0)), np.logspace(1, 6, 4))
    ops = c.ops
    dev = "cuda"
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    K = mpt.Csr.from_scipy(ops.K, row_blocks=3)
    args = (T(ops.c, torch.float64), ops.eps_h, T(c.w, torch.float64), T(c.o, torch.float64),
            T(ops.vol, torch.float64), ops.alpha)
    cert_in = (T(c.Vt, torch.float64), T(c.lam, torch.float64), T(c.s_ref, torch.float64))
    cond = T(ops.cond_idx, torch.int32)
    bases, Ds = [], [c.D.copy()]
    tol, cap = 1e-8, 12

    def project(U):
        bases.append(U.cpu().numpy())
        return mpt.mpt_project(K, *args, U, cond, *cert_in)

    def solve(new):
        Q, hist = c.fs.snapshots(np.asarray(new), c.w, tol=1e-12, max_iter=12)
        assert hist[-1] <= 1e-12
        Ds.append(np.concatenate([Ds[-1], Q], 1))
        return T(Q, torch.complex128)

    omega = np.logspace(1, 6, 300)
    snap0 = c.snap.copy()
    _, snaps, rounds, last = adaptive_pod(
        T(c.D, torch.complex128), snap0, T(omega, torch.float64), solve, project,
        tol_sigma=tol, m_cap=cap, n_star=2, volume=ops.volume, tol_delta=1e-3,
        max_rounds=2, stop=True, sweep="lu")
    assert len(rounds) == len(bases) and rounds[0]["Lambda_rel"] > 1e-3
    fo = c.oracle_fo()
    spec = c.spec
    snap_set = np.sort(snap0)
    for r, rec in enumerate(rounds):
        _, _, M_o = R.pod_basis(Ds[r], tol, cap)
        assert rec["M"] == M_o, f"round {r}: M {rec['M']} vs oracle {M_o}"
        U = bases[r][:, :rec["M"]]
        rom_o, cert, _ = oracle_rom(fo, U, c.w, c.o, spec, ops.cond_idx, c.s_ref)
        ref, a = R.sweep(rom_o, omega, cert, ops.alpha)
        A0 = rom_o["KM"] + rom_o["eps_h"] * rom_o["UhU"]
        dp_abs = [1e-8 * np.abs(A0 + s * rom_o["CM"]).max() for s in cert["s_ref"]]
        fl = delta_floor(cert, a, omega, ops.alpha, dp_abs=dp_abs).max(1)
        new_o, Lam_o, lam_n = R.select_snapshots(omega, ref[:, 12:], snap_set, 2)
        print(f"round {r}: M={rec['M']} Lambda gpu {rec['Lambda']:.6e} oracle {Lam_o:.6e} "
              f"rel {rec['Lambda_rel']:.3e} new gpu {rec['new_omega']} oracle {list(new_o)}",
              flush=True)
        assert abs(rec["Lambda"] - Lam_o) <= 1e-8 * Lam_o + fl.max(), f"round {r}"
        assert rec["Lambda_rel"] == pytest.approx(rec["Lambda"] / ops.volume, rel=1e-15)
        assert rec["converged"] == (rec["Lambda"] / ops.volume <= 1e-3)
        if rec["new_omega"]:
            got = np.sort(rec["new_omega"])
            if not np.array_equal(got, np.sort(new_o)):
                # a near tie: each GPU choice attains its interval's oracle
                # Lambda_n within the rounding floor there
                dmax = ref[:, 12:].max(1)
                for x in got:
                    k = int(np.flatnonzero(omega == x)[0])
                    n = int(np.searchsorted(snap_set, x)) - 1
                    assert dmax[k] >= lam_n[n] - 2 * fl[k], f"round {r}: {x}"
            snap_set = np.sort(np.concatenate([snap_set, rec["new_omega"]]))
    assert np.allclose(np.sort(snaps), snap_set)
