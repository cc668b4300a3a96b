"""Control flow of the adaptive loop (Algorithm 1, Section 4.4) with stand-ins
for the device calls: the stopping rule Lambda / |B_alpha| <= TOL_Delta, the
round cap, and the end when no interval holds an output frequency."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


class _Fake:
    """Stand-ins for the library calls: the certificate maximum of round r is
    lambdas[r]; the selection returns the given frequencies."""

    def __init__(self, lambdas, picks):
        self.lambdas, self.picks, self.r = list(lambdas), picks, 0

    def pod(self, D, tol, cap):
        return torch.zeros(D.shape[0], 1, dtype=torch.complex128), torch.ones(1), min(cap, D.shape[1])

    def sweep(self, rom, omega):
        return torch.zeros(omega.numel(), 18, dtype=torch.float64), torch.zeros(omega.numel(),
                                                                                 dtype=torch.int32)

    def select(self, omega, out, snap, n_star):
        lam = self.lambdas[self.r]
        pick = self.picks[self.r] if self.r < len(self.picks) else [np.nan] * n_star
        self.r += 1
        return (torch.tensor(pick, dtype=torch.float64), torch.zeros(snap.numel() - 1),
                torch.tensor([lam], dtype=torch.float64))


@pytest.fixture
def loop(monkeypatch):
    from paper_2307_05590_amd import adaptive, mpt

    def make(lambdas, picks):
        f = _Fake(lambdas, picks)
        monkeypatch.setattr(mpt, "mpt_pod_basis", f.pod)
        monkeypatch.setattr(mpt, "mpt_sweep", f.sweep)
        monkeypatch.setattr(mpt, "mpt_select_snapshots", f.select)
        return adaptive.adaptive_pod
    return make


def _run(run, stop, max_rounds, volume=2.0, tol=1e-3):
    added = []

    def solve(new):
        added.append(list(new))
        return torch.ones(4, 3 * len(new), dtype=torch.complex128)

    D = torch.ones(4, 6, dtype=torch.complex128)
    omega = torch.linspace(1, 100, 50, dtype=torch.float64)
    return run(D, np.array([1.0, 100.0]), omega, solve, lambda U: None, tol_sigma=1e-8, m_cap=8,
               n_star=2, volume=volume, tol_delta=tol, max_rounds=max_rounds, stop=stop,
               sweep="lu"), added


def test_stops_when_the_rule_is_met(loop):
    run = loop([1.0, 0.1, 1e-3, 1e-4], [[10.0, 20.0], [30.0, 40.0], [50.0, 60.0]])
    (D, snap, rounds, _), added = _run(run, stop=True, max_rounds=10)
    # Lambda / |B| = 0.5, 0.05, 5e-4 <= 1e-3: two enrichments, then stop
    assert [r["converged"] for r in rounds] == [False, False, True]
    assert added == [[10.0, 20.0], [30.0, 40.0]]
    assert D.shape[1] == 6 + 12 and sorted(snap) == [1.0, 10.0, 20.0, 30.0, 40.0, 100.0]
    assert rounds[0]["Lambda_rel"] == pytest.approx(0.5)
    assert rounds[-1]["new_omega"] == []


def test_fixed_rounds_ignore_the_rule(loop):
    run = loop([1e-5, 1e-5, 1e-5], [[10.0, 20.0], [30.0, 40.0]])
    (D, snap, rounds, _), added = _run(run, stop=False, max_rounds=2)
    assert len(rounds) == 3 and all(r["converged"] for r in rounds)
    assert len(added) == 2 and D.shape[1] == 18


def test_ends_when_no_interval_has_an_output_frequency(loop):
    run = loop([1.0, 1.0], [[np.nan, np.nan]])
    (D, snap, rounds, _), added = _run(run, stop=True, max_rounds=5)
    assert added == [] and len(rounds) == 1 and D.shape[1] == 6
