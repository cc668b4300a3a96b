"""The allocation-free selection entry point (static device scratch) against
the workspace entry point, through the C ABI: two calls in a row, the second
with a smaller input, and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mpt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_05590_amd import mpt as m
    m.lib()
    return m


def _case(seed, n, n_snap):
    rng = np.random.default_rng(seed)
    om = np.sort(rng.uniform(10.0, 1e6, n))
    out = np.zeros((n, 18))
    out[:, 12:] = rng.integers(0, 50, (n, 6)).astype(float)  # many ties
    snaps = np.sort(np.r_[rng.choice(om, n_snap - 2, replace=False), 5.0, 2e6])
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    return dev(om), dev(out), dev(snaps)


def test_static_selection_equals_workspace_selection(mpt):
    # first call: 3000 snapshot frequencies; second call: a smaller input
    for seed, n, n_snap, n_star in ((1, 200_000, 3000, 7), (2, 5_000, 40, 2)):
        om, out, snaps = _case(seed, n, n_snap)
        ref = mpt.mpt_select_snapshots(om, out, snaps, n_star)
        got = mpt.mpt_select_snapshots_static(om, out, snaps, n_star)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b) or (torch.isnan(a).equal(torch.isnan(b)) and
                                         torch.equal(a[~torch.isnan(a)], b[~torch.isnan(b)]))
    # beyond the static array's size: rejected on the host
    om, out, snaps = _case(3, 10_000, 10)
    big = torch.linspace(1.0, 2e6, 4097, dtype=torch.float64, device="cuda")
    with pytest.raises(mpt.MptError):
        mpt.mpt_select_snapshots_static(om, out, big, 2)
