"""Per-direction bases on the GPU (mpt_project_dirs + mpt_sweep's per-direction
form) against the oracle of the per-direction method (oracle/perdir.py): one
GPU POD basis per direction, the same bases given to the oracle, tensors to
1e-10 of their term scales, certificates to 1e-8 plus their rounding floor,
the per-direction solutions and the defect forms; a two-material sphere in the
32-lane bucket and an ellipsoid in the 64-lane bucket."""
import numpy as np
import pytest

from oracle import perdir as P
from oracle import rom as R
from tests import _cases
from tests._gpu_helpers import delta_floor, tensor_errors, term_scales

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mpt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_05590_amd import mpt as m
    m.lib()
    return m


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _gpu_dirs(mpt, c, cap):
    ops = c.ops
    K = c.snap.size
    Us = []
    for i in range(3):
        U, sig, M = mpt.mpt_pod_basis(_dev(c.D[:, i * K:(i + 1) * K], torch.complex128), 1e-8, cap)
        Us.append(U[:, :M].contiguous())
    rom, Ut = mpt.mpt_project_dirs(
        mpt.Csr.from_scipy(ops.K, row_blocks=3), _dev(ops.c, torch.float64), ops.eps_h,
        _dev(c.w, torch.float64), _dev(c.o, torch.float64), _dev(ops.vol, torch.float64),
        ops.alpha, Us, _dev(ops.cond_idx, torch.int32), _dev(c.Vt, torch.float64),
        _dev(c.lam, torch.float64), _dev(c.s_ref, torch.float64))
    return rom, [u.cpu().numpy() for u in Us]


@pytest.mark.parametrize("case,cap", [("shell16", 6), ("ellipsoid16_k32", 20)])
def test_per_direction_sweep_matches_oracle(mpt, case, cap):
    c = getattr(_cases, case)()
    ops = c.ops
    rom, Us = _gpu_dirs(mpt, c, cap)
    Ms = [u.shape[1] for u in Us]
    assert tuple(rom.dirs) == tuple(Ms) and rom.M == sum(Ms)
    omega = np.logspace(1, 6, 97)
    out, st, a_gpu = mpt.mpt_sweep(rom, _dev(omega, torch.float64), want_a=True)
    torch.cuda.synchronize()
    assert int(st.abs().max()) == 0
    out = out.cpu().numpy()
    a_gpu = a_gpu.cpu().numpy()  # (n, 3, M)
    fo = c.oracle_fo()
    pr = P.project(fo.K, fo.c, fo.eps_h, c.w, Us)
    pr["N0"] = R.static_tensor_mesh(fo, c.o)
    Ut = np.concatenate(Us, 1)
    rt = R.project(fo.K, fo.c, fo.eps_h, c.w, Ut)
    A0t = rt["KM"] + fo.eps_h * rt["UhU"]
    lam, V, dc = c.spec
    cert = P.certificate_data(pr, c.s_ref, lambda s: R.residual_gram_spectral(
        lam, V, dc, ops.cond_idx, c.w, Ut, A0t, s))
    ref, a_o = P.sweep(pr, omega, cert, fo.alpha)
    # solutions: direction i in the slots of U_i, zero elsewhere
    off = np.r_[0, np.cumsum(Ms)]
    for i in range(3):
        ai = a_gpu[:, i, :]
        assert np.abs(np.delete(ai, np.s_[off[i]:off[i + 1]], 1)).max() == 0.0
        err = np.abs(ai[:, off[i]:off[i + 1]] - a_o[i]).max(1) / np.abs(a_o[i]).max(1)
        assert err.max() <= 1e-9, (i, err.max())
    # defect forms: Dp[k][i] is block diagonal with D'_{i<-j}
    Dg = rom.Dp.cpu().numpy()
    for k in range(c.s_ref.size):
        for i in range(3):
            for j in range(3):
                blk = Dg[k, i, off[j]:off[j + 1], off[j]:off[j + 1]]
                refb = cert["Dp"][k][i][j]
                A0s = np.abs(A0t + c.s_ref[k] * rt["CM"]).max()
                assert np.abs(blk - refb).max() <= 1e-8 * A0s, (k, i, j)
    sc = term_scales(ref, omega, pr["N0"], pr["E"], fo.alpha)
    eR, eI = tensor_errors(out[:, :12], ref[:, :12], sc)
    # rounding floor of Delta from the concatenated form (defect magnitudes
    # of all targets together)
    ac = P.concat(a_o)
    cf = {"s_ref": cert["s_ref"], "G": cert["G"],
          "Dp": [sum(np.abs(np.block([[cert["Dp"][k][i][j] if j == jj else
                                         np.zeros((Ms[j], Ms[jj])) for jj in range(3)]
                                        for j in range(3)])) for i in range(3))
                 for k in range(c.s_ref.size)]}
    dp_abs = [1e-8 * np.abs(A0t + s * rt["CM"]).max() for s in cert["s_ref"]]
    fl = delta_floor(cf, ac, omega, fo.alpha, dp_abs=dp_abs)
    d = np.abs(out[:, 12:] - ref[:, 12:])
    print(f"{case} per-direction M={Ms}: R~ {eR.max():.2e} I {eI.max():.2e} "
          f"Delta err/floor {np.max(d / fl):.2e}", flush=True)
    assert eR.max() <= 1e-10 and eI.max() <= 1e-10
    assert np.all(d <= 1e-8 * np.abs(ref[:, 12:]) + fl)


def test_per_direction_rom_rejected_elsewhere(mpt):
    c = _cases.shell16()
    rom, _ = _gpu_dirs(mpt, c, 4)
    w = _dev(np.logspace(1, 6, 8), torch.float64)
    with pytest.raises(mpt.MptError):
        mpt.mpt_sweep_adjoint(rom, w, torch.zeros((8, 18), dtype=torch.float64, device="cuda"))
    with pytest.raises(mpt.MptError):
        mpt.mpt_pencil_reduce(rom)
