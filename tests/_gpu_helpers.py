"""Helpers for GPU parity tests: oracle reduced models and tolerances."""
import numpy as np

from oracle import rom as R

PAIRS = R.PAIRS


def oracle_rom(fo, U, w, o, S, cond):
    """Oracle projection (plain products) in the GPU's Rom layout."""
    r = R.project(fo.K, fo.c, fo.eps_h, w, U)
    r["N0"] = R.static_tensor_mesh(fo, o)
    G = R.residual_gram_schur(S, cond, fo.c, w, U, r["KM"], r["UhU"], fo.eps_h)
    host = {"KM": r["KM"], "A0": r["KM"] + fo.eps_h * r["UhU"], "CM": r["CM"],
            "g": np.ascontiguousarray(r["g"].T), "G": G, "E": r["E"], "N0": r["N0"]}
    return r, G, host


def random_rom(M, seed, alpha=1e-2):
    """A well-conditioned synthetic reduced model with the structure of the real
    ones: A0 Hermitian positive definite, C_M Hermitian PSD, G Hermitian PSD whose
    x-block is A0 and whose (x, c) block is C_M."""
    rng = np.random.default_rng(seed)

    def herm_psd(n, scale, shift=0.0):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        return scale * (X @ X.conj().T) / n + shift * np.eye(n)

    A0 = herm_psd(M, 1.0, 0.5)
    CM = herm_psd(M, 1e-3)
    KM = A0 - 1e-11 * np.eye(M)
    g = (rng.standard_normal((3, M)) + 1j * rng.standard_normal((3, M))) * 1e-3
    Z = rng.standard_normal((4 * M + 8, 2 * M + 3)) + 1j * rng.standard_normal((4 * M + 8, 2 * M + 3))
    G = Z.conj().T @ Z / (4 * M)
    G[3:3 + M, 3:3 + M] = A0
    G[3:3 + M, 3 + M:] = CM
    G[3 + M:, 3:3 + M] = CM.conj().T
    G[3:3 + M, :3] = g.T
    G[:3, 3:3 + M] = g.conj()
    E = np.eye(3) * 2e-3
    N0 = np.diag([1e-7, 2e-7, 3e-7])
    host = {"KM": KM, "A0": A0, "CM": CM, "g": g, "G": G, "E": E, "N0": N0}
    rom = {"KM": KM, "CM": CM, "UhU": (A0 - KM) / 1e-11, "g": g.T, "E": E, "N0": N0,
           "eps_h": 1e-11}
    return rom, G, host, alpha


def delta_floor(G, a, omega, alpha, alpha_lb=1.0):
    """Rounding floor of the G-form certificate: |w|^T |G| |w| per pair, scaled."""
    nw, M, _ = a.shape
    absG = np.abs(G)
    out = np.empty((nw, 6))
    for k in range(nw):
        W = np.zeros((2 * M + 3, 3))
        for i in range(3):
            W[i, i] = omega[k]
        W[3:3 + M, :] = np.abs(a[k])
        W[3 + M:, :] = omega[k] * np.abs(a[k])
        mag = W.T @ absG @ W
        for p, (i, j) in enumerate(PAIRS):
            out[k, p] = alpha ** 3 / (8 * alpha_lb) * (2 * mag[i, i] + 2 * mag[j, j] + 2 * mag[i, j])
    return out


def term_scales(orc, omega, N0, E, alpha):
    """Per-frequency magnitude of the terms each tensor entry is summed from.

    R~ = N0 + R and I = w a^3/4 (E + Re(...)) are differences of larger terms
    where they cross zero (R~) or where the field is expelled at high frequency
    (I -> 0 while E and the quadratic terms stay large); the normwise error of
    an FP64 evaluation is bounded by eps times these magnitudes, so the parity
    tolerance is relative to them: max(|R~|, |N0|, |R~ - N0|) for R~ and
    max(|I|, w a^3/4 |E|) for I."""
    n0 = np.array([N0[i, j] for i, j in PAIRS])
    e = np.array([E[i, j] for i, j in PAIRS])
    sR = np.maximum(np.max(np.abs(orc[:, 0:6]), 1),
                    np.maximum(np.abs(n0).max(), np.max(np.abs(orc[:, 0:6] - n0), 1)))
    sI = np.maximum(np.max(np.abs(orc[:, 6:12]), 1), 0.25 * alpha ** 3 * np.asarray(omega) * np.abs(e).max())
    return sR, sI


def tensor_errors(gpu, orc, scales=None):
    """Normwise per-frequency errors of R~ and I relative to the given scales
    (default: each part's own largest entry)."""
    if scales is None:
        scales = (np.max(np.abs(orc[:, 0:6]), 1), np.max(np.abs(orc[:, 6:12]), 1))
    eR = np.max(np.abs(gpu[:, 0:6] - orc[:, 0:6]), 1) / scales[0]
    eI = np.max(np.abs(gpu[:, 6:12] - orc[:, 6:12]), 1) / scales[1]
    return eR, eI
