"""Helpers for GPU parity tests: oracle reduced models and tolerances."""
import numpy as np

from oracle import rom as R

PAIRS = R.PAIRS


def oracle_rom(fo, U, w, o, spec, cond, s_ref):
    """Oracle projection (plain products) and certificate data (residual Grams
    from the conductor block's eigenpairs spec = (lam, V, sqrt(c)), defect
    forms) in the GPU's Rom layout.  Returns (rom dict, cert dict, host dict)."""
    r = R.project(fo.K, fo.c, fo.eps_h, w, U)
    r["N0"] = R.static_tensor_mesh(fo, o)
    A0 = r["KM"] + fo.eps_h * r["UhU"]
    lam, V, dc = spec
    cert = R.certificate_data(r, s_ref, lambda s: R.residual_gram_spectral(
        lam, V, dc, cond, w, U, A0, s))
    host = {"KM": r["KM"], "A0": A0, "CM": r["CM"], "g": np.ascontiguousarray(r["g"].T),
            "G": np.stack(cert["G"]), "Dp": np.stack(cert["Dp"]), "s_ref": cert["s_ref"],
            "E": r["E"], "N0": r["N0"]}
    return r, cert, host


def random_rom(M, seed, alpha=1e-2):
    """A well-conditioned synthetic reduced model with the structure the
    kernels rely on: A0 Hermitian positive definite, C_M Hermitian PSD, three
    reference shifts, each with a Hermitian PSD residual Gram whose
    [X U, C U] block is Hermitian and a Hermitian PSD defect form."""
    rng = np.random.default_rng(seed)

    def herm_psd(n, scale, shift=0.0):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        return scale * (X @ X.conj().T) / n + shift * np.eye(n)

    A0 = herm_psd(M, 1.0, 0.5)
    CM = herm_psd(M, 1e-3)
    KM = A0 - 1e-11 * np.eye(M)
    g = (rng.standard_normal((3, M)) + 1j * rng.standard_normal((3, M))) * 1e-3
    s_ref = np.array([0.0, 1e3, 1e5])
    Gs, Dps = [], []
    for k in range(s_ref.size):
        Z = (rng.standard_normal((4 * M + 8, 2 * M + 3)) +
             1j * rng.standard_normal((4 * M + 8, 2 * M + 3)))
        G = Z.conj().T @ Z / (4 * M) / (1.0 + s_ref[k] * 1e-3)
        Hxc = herm_psd(M, 1e-3)
        G[3:3 + M, 3 + M:] = Hxc
        G[3 + M:, 3:3 + M] = Hxc
        Gs.append(G)
        Dps.append(herm_psd(M, 1e-6))
    E = np.eye(3) * 2e-3
    N0 = np.diag([1e-7, 2e-7, 3e-7])
    host = {"KM": KM, "A0": A0, "CM": CM, "g": g, "G": np.stack(Gs), "Dp": np.stack(Dps),
            "s_ref": s_ref, "E": E, "N0": N0}
    rom = {"KM": KM, "CM": CM, "UhU": (A0 - KM) / 1e-11, "g": g.T, "E": E, "N0": N0,
           "eps_h": 1e-11}
    cert = {"s_ref": s_ref, "G": Gs, "Dp": Dps}
    return rom, cert, host, alpha


def delta_floor(cert, a, omega, alpha, alpha_lb=R.ALPHA_LB, dp_abs=None):
    """Rounding floor of the G-form certificate per frequency and pair: the
    quadratic part from |w|^T |G_s| |w|, and the linear part from the
    resulting uncertainty of n = sqrt(n^2) and e = sqrt(a^H D' a).  dp_abs
    (per shift): an absolute uncertainty of the entries of D'_s when the two
    sides formed it separately."""
    nw, M, _ = a.shape
    ks = R.ref_index(cert["s_ref"], omega)
    eps = 2.2e-16
    out = np.empty((nw, 6))
    a3 = alpha ** 3
    for k in range(nw):
        G, Dp = cert["G"][ks[k]], cert["Dp"][ks[k]]
        W = np.zeros((2 * M + 3, 3))
        for i in range(3):
            W[i, i] = omega[k]
        W[3:3 + M, :] = np.abs(a[k])
        W[3 + M:, :] = omega[k] * np.abs(a[k])
        mag = W.T @ np.abs(G) @ W
        Wc = np.zeros((2 * M + 3, 3), complex)
        for i in range(3):
            Wc[i, i] = 1j * omega[k]
        Wc[3:3 + M, :] = -a[k]
        Wc[3 + M:, :] = 1j * omega[k] * a[k]
        n2 = np.maximum(np.real(np.einsum("mi,mn,ni->i", Wc.conj(), G, Wc)), 0.0)
        e2 = np.maximum(np.real(np.einsum("mi,mn,ni->i", a[k].conj(), Dp, a[k])), 0.0)
        dn2 = 64 * eps * np.diag(mag)
        de2 = 64 * eps * np.einsum("mi,mn,ni->i", np.abs(a[k]), np.abs(Dp), np.abs(a[k]))
        if dp_abs is not None:
            de2 = de2 + dp_abs[ks[k]] * np.sum(np.abs(a[k]), axis=0) ** 2
        dn = np.minimum(np.sqrt(dn2), dn2 / (2 * np.sqrt(np.maximum(n2, 1e-300))))
        de = np.minimum(np.sqrt(de2), de2 / (2 * np.sqrt(np.maximum(e2, 1e-300))))
        n, e = np.sqrt(n2), np.sqrt(e2)
        for p, (i, j) in enumerate(PAIRS):
            quad = a3 / (8 * alpha_lb) * 64 * eps * (2 * mag[i, i] + 2 * mag[j, j] + 2 * mag[i, j])
            lin = 0.25 * a3 * ((n[i] + dn[i]) * de[j] + dn[i] * e[j] +
                               (n[j] + dn[j]) * de[i] + dn[j] * e[i])
            out[k, p] = quad + lin
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
