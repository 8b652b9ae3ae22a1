"""Exact expectations of the binned multipoles for the synthetic lattice
catalogs (shared by the oracle's and the GPU path's physics tests)."""
import numpy as np

from oracle import mesh as M, special as S
from synth import power_spectrum


def _expected_lattice(cfg, s2, amp, nhat):
    """Exact expectation of each binned multipole for the lattice catalogs of
    synth.lattice_catalogs at a distant observer along nhat: per mode,
    E|delta(k)|^2 = s^2 P(k) N^3/H^3; gamma(k) e^{-2 i phi} = -(A/2)(1-mu^2) delta(k)
    (Sec. IV.A eq. power_for_validation) summed over the discrete shell."""
    n = cfg.mesh
    kf = 2 * np.pi / cfg.box
    m = M.signed_modes(n).astype(float)
    kx, ky, kz = np.meshgrid(m, m, m, indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    mu = np.where(kk > 0, (kx * nhat[0] + ky * nhat[1] + kz * nhat[2]) / np.where(kk > 0, kk, 1), 0)
    P = np.where(kk > 0, s2 * power_spectrum(kk * kf), 0.0)
    num, den = cfg.bin_width()
    b = M.bin_index(n, cfg.n_kbins, num, den)
    sel = b >= 0
    cnt = np.bincount(b[sel], minlength=cfg.n_kbins).astype(float)

    def avg(f):
        return np.bincount(b[sel], weights=f[sel], minlength=cfg.n_kbins) / np.maximum(cnt, 1)

    lp = lambda l: S.peval(S.legendre(l), mu)
    out = {
        "DD_l0": avg(P), "DD_l2": 5 * avg(lp(2) * P), "DD_l4": 9 * avg(lp(4) * P),
        "GD_L2": float(S.prefactor(2, 2)) * avg(S.assoc_legendre(2, 2, mu) * (-amp / 2) * (1 - mu ** 2) * P),
        "GD_L4": float(S.prefactor(2, 4)) * avg(S.assoc_legendre(2, 4, mu) * (-amp / 2) * (1 - mu ** 2) * P),
    }
    pp = amp ** 2 / 4 * (1 - mu ** 2) ** 2 * P
    for l in (0, 2, 4):
        out[f"PLUS_l{l}"] = (2 * l + 1) * avg(lp(l) * pp)
    out["MINUS_L4"] = float(S.prefactor(4, 4)) * avg(S.assoc_legendre(4, 4, mu) * pp)
    return out
