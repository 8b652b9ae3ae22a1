"""Seeded synthetic inputs for the LPP projected-tensor power-spectrum estimator.

This module only *makes inputs*: Gaussian random fields, their tidal tensor,
survey-like footprints, galaxy and random catalogs and their shapes.  It holds
none of the estimator's arithmetic and is imported by both the CPU oracle tests
and the GPU path's tests and benchmark, so that both sides see identical inputs.

Conventions (used by every consumer):
  * positions are Cartesian comoving coordinates in Mpc/h with the observer at
    ``observer`` (default the origin);
  * a catalog is a :class:`Catalog` of float64 structure-of-arrays;
  * shapes (g1, g2) are the components of the projected tensor in the
    (e_theta, e_phi) basis of each object's own line of sight, gamma = g1 + i g2
    (Sec. II.B, eq. gamma_def);
  * seeds: ``numpy.random.SeedSequence([2202, 11839, config_id, mock, stream])``.

Workload recipes (the paper's BOSS-like setup, Sec. IV.A, scaled to synthetic
sizes) are listed in :data:`WORKLOADS`.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np

try:  # scipy's FFT is multi-threaded; numpy's is the fallback
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None

__all__ = [
    "Catalog", "WORKLOADS", "power_spectrum", "seed_seq", "grf", "tidal_at",
    "wedge_uniform", "box_uniform", "make_catalogs", "los_basis_synth",
    "pure_noise_catalogs", "lattice_catalogs",
]

STREAM_GRF, STREAM_POS, STREAM_NOISE, STREAM_RAN = 0, 1, 2, 3


@dataclasses.dataclass
class Catalog:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    w: np.ndarray
    nbar: np.ndarray
    g1: Optional[np.ndarray] = None
    g2: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def take(self, idx) -> "Catalog":
        f = lambda a: None if a is None else np.ascontiguousarray(a[idx])
        return Catalog(f(self.x), f(self.y), f(self.z), f(self.w), f(self.nbar),
                       f(self.g1), f(self.g2))


def power_spectrum(k):
    """Analytic linear spectrum P(k) = 2e4 (k/0.02) / (1+(k/0.02)^2)^1.4 (Mpc/h)^3."""
    q = np.asarray(k, dtype=np.float64) / 0.02
    return 2.0e4 * q / (1.0 + q * q) ** 1.4


def seed_seq(config_id: int, mock: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2202, 11839, int(config_id), int(mock), int(stream)]))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rfftn(a):
    if _sfft is not None:
        return _sfft.rfftn(a, workers=_workers())
    return np.fft.rfftn(a)


def _irfftn(a, s):
    if _sfft is not None:
        return _sfft.irfftn(a, s=s, workers=_workers())
    return np.fft.irfftn(a, s=s)


def _kgrid_r(n: int, box: float):
    kf = 2.0 * math.pi / box
    kx = np.fft.fftfreq(n, d=1.0 / n) * kf
    kz = np.fft.rfftfreq(n, d=1.0 / n) * kf
    return kx, kz


def grf(n: int, box: float, rng: np.random.Generator, amplitude: float = 1.0,
        pk=power_spectrum) -> np.ndarray:
    """Real Gaussian random field on an n^3 mesh (index order [ix, iy, iz]).

    Its discrete Fourier modes obey E|FFT(delta)|^2 = n^3 P(k) / H^3 with
    H = box/n, i.e. the continuum spectrum P(k) (zero DC mode)."""
    white = rng.standard_normal((n, n, n))
    wk = _rfftn(white)
    del white
    kx, kz = _kgrid_r(n, box)
    h3 = (box / n) ** 3
    kk = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = np.sqrt(pk(kk[nz]) / h3) * amplitude
    wk *= amp
    del amp, kk
    return _irfftn(wk, (n, n, n))


def tidal_at(delta: np.ndarray, box: float, idx: np.ndarray) -> np.ndarray:
    """Tidal tensor T_ij = (k_i k_j / k^2 - delta_ij/3) delta (Sec. IV.A) sampled
    at mesh cells ``idx`` (shape (n_obj, 3) integer); returns (n_obj, 3, 3)."""
    n = delta.shape[0]
    dk = _rfftn(delta)
    kx, kz = _kgrid_r(n, box)
    comps = [kx[:, None, None], kx[None, :, None], kz[None, None, :]]
    k2 = comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2
    k2 = np.where(k2 == 0, 1.0, k2)
    out = np.zeros((idx.shape[0], 3, 3))
    for i in range(3):
        for j in range(i, 3):
            f = comps[i] * comps[j] / k2
            if i == j:
                f = f - 1.0 / 3.0
            tij = _irfftn(dk * f, (n, n, n))
            v = tij[idx[:, 0], idx[:, 1], idx[:, 2]]
            out[:, i, j] = v
            out[:, j, i] = v
            del tij
    return out


def los_basis_synth(pos: np.ndarray, observer):
    """Unit vectors (xhat, e_theta, e_phi) of each object's own line of sight.
    e_theta, e_phi are the first two columns of the standard rotation S(xhat)
    (App. E, eq. def_standard_rotation); at the poles phi is taken as 0."""
    r = pos - np.asarray(observer, dtype=np.float64)[None, :]
    rn = np.linalg.norm(r, axis=1)
    xh = r / rn[:, None]
    ct = np.clip(xh[:, 2], -1.0, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    rho = np.hypot(xh[:, 0], xh[:, 1])
    cp = np.where(rho > 0, xh[:, 0] / np.where(rho > 0, rho, 1.0), 1.0)
    sp = np.where(rho > 0, xh[:, 1] / np.where(rho > 0, rho, 1.0), 0.0)
    et = np.stack([ct * cp, ct * sp, -st], axis=1)
    ep = np.stack([-sp, cp, np.zeros_like(cp)], axis=1)
    return xh, et, ep


def project_shapes(tij: np.ndarray, pos: np.ndarray, observer) -> tuple:
    """gamma = e_ij(xhat) T_ij with e_ij = e+_i e+_j, e+ = (e_theta + i e_phi)/sqrt2
    (Sec. II.B, eqs. gamma_def, def_of_eij_+2): g1 = (T_tt - T_pp)/2, g2 = T_tp."""
    _, et, ep = los_basis_synth(pos, observer)
    ttt = np.einsum("ni,nij,nj->n", et, tij, et)
    tpp = np.einsum("ni,nij,nj->n", ep, tij, ep)
    ttp = np.einsum("ni,nij,nj->n", et, tij, ep)
    return 0.5 * (ttt - tpp), ttp


# ---------------------------------------------------------------------------
# footprints

def wedge_volume(ra, dec, r):
    dra = math.radians(ra[1] - ra[0])
    return dra * (math.sin(math.radians(dec[1])) - math.sin(math.radians(dec[0]))) * (r[1] ** 3 - r[0] ** 3) / 3.0


def wedge_uniform(n: int, rng, ra, dec, r) -> np.ndarray:
    """Uniform points in the wedge RA in ra, Dec in dec (degrees), distance in r."""
    u = rng.random((n, 3))
    rr = (r[0] ** 3 + u[:, 0] * (r[1] ** 3 - r[0] ** 3)) ** (1.0 / 3.0)
    s0, s1 = math.sin(math.radians(dec[0])), math.sin(math.radians(dec[1]))
    sd = s0 + u[:, 1] * (s1 - s0)
    cd = np.sqrt(1.0 - sd * sd)
    a = np.radians(ra[0] + u[:, 2] * (ra[1] - ra[0]))
    return np.stack([rr * cd * np.cos(a), rr * cd * np.sin(a), rr * sd], axis=1)


def box_uniform(n: int, rng, origin, box) -> np.ndarray:
    return np.asarray(origin, dtype=np.float64)[None, :] + rng.random((n, 3)) * box


# ---------------------------------------------------------------------------
# workload recipes

def _c1_origin():
    c = 1000.0 / math.sqrt(3.0)
    return (c - 200.0, c - 200.0, c - 200.0)


WORKLOADS = {
    # plain FP64 estimator: 32^3, cubic box of side 400 centred 1000 from the observer
    "c1": dict(config_id=1, mesh=32, box=400.0, origin=_c1_origin(), observer=(0.0, 0.0, 0.0),
               geometry="box", n_gal=5000, n_ran=50000, amp=0.01, sigma=0.2, assignment=2,
               interlacing=0, n_kbins=16, lmax=4, precision="f64"),
    # headline single mock: 512^3, wedge RA 0-90, Dec 0-40, r 1000-1600
    "c2": dict(config_id=2, mesh=512, box=1700.0, origin=(-50.0, -50.0, -50.0), observer=(0.0, 0.0, 0.0),
               geometry="wedge", ra=(0.0, 90.0), dec=(0.0, 40.0), r=(1000.0, 1600.0),
               n_gal=1_500_000, n_ran=15_000_000, amp=0.01, sigma=0.2, assignment=3,
               interlacing=1, n_kbins=50, lmax=4, precision="f32"),
    # batched mocks: 64 catalogs at 256^3 on the same wedge
    "c3": dict(config_id=3, mesh=256, box=1700.0, origin=(-50.0, -50.0, -50.0), observer=(0.0, 0.0, 0.0),
               geometry="wedge", ra=(0.0, 90.0), dec=(0.0, 40.0), r=(1000.0, 1600.0),
               n_gal=None, n_ran=None, n_mocks=64, amp=0.01, sigma=0.2, assignment=3,
               interlacing=1, n_kbins=50, lmax=4, precision="f32"),
    # large single mock: 1024^3, 1000-1800 shell
    "c4": dict(config_id=4, mesh=1024, box=1900.0, origin=(-50.0, -50.0, -50.0), observer=(0.0, 0.0, 0.0),
               geometry="wedge", ra=(0.0, 90.0), dec=(0.0, 40.0), r=(1000.0, 1800.0),
               n_gal=10_000_000, n_ran=50_000_000, amp=0.01, sigma=0.2, assignment=3,
               interlacing=1, n_kbins=80, lmax=4, precision="f32"),
}


def c3_sizes(n_mocks: int = 64):
    """Uneven batch sizes N_i = round(0.2e6 * 10^(i/63)), i = 0..63 (0.2M-2M)."""
    return [int(round(0.2e6 * 10 ** (i / 63.0))) for i in range(n_mocks)]


def make_catalogs(wl: dict, mock: int = 0, n_gal: Optional[int] = None, n_ran: Optional[int] = None,
                  grf_mesh: Optional[int] = None, amp: Optional[float] = None,
                  sigma: Optional[float] = None, observer=None):
    """Galaxy + random catalogs for a workload recipe.

    Galaxies are drawn by rejection from uniform footprint points with
    acceptance proportional to max(0, 1+delta_NGP) of a seeded GRF on a
    ``grf_mesh``^3 mesh covering the box; shapes are -amp * e_ij(xhat) T_ij at
    the galaxy's cell plus Gaussian noise ``sigma`` per component; randoms are
    uniform in the same footprint; nbar = n_gal / V_footprint for all objects,
    weights are 1.
    """
    cid = wl["config_id"]
    n = wl["mesh"] if grf_mesh is None else grf_mesh
    box = wl["box"]
    origin = np.asarray(wl["origin"], dtype=np.float64)
    obs = np.asarray(wl["observer"] if observer is None else observer, dtype=np.float64)
    ng = wl["n_gal"] if n_gal is None else n_gal
    nr = wl["n_ran"] if n_ran is None else n_ran
    A = wl["amp"] if amp is None else amp
    sig = wl["sigma"] if sigma is None else sigma

    delta = grf(n, box, seed_seq(cid, mock, STREAM_GRF))
    prng = seed_seq(cid, mock, STREAM_POS)
    if wl["geometry"] == "box":
        sampler = lambda m: box_uniform(m, prng, origin, box)
        vol = box ** 3
    else:
        sampler = lambda m: wedge_uniform(m, prng, wl["ra"], wl["dec"], wl["r"]) + (obs - 0.0)
        vol = wedge_volume(wl["ra"], wl["dec"], wl["r"])
    cap = float(1.0 + delta.max())
    h = box / n
    chunks, got = [], 0
    while got < ng:
        m = max(1024, int(1.3 * (ng - got) * cap))
        p = sampler(m)
        idx = np.floor((p - origin[None, :]) / h).astype(np.int64)
        np.clip(idx, 0, n - 1, out=idx)
        acc = np.maximum(0.0, 1.0 + delta[idx[:, 0], idx[:, 1], idx[:, 2]]) / cap
        keep = prng.random(m) < acc
        chunks.append(p[keep])
        got += int(keep.sum())
    gpos = np.concatenate(chunks, axis=0)[:ng]
    del chunks
    gidx = np.clip(np.floor((gpos - origin[None, :]) / h).astype(np.int64), 0, n - 1)
    tij = tidal_at(delta, box, gidx)
    del delta
    g1, g2 = project_shapes(tij, gpos, obs)
    nrng = seed_seq(cid, mock, STREAM_NOISE)
    g1 = -A * g1 + sig * nrng.standard_normal(ng)
    g2 = -A * g2 + sig * nrng.standard_normal(ng)
    rrng = seed_seq(cid, mock, STREAM_RAN)
    if wl["geometry"] == "box":
        rpos = box_uniform(nr, rrng, origin, box)
    else:
        rpos = wedge_uniform(nr, rrng, wl["ra"], wl["dec"], wl["r"]) + obs
    nbar = ng / vol
    gal = Catalog(gpos[:, 0].copy(), gpos[:, 1].copy(), gpos[:, 2].copy(), np.ones(ng),
                  np.full(ng, nbar), g1, g2)
    ran = Catalog(rpos[:, 0].copy(), rpos[:, 1].copy(), rpos[:, 2].copy(), np.ones(nr),
                  np.full(nr, nbar))
    return gal, ran


def pure_noise_catalogs(n_gal, n_ran, origin, box, sigma, seed):
    """Uniform positions in a cube, pure Gaussian shape noise, no clustering."""
    rng = np.random.default_rng(np.random.SeedSequence([2202, 11839, 90, seed, 0]))
    gp = box_uniform(n_gal, rng, origin, box)
    rp = box_uniform(n_ran, rng, origin, box)
    nbar = n_gal / box ** 3
    gal = Catalog(gp[:, 0].copy(), gp[:, 1].copy(), gp[:, 2].copy(), np.ones(n_gal), np.full(n_gal, nbar),
                  sigma * rng.standard_normal(n_gal), sigma * rng.standard_normal(n_gal))
    ran = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), np.ones(n_ran), np.full(n_ran, nbar))
    return gal, ran


def lattice_catalogs(n, box, origin, observer, seed, delta_rms=0.1, amp=1.0):
    """Field-level catalogs: one galaxy and one random at every cell node.

    Galaxy weights are 1 + delta (a GRF scaled to rms ``delta_rms``), galaxy
    shapes are gamma = -amp e_ij T_ij / (1 + delta), so that with nearest-grid-
    point assignment the deposited density is delta - <delta> and the deposited
    shape field is -amp e_ij(xhat) T_ij exactly (the paper's grid-level
    validation fields, Sec. IV.A).  Returns (gal, ran, scale) where the input
    spectrum of delta is scale^2 P(k)."""
    rng = seed_seq(70, seed, STREAM_GRF)
    delta = grf(n, box, rng)
    s = delta_rms / float(delta.std())
    delta *= s
    h = box / n
    ii = np.arange(n)
    gx, gy, gz = np.meshgrid(ii, ii, ii, indexing="ij")
    idx = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    pos = np.asarray(origin, dtype=np.float64)[None, :] + idx * h
    tij = tidal_at(delta, box, idx)
    g1, g2 = project_shapes(tij, pos, observer)
    d = delta.ravel()
    w = 1.0 + d
    g1 = -amp * g1 / w
    g2 = -amp * g2 / w
    nbar = np.full(n ** 3, 1.0 / h ** 3)
    gal = Catalog(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), w, nbar.copy(), g1, g2)
    ran = Catalog(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.ones(n ** 3), nbar)
    return gal, ran, s


# ---------------------------------------------------------------------------
# emulator training design

EMU_RANGES = ((0.0, 0.05), (1.0, 3.0), (0.5, 1.0), (0.6, 1.0), (0.5, 2.0))  # A, b, f, sigma8, s_N


def latin_hypercube(n: int, ranges=EMU_RANGES, seed: int = 0) -> np.ndarray:
    """Seeded Latin hypercube of n points over the box `ranges` (one stratum
    per point and axis, strata shuffled independently per axis)."""
    rng = seed_seq(5, seed, 0)
    d = len(ranges)
    u = (rng.permuted(np.tile(np.arange(n), (d, 1)), axis=1).T + rng.random((n, d))) / n
    lo = np.array([r[0] for r in ranges])
    hi = np.array([r[1] for r in ranges])
    return lo + u * (hi - lo)
