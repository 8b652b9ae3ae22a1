"""Pins of oracle functions that the other oracle tests only use or restate.

Each pin checks the oracle against something fixed outside it: an
expectation value that holds for any catalog of a known kind, scipy's
quadrature and special functions, exact rational arithmetic, or an identity
of the mass-assignment kernels.

* shot_dd (the density shot noise (sum w_g^2 + alpha^2 sum w_r^2)/I, a
  reading of the normalisation of Sec. III.A): for Poisson catalogs with
  nearest-grid-point assignment the expected shell power is exactly the
  self-pair term, so DD_l0 after subtraction averages to zero and every
  DD_l averages to its self-pair sum.
* EE/BB rows (eq. relation_pm_EB with the truncated m=4 series): a linear
  tidal field is pure E (BB ~ 0, EE = P_+), and the same shapes turned by
  45 degrees (gamma -> i gamma) are pure B.
* gd_moments (the m=2 moments of the cross spectrum of the emulator model):
  quadrature with scipy's associated Legendre functions.
* sigma8 (top-hat rms of the linear spectrum): scipy quadrature.
* r_thresholds and the window multipoles' shell counts: exact rational
  comparison of every mesh separation with the shell edges.
* compensation: averaged over an object's offset inside a cell, the
  assignment stencil's phase equals the Fourier transform of the assignment
  window, prod_i sinc(pi n_i / N)^p.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import eval_legendre, lpmv

from oracle import estimator as E, mesh as M, window as W
from synth import Catalog, box_uniform, lattice_catalogs


# ---------------------------------------------------------------------------
# density shot noise


def _poisson_pair(seed, ng, nr, origin, box):
    rng = np.random.default_rng(np.random.SeedSequence([2202, 11839, 91, seed]))
    gp = box_uniform(ng, rng, origin, box)
    rp = box_uniform(nr, rng, origin, box)
    g = Catalog(gp[:, 0], gp[:, 1], gp[:, 2], 0.5 + rng.random(ng), np.full(ng, 1e-3),
                np.zeros(ng), np.zeros(ng))
    r = Catalog(rp[:, 0], rp[:, 1], rp[:, 2], 0.5 + rng.random(nr), np.full(nr, 1e-3))
    return g, r


def _self_pair_sums(cfg, g, r, alpha, norm):
    """(2l+1)/(I N_b) sum_{k in b} [sum_g w^2 L_l(khat.xhat) + alpha^2 sum_r w^2 L_l(khat.xhat)],
    evaluated directly from the catalog (numpy Legendre of scipy)."""
    n = cfg.mesh
    m = np.fft.fftfreq(n, 1.0 / n)
    kx, ky, kz = np.meshgrid(m, m, m, indexing="ij")
    num, den = cfg.bin_width()
    b = M.bin_index(n, cfg.n_kbins, num, den)
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    sel = b >= 0
    kh = np.stack([kx[sel], ky[sel], kz[sel]], axis=1) / kk[sel][:, None]
    bs = b[sel]
    pos = np.concatenate([g.pos(), r.pos()])
    xh = pos - np.asarray(cfg.observer)[None, :]
    xh /= np.linalg.norm(xh, axis=1)[:, None]
    w2 = np.concatenate([g.w ** 2, alpha ** 2 * r.w ** 2])
    counts = np.bincount(bs, minlength=cfg.n_kbins)
    out = {}
    for l in (0, 2, 4):
        per_mode = np.zeros(bs.size)
        for i0 in range(0, pos.shape[0], 2000):
            mu = kh @ xh[i0:i0 + 2000].T
            per_mode += eval_legendre(l, mu) @ w2[i0:i0 + 2000]
        out[l] = (2 * l + 1) * np.bincount(bs, weights=per_mode, minlength=cfg.n_kbins) / (norm * counts)
    return out


def test_density_shot_noise_poisson_expectation():
    """Poisson galaxies and randoms (unequal weights, alpha = 1/3), NGP, no
    interlacing or compensation: E|F_delta(k)|^2 is exactly the self-pair sum
    for k != 0, so <DD_l0> = 0 after the subtraction of shot_dd, and <DD_l> for
    l = 2, 4 equals the self-pair sum with L_l(khat.xhat) of each object (zero
    for l = 2 on the cubic-symmetric shells).  An alpha in place of alpha^2 in
    shot_dd shifts <DD_l0> by half the shot noise."""
    n, box, origin = 16, 200.0, (140.0, -60.0, 90.0)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=(0.0, 0.0, 0.0), assignment=1, interlacing=0,
                   compensate=0, n_kbins=6, lmax=4, families=("DD",))
    resid = {0: [], 2: [], 4: []}
    shot = []
    for seed in range(20):
        g, r = _poisson_pair(seed, 1500, 4500, origin, box)
        res = E.mesh64(g, r, cfg)
        d = dict(zip(res["series"], res["re"]))
        selfp = _self_pair_sums(cfg, g, r, res["alpha"], res["norm_I"])
        resid[0].append(d["DD_l0"] + res["shot_dd"] - selfp[0])
        resid[2].append(d["DD_l2"] - selfp[2])
        resid[4].append(d["DD_l4"] - selfp[4])
        shot.append(res["shot_dd"])
        # the self-pair monopole is the closed form itself (shells of any size)
        assert np.allclose(selfp[0], res["shot_dd"], rtol=1e-12)
        if seed == 0:
            assert np.max(np.abs(selfp[2])) < 1e-12 * res["shot_dd"]   # cubic shells: l = 2 self term is 0
            assert np.max(np.abs(selfp[4])) > 1e-3 * res["shot_dd"]    # l = 4 is not
    S = float(np.mean(shot))
    for l, v in resid.items():
        v = np.asarray(v)[:, 1:]   # bin 0 has only the few lowest modes
        mean, err = float(v.mean()), float(v.std(ddof=1) / math.sqrt(v.size))
        assert abs(mean) < 4 * err + 1e-3 * S, (l, mean, err, S)
        assert err < 0.05 * S   # an alpha for alpha^2 shifts the mean by S/2
    # resid[0] is the returned DD_l0 itself (the self-pair monopole equals shot_dd)


# ---------------------------------------------------------------------------
# EE / BB rows


@pytest.mark.parametrize("lmax", [4, 8])
def test_eb_rows_pure_e_and_pure_b(lmax):
    """A linear tidal field seen from a distant observer is pure E: the
    oracle's BB_l rows vanish and its EE_l rows equal P_+^(l) (P_+ = P_- for
    an E field).  Turning every shape by 45 degrees (gamma -> i gamma) maps
    E to B: EE and BB trade places.  On the discrete shells the m=4 series
    truncated at L = 4 leaves a residual of up to ~20 % at l = 4 (the
    per-mode power of one realisation is not a smooth function of mu), so
    l = 4 is checked with lmax = 8, where the L = 6, 8 terms bring the
    residuals at l <= 6 below 4 %."""
    n, box = 16, 800.0
    nhat = np.array([0.0, 0.6, 0.8])
    origin = tuple(1.0e7 * nhat - box / 2)
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=1, interlacing=0, compensate=0,
                   n_kbins=8, lmax=lmax, families=("PLUS", "MINUS"))
    ells = (0, 2) if lmax == 4 else (0, 2, 4, 6)   # l = lmax is the most truncated row
    tol = 0.05 if lmax == 4 else 0.04
    for seed in range(4):
        g, r, _ = lattice_catalogs(n, box, origin, (0.0, 0.0, 0.0), 200 + seed, amp=1.0)
        res = E.mesh64(g, r, cfg)
        s = res["series"]

        def row(name, rr=res):
            # the lattice has no shape noise: add back the N_+ subtracted from l = 0
            v = rr["re"][s.index(name)]
            if name.endswith("_l0"):
                v = v + (0.5 if name[:2] in ("EE", "BB") else 1.0) * rr["shot_plus"]
            return v
        big = res["n_modes"] > 400
        e0 = np.abs(row("EE_l0"))[big]
        for l in ells:
            bb = row(f"BB_l{l}")[big]
            ee = row(f"EE_l{l}")[big]
            pp = row(f"PLUS_l{l}")[big]
            assert np.all(np.abs(bb) < tol * e0), (l, bb / e0)
            assert np.all(np.abs(ee - pp) < tol * e0), (l, (ee - pp) / e0)
        # the same field turned into pure B
        gb = Catalog(g.x, g.y, g.z, g.w, g.nbar, -g.g2, g.g1)
        rb = E.mesh64(gb, r, cfg)
        for l in ells:
            assert np.allclose(row(f"BB_l{l}", rb)[big], row(f"EE_l{l}")[big], rtol=1e-9, atol=1e-12 * e0.max())
            assert np.all(np.abs(row(f"EE_l{l}", rb)[big]) < tol * e0)


# ---------------------------------------------------------------------------
# emulator model moments and sigma8


@pytest.mark.parametrize("b,f", [(1.0, 0.0), (2.0, 0.7), (1.3, 0.95), (2.9, 0.5)])
def test_gd_moments_by_quadrature(b, f):
    """(2L+1)(L-2)!/(L+2)! int dmu/2 [-(1/2)(1-mu^2)(b+f mu^2)] L^2_L(mu) with
    scipy's lpmv (Condon-Shortley phase, +1 at m = 2)."""
    got = W.gd_moments(b, f)
    for L in (2, 4):
        c = (2 * L + 1) * math.factorial(L - 2) / math.factorial(L + 2)
        val = quad(lambda mu: -0.5 * (1 - mu * mu) * (b + f * mu * mu) * lpmv(2, L, mu), -1, 1,
                   epsabs=1e-15, epsrel=1e-13)[0] / 2.0
        assert abs(got[L] - c * val) <= 1e-12 * max(1.0, abs(c * val)), (L, got[L], c * val)
    # and the moments beyond L = 4 vanish (the model is a degree-4 polynomial times (1-mu^2))
    c6 = quad(lambda mu: (1 - mu * mu) * (b + f * mu * mu) * lpmv(2, 6, mu), -1, 1)[0]
    assert abs(c6) < 1e-12


def test_sigma8_by_quadrature():
    """sigma8^2 = int dk k^2 P(k) W_TH(8k)^2 / (2 pi^2) by adaptive quadrature
    in ln k, against the trapezoid of the oracle on the template's log grid."""
    from synth import power_spectrum
    k = W.log_grid(1e-5, 1e3, 4096)
    got = W.sigma8(k, power_spectrum(k))

    def f(lnk):
        kk = math.exp(lnk)
        x = 8.0 * kk
        wth = 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3 if x > 1e-3 else 1.0 - x * x / 10.0
        return kk ** 3 * float(power_spectrum(kk)) * wth ** 2 / (2 * math.pi ** 2)
    pts = np.log([1e-3, 1e-2, 0.05, 0.1, 0.3, 1.0, 3.0, 10.0])
    want = quad(f, math.log(1e-5), math.log(1e3), points=pts, limit=2000, epsabs=0, epsrel=1e-12)[0]
    assert abs(got - math.sqrt(want)) <= 1e-6 * math.sqrt(want), (got, math.sqrt(want))


# ---------------------------------------------------------------------------
# separation shells of the window multipoles


@pytest.mark.parametrize("n,box,nb,rmax", [(32, 200.0, 16, 100.0), (32, 600.0, 12, 240.0), (16, 500.0, 10, 200.0),
                                           (24, 170.0, 7, 80.0)])
def test_r_thresholds_exact(n, box, nb, rmax):
    """Every minimum-image offset q = |n|^2 falls in the shell b with
    b dr <= |n| H < (b+1) dr, decided in exact rationals from the FP64 values
    of u = dr / H; q = 0 and q beyond the last edge are in no shell."""
    T = W.r_thresholds(n, box, nb, rmax)
    u = Fraction((rmax / nb) / (box / n))
    qmax = 3 * (n // 2) ** 2
    for q in range(qmax + 1):
        want = -1
        if q > 0:
            for b in range(nb):
                if (b * u) ** 2 <= q < ((b + 1) * u) ** 2:
                    want = b
                    break
        got = int(np.searchsorted(T, q, side="right") - 1)
        if q == 0 or q >= T[-1]:
            got = -1
        assert got == want, (q, got, want)


def test_window_shell_counts_exact():
    """The window multipoles' per-shell counts against a brute-force count of
    every mesh offset (minimum image) in exact rational arithmetic."""
    from synth import wedge_uniform
    n, box, nb, rmax = 16, 500.0, 9, 230.0
    rng = np.random.default_rng(5)
    rp = wedge_uniform(3000, rng, (5.0, 80.0), (5.0, 60.0), (60.0, 200.0))
    ran = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), np.ones(3000), np.full(3000, 1e-3))
    out = W.window_multipoles(ran, 0.1, n, box, (-80.0, -80.0, -80.0), (0.0, 0.0, 0.0), 2, 0, 1, 2, nb, rmax)
    u = Fraction((rmax / nb) / (box / n))
    m = [i if i < n // 2 else i - n for i in range(n)]
    want = [0] * nb
    for a in m:
        for b in m:
            for c in m:
                q = a * a + b * b + c * c
                if q == 0:
                    continue
                for s in range(nb):
                    if (s * u) ** 2 <= q < ((s + 1) * u) ** 2:
                        want[s] += 1
                        break
    assert list(out["counts"]) == want


# ---------------------------------------------------------------------------
# assignment window (compensation)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_compensation_is_the_stencil_transform(p):
    """Averaged over the object's offset u in one cell, the phase of its
    assignment stencil relative to its own position,
    sum_c W_p(u - c) exp(2 pi i m (u - c) / N), is the Fourier transform of
    the assignment window at k = 2 pi m / (N H): sinc(pi m / N)^p.  The
    average is taken by Gauss-Legendre quadrature on the sub-intervals where
    the stencil is one polynomial (the oracle's stencil gives the weights)."""
    n = 16
    comp = M.compensation(n, p)
    modes = M.signed_modes(n)
    # breakpoints of the piecewise-polynomial stencil inside [0, 1)
    cuts = [0.0, 0.5, 1.0] if p in (1, 3) else [0.0, 1.0]
    xg, wg = np.polynomial.legendre.leggauss(24)
    acc = np.zeros(n, dtype=np.complex128)
    for a, b in zip(cuts[:-1], cuts[1:]):
        u = 0.5 * (b - a) * xg + 0.5 * (b + a)
        wq = 0.5 * (b - a) * wg
        # keep the quadrature nodes off the breakpoints where NGP/TSC switch node
        c, w = M.stencil_1d(u + 3.0, p)   # any integer shift; the phase uses u - c only
        d = (u + 3.0)[:, None] - c
        ph = np.exp(2j * np.pi * modes[None, None, :] * d[:, :, None] / n)
        acc += np.sum(wq[:, None] * np.sum(w[:, :, None] * ph, axis=1), axis=0)
    want = comp[:, 0, 0]
    assert np.max(np.abs(acc - want)) < 1e-12, (p, acc, want)
    # the 3D window is the product over axes
    assert np.allclose(comp, want[:, None, None] * want[None, :, None] * want[None, None, :], rtol=0, atol=1e-15)
