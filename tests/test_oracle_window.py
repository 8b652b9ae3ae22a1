"""Pins of the window / template oracle (oracle/window.py) against closed
forms, quadrature and geometry, independent of its own formulas."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import eval_legendre, spherical_jn

from oracle import special as S
from oracle import window as W
from synth import Catalog, box_uniform


def test_mellin_transform_of_spherical_bessel_closed_forms():
    # int_0^inf j_0 = pi/2, int_0^inf j_2 = pi/4, int_0^inf t^(1/2) j_0 = Gamma(1/2) sin(pi/4)
    assert abs(W.mellin_jl(0, np.array([1.0 + 0j]))[0] - math.pi / 2) < 1e-14
    assert abs(W.mellin_jl(2, np.array([1.0 + 0j]))[0] - math.pi / 4) < 1e-14
    assert abs(W.mellin_jl(0, np.array([1.5 + 0j]))[0] - math.sqrt(math.pi) * math.sin(math.pi / 4)) < 1e-14


K = W.log_grid(1e-5, 1e3, 4096)


@pytest.mark.parametrize("l", [0, 2, 4])
def test_inverse_hankel_matches_quadrature(l):
    sig = 2.0
    r, xi = W.hankel(K, np.exp(-(K * sig) ** 2), l, inverse=True)
    pts = np.exp(np.linspace(math.log(0.5), math.log(15.0), 22))
    scale = np.max(np.abs(xi[(r > 0.1) & (r < 50)]))
    for rr in pts:
        i = int(np.argmin(np.abs(np.log(r / rr))))
        val = quad(lambda k: k * k * spherical_jn(l, k * r[i]) * math.exp(-(k * sig) ** 2), 0, 14 / sig,
                   limit=500, epsabs=1e-16, epsrel=1e-13)[0]
        ref = (-1) ** (l // 2) * val / (2 * math.pi ** 2)
        assert abs(xi[i] - ref) <= 1e-6 * scale, (l, r[i], xi[i], ref)


@pytest.mark.parametrize("l", [0, 2, 4])
def test_forward_hankel_matches_quadrature(l):
    R = 1.0 / K[::-1]
    g = np.exp(-R ** 2 / 16.0) * (1.0 + R * R / 10.0)
    k, P = W.hankel(R, g, l, inverse=False)
    scale = np.max(np.abs(P[(k > 1e-3) & (k < 3)]))
    for kk in np.exp(np.linspace(math.log(0.01), math.log(2.0), 20)):
        i = int(np.argmin(np.abs(np.log(k / kk))))
        val = quad(lambda r: r * r * spherical_jn(l, k[i] * r) * math.exp(-r * r / 16.0) * (1 + r * r / 10.0),
                   0, 60.0, limit=800, epsabs=1e-14, epsrel=1e-13)[0]
        ref = 4 * math.pi * (-1) ** (l // 2) * val
        assert abs(P[i] - ref) <= 1e-6 * scale, (l, k[i], P[i], ref)


@pytest.mark.parametrize("l", [0, 2, 4])
def test_hankel_round_trip(l):
    P = np.exp(-(K * 2.0) ** 2) * K / (1 + K)
    r, xi = W.hankel(K, P, l, inverse=True)
    k2, P2 = W.hankel(r, xi, l, inverse=False)
    sel = (k2 > 1e-2) & (k2 < 1.0)  # the template path's range
    assert np.allclose(k2, K)
    # the two directions use different biases, so the discrete round trip is
    # not exact; the quadrature pins above fix each direction at 1e-6
    assert np.max(np.abs(P2[sel] - P[sel])) <= 1e-5 * np.max(np.abs(P[sel]))


def test_monomial_expansion_reproduces_legendre():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((50, 3))
    b = rng.standard_normal((50, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    b /= np.linalg.norm(b, axis=1)[:, None]
    for l in (0, 2, 4, 6, 8):
        tot = np.zeros(50)
        for j, c in enumerate(S.legendre(l)):
            for al, mult in W._multinomial_monomials(j).items():
                tot += float(c) * mult * np.prod(a ** np.array(al), axis=1) * np.prod(b ** np.array(al), axis=1)
        assert np.allclose(tot, eval_legendre(l, np.sum(a * b, axis=1)), atol=1e-12)


def _box_window(n_ran, sides, origin_in, observer, seed=3):
    rng = np.random.default_rng(seed)
    p = np.asarray(origin_in)[None, :] + rng.random((n_ran, 3)) * np.asarray(sides)[None, :]
    vol = float(np.prod(sides))
    nbar = 1e-3
    ran = Catalog(p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(), np.ones(n_ran), np.full(n_ran, nbar))
    alpha = nbar * vol / n_ran  # randoms weighted to the galaxy density
    return ran, alpha


def test_box_window_multipoles_match_overlap_volume():
    """A rectangular window W = 1 inside sides (a, a, a/2), observer far away
    along -z (line of sight ~ z for every point): Q_l(r)/I is the shell
    average of (2l+1) prod_i (1 - |r_i|/a_i) L_l(rhat_z), evaluated on the same
    mesh shells.  Mesh 32^3, TSC + interlacing, compensated; r in 4-10 cells."""
    n, box = 32, 200.0
    sides = np.array([80.0, 80.0, 40.0])
    origin = (0.0, 0.0, 0.0)
    obs = (100.0, 100.0, -1.0e7)
    ran, alpha = _box_window(400_000, sides, (20.0, 20.0, 20.0), obs)
    nb, rmax = 16, 100.0
    out = W.window_multipoles(ran, alpha, n, box, origin, obs, 3, 1, 1, 4, nb, rmax)
    m = np.fft.fftfreq(n, 1.0 / n)
    rx, ry, rz = np.meshgrid(m, m, m, indexing="ij")
    h = box / n
    q = (rx * rx + ry * ry + rz * rz).astype(np.int64)
    T = out["thresholds"]
    b = np.searchsorted(T, q, side="right") - 1
    b[(q <= 0) | (q >= T[-1])] = -1
    rr = np.sqrt(q.astype(float))
    ov = np.clip(1 - np.abs(rx) * h / sides[0], 0, None) * np.clip(1 - np.abs(ry) * h / sides[1], 0, None) \
        * np.clip(1 - np.abs(rz) * h / sides[2], 0, None)
    mu = np.where(rr > 0, rz / np.where(rr > 0, rr, 1), 0)
    for i, l in enumerate(out["ells"]):
        ref = np.array([(2 * l + 1) * np.mean((ov * eval_legendre(l, mu))[b == j]) for j in range(nb)])
        r_lo = (np.arange(nb) * rmax / nb) / h
        sel = (r_lo >= 4) & (r_lo <= 10)
        err = np.abs(out["Q"][i][sel] - ref[sel])
        assert np.max(err) < 0.01, (l, err, ref[sel])
    assert abs(out["norm_I"] - 1e-3 ** 2 * np.prod(sides)) < 1e-9 * out["norm_I"]
    assert np.array_equal(out["counts"], np.bincount(b[b >= 0], minlength=nb))


def test_identity_window_returns_model_multipoles():
    """Q_0 = 1 and Q_l>0 = 0 at every separation: the template path must
    return the model multipoles themselves (damping negligible at k <= 0.3)."""
    pfid = 2e4 * (K / 0.02) / (1 + (K / 0.02) ** 2) ** 1.4
    r_q = 1.0 / K[::-1]
    Q = np.zeros((5, r_q.size))
    Q[0] = 1.0
    kout = np.arange(1, 31) * 0.01
    pars = np.array([[0.03, 2.0, 0.7, 0.8, 1.0], [0.01, 1.2, 0.9, 0.65, 0.0]])
    s8f = W.sigma8(K, pfid)
    out = W.template_plain(K, pfid, r_q, Q, pars, kout, nbar=1e-3, sigma_gamma=0.2, sigma8_fid=s8f)
    for p, o in zip(pars, out):
        A, b, f, s8, sN = p
        plin = (s8 / s8f) ** 2 * np.interp(np.log(kout), np.log(K), pfid)
        want = [A * A * 2 / 15 * plin + sN * 2 * 0.2 ** 2 / 1e-3, -A * A * 4 / 21 * plin, A * A * 2 / 35 * plin,
                -A * (7 * b + f) / 42 * plin, -A * f / 105 * plin]
        for got, w in zip(o, want):
            assert np.max(np.abs(got - w)) <= 2e-5 * np.max(np.abs(w)) + 1e-12


def test_template_is_linear_in_its_amplitudes():
    """P~_+ scales as A^2 sigma8^2, P~_gd as A sigma8^2 (7b+f | f): exact
    invariants of the plain path for any window."""
    pfid = 2e4 * (K / 0.02) / (1 + (K / 0.02) ** 2) ** 1.4
    r_q = np.linspace(5, 3000, 300)
    Q = np.vstack([np.exp(-r_q / 800.0) * (1 - 0.1 * i) * (0.2 if i else 1.0) for i in range(5)])
    kout = np.arange(1, 31) * 0.01
    base = np.array([[0.02, 1.5, 0.6, 0.7, 0.0]])
    o1 = W.template_plain(K, pfid, r_q, Q, base, kout, 1e-3, 0.2)[0]
    o2 = W.template_plain(K, pfid, r_q, Q, base * np.array([[2.0, 1, 1, 1, 1]]), kout, 1e-3, 0.2)[0]
    o3 = W.template_plain(K, pfid, r_q, Q, base * np.array([[1.0, 1, 1, 1.5, 1]]), kout, 1e-3, 0.2)[0]
    assert np.allclose(o2[:3], 4 * o1[:3], rtol=1e-12, atol=0)
    assert np.allclose(o2[3:], 2 * o1[3:], rtol=1e-12, atol=0)
    assert np.allclose(o3, 2.25 * o1, rtol=1e-12, atol=0)
    # the hexadecapole of the cross term depends on f only
    o4 = W.template_plain(K, pfid, r_q, Q, np.array([[0.02, 2.5, 0.6, 0.7, 0.0]]), kout, 1e-3, 0.2)[0]
    assert not np.allclose(o4[3], o1[3])


@pytest.mark.parametrize("b,f", [(1.0, 0.0), (2.0, 0.7), (1.3, 0.95)])
def test_density_and_minus_model_moments_by_quadrature(b, f):
    """(2l+1) int dmu/2 (b + f mu^2)^2 L_l(mu) (Kaiser) with scipy's Legendre
    polynomials, and the minus spectrum's m=4 moment of (1/4)(1-mu^2)^2:
    (2L+1)(L-4)!/(L+4)! int dmu/2 (1/4)(1-mu^2)^2 L^4_L(mu) = 1/420 at L = 4
    (eq. xi_relations_normalization_coefficients) and 0 at L = 6, 8."""
    from scipy.special import lpmv
    got = W.dd_moments(b, f)
    for l in (0, 2, 4):
        val = (2 * l + 1) * quad(lambda mu: (b + f * mu * mu) ** 2 * eval_legendre(l, mu), -1, 1,
                                 epsabs=1e-15, epsrel=1e-13)[0] / 2.0
        assert abs(got[l] - val) <= 1e-12 * max(1.0, abs(val)), (l, got[l], val)
    for L in (4, 6, 8):
        c = (2 * L + 1) * math.factorial(L - 4) / math.factorial(L + 4)
        val = c * quad(lambda mu: 0.25 * (1 - mu * mu) ** 2 * lpmv(4, L, mu), -1, 1,
                       epsabs=1e-16, epsrel=1e-13)[0] / 2.0
        want = float(W.MINUS_XI.get(L, 0))
        assert abs(val - want) <= 1e-12, (L, val, want)


def test_all_families_follow_the_printed_convolutions():
    """For the validation model of Sec. IV.C (b = 1, f = 0, shapes e_ij T_ij,
    i.e. A = -1, sigma8 = sigma8_fid, no shot noise) every template row that
    the paper prints (eq. all_convolutions and the leakage equations) equals
    H_l of the printed combination: the xi relations (1/6, 2/15, -4/21, 2/35,
    1/420) times xi^(l') = H^{-1}_{l'}[P], times the printed coefficients of
    Q_0..Q_8 (tests/golden/window_coefficients.json)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "window_coefficients.json")))
    xr = {k: float(Fraction(v)) for k, v in gold["xi_relations"].items() if k != "cite"}
    pfid = 2e4 * (K / 0.02) / (1 + (K / 0.02) ** 2) ** 1.4
    r_q = np.linspace(5, 3000, 300)
    Q = np.vstack([np.exp(-r_q / 900.0) * (1.0 if i == 0 else 0.3 * (-1) ** i / (i + 1)) *
                   (1 + 0.2 * np.sin(r_q / 300.0 + i)) for i in range(5)])
    kout = np.arange(1, 31) * 0.01
    s8f = W.sigma8(K, pfid)
    got = W.template_multipoles(K, pfid, r_q, Q, np.array([[-1.0, 1.0, 0.0, s8f, 0.0]]), kout, 1e-3, 0.2,
                                sigma8_fid=s8f)[0]
    rows = ["dd_0", "dd_2", "dd_4", "gd_2", "gd_4", "plus_0", "plus_2", "plus_4", "minus_4"]
    r = 1.0 / K[::-1]
    Qg = W.q_on_grid(r_q, Q, r)
    plin = pfid * np.exp(-(K / 10.0) ** 2)
    xi = {lp: W.hankel(K, plin, lp, inverse=True)[1] for lp in (0, 2, 4)}
    norm = {("dd", 0): 1.0, ("gd", 2): xr["gd_L2"], ("plus", 0): xr["plus_l0"], ("plus", 2): xr["plus_l2"],
            ("plus", 4): xr["plus_l4"], ("minus", 4): xr["minus_L4"]}
    seen = set()
    for e in gold["entries"]:
        seen.add((e["X"], e["l"]))
    for X, l in sorted(seen):
        g = np.zeros_like(r)
        for e in gold["entries"]:
            if e["X"] == X and e["l"] == l:
                q = np.array([float(Fraction(v)) for v in e["q"]])
                g += norm[(X, e["lp"])] * xi[e["lp"]] * np.tensordot(q, Qg, axes=(0, 0))
        kk, P = W.hankel(r, g, l, inverse=False)
        want = W.interp_lnk(kk, P, kout)
        row = got[rows.index(f"{X}_{l}")]
        assert np.max(np.abs(row - want)) <= 1e-10 * np.max(np.abs(want)), (X, l)
    # the unprinted rows of this model: the density hexadecapole is leakage too,
    # and with f = 0 every model multipole of dd and gd above the lowest is zero
    assert np.max(np.abs(got[rows.index("dd_4")])) > 0


def _box_shell_average(sides, nb, rmax, ells, N):
    """(1 - 1/N) times the average over each spherical shell (volume weight)
    of (2l+1) prod_i (1 - |r_i|/a_i)_+ L_l(rhat_z): the expected Q_l/I of N
    uniform points in a box seen along z.  Gauss-Legendre in r and in mu
    (split at the kink mu = 0), midpoint rule in phi (kinks on the nodes'
    interval edges)."""
    from scipy.special import eval_legendre
    dr = rmax / nb
    xr, wr = np.polynomial.legendre.leggauss(8)
    xm, wm = np.polynomial.legendre.leggauss(32)
    phi = (np.arange(256) + 0.5) * 2 * np.pi / 256
    out = np.zeros((len(ells), nb))
    for b in range(nb):
        r = b * dr + 0.5 * dr * (xr + 1)
        wrr = 0.5 * dr * wr * r * r
        tot, norm = np.zeros(len(ells)), 0.0
        for half in (-1, 1):
            R, M, P = np.meshgrid(r, 0.5 * (xm + 1) * half, phi, indexing="ij")
            st = np.sqrt(1 - M * M)
            ov = (np.clip(1 - np.abs(R * st * np.cos(P)) / sides[0], 0, None) *
                  np.clip(1 - np.abs(R * st * np.sin(P)) / sides[1], 0, None) *
                  np.clip(1 - np.abs(R * M) / sides[2], 0, None))
            wt = wrr[:, None, None] * (0.5 * wm)[None, :, None] * np.ones_like(P)
            for k, l in enumerate(ells):
                tot[k] += (2 * l + 1) * np.sum(wt * ov * eval_legendre(l, M))
            norm += np.sum(wt)
        out[:, b] = tot / norm * (1 - 1 / N)
    return out


def test_window_pairs_box_window_matches_overlap_volume():
    """Pair counts of N uniform points in a box (sides 80, 80, 40) seen along
    z from far away: the mean over four catalogs of Q_l/I (alpha = nbar V/N,
    I = nbar^2 V) is the shell-volume average of (1 - 1/N)(2l+1) times the
    overlap fraction prod_i (1 - |r_i|/a_i) times L_l(rhat_z), within the
    pair-count noise (about 0.007 per catalog); end-point and midpoint lines
    of sight agree for a distant observer."""
    sides = np.array([80.0, 80.0, 40.0])
    N, nb, rmax = 4000, 6, 30.0
    want = _box_shell_average(sides, nb, rmax, [0, 2, 4], N)
    nbar, V = 1e-3, float(np.prod(sides))
    got = {"endpoint": [], "midpoint": []}
    for seed in range(4):
        rng = np.random.default_rng(seed)
        p = rng.random((N, 3)) * sides + 20.0
        cat = Catalog(p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(), np.ones(N), np.full(N, nbar))
        for los in got:
            out = W.window_pairs(cat, nbar * V / N, nbar ** 2 * V, (60.0, 60.0, -1e7), los, 4, nb, rmax)
            got[los].append(out["Q"])
    for los, qs in got.items():
        mean = np.mean(qs, axis=0)[:, 1:]      # shell 0 (r < 5) has few pairs
        assert np.max(np.abs(mean - want[:, 1:])) < 0.02, (los, mean - want[:, 1:])
    assert np.allclose(got["endpoint"], got["midpoint"], rtol=0, atol=1e-6)


def test_window_pairs_agree_with_the_mesh_route_at_large_separation():
    """The end-point pair counts and the mesh FFT route (window_multipoles,
    same catalog, same end-point line of sight) estimate the same Q_l: at
    separations of 4-8 cells they agree within the mesh route's assignment
    and shell discreteness (a few per cent of Q_0), while the midpoint pair
    counts of a near observer differ from both in l = 2 (wide angles)."""
    from synth import wedge_uniform
    rng = np.random.default_rng(8)
    n_ran = 6000
    rp = wedge_uniform(n_ran, rng, (5.0, 80.0), (5.0, 60.0), (60.0, 200.0))
    cat = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), np.ones(n_ran), np.full(n_ran, 1e-3))
    n, box, origin = 32, 500.0, (-80.0, -80.0, -80.0)
    nb, rmax, alpha = 10, 200.0, 0.1
    mesh = W.window_multipoles(cat, alpha, n, box, origin, (0.0, 0.0, 0.0), 3, 1, 1, 4, nb, rmax)
    ep = W.window_pairs(cat, alpha, mesh["norm_I"], (0.0, 0.0, 0.0), "endpoint", 4, nb, rmax)
    mp = W.window_pairs(cat, alpha, mesh["norm_I"], (0.0, 0.0, 0.0), "midpoint", 4, nb, rmax)
    h = box / n
    sel = (np.arange(nb) * rmax / nb >= 4 * h) & (np.arange(nb) * rmax / nb <= 8 * h)
    scale = np.max(np.abs(mesh["Q"][0][sel]))
    assert np.max(np.abs(ep["Q"][:, sel] - mesh["Q"][:, sel])) < 0.05 * scale
    assert np.max(np.abs(mp["Q"][1][sel] - ep["Q"][1][sel])) > 0.01 * scale
