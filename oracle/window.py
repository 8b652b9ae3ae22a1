"""FP64 oracle of the window-convolved template path (Sec. III.B and IV.C).

Test infrastructure only: the HIP path never imports this module.

``window_multipoles``  the multipoles Q_l(r) of the window's auto-correlation
    (eqs. windowQ, windowQ_ell) on the mesh, with the end-point line of
    sight d = xhat of the first point of the pair.  The window is W(x) =
    alpha sum_r w_r delta_D(x - x_r) (the randoms weighted to the galaxy
    density), deposited like the estimator's density field.  The Legendre
    polynomial L_l(rhat . xhat) is expanded in monomials of the Cartesian
    components of rhat and xhat; every monomial coefficient of xhat is
    deposited and transformed, cross-correlated with W by FFT, and contracted
    with the same monomial of rhat in configuration space.  Q_l is the shell
    average times (2l+1), divided by the cell volume (mesh sum -> integral)
    and by I = alpha sum_r w_r^2 nbar_r, so that Q_0 -> 1 as r -> 0.

``hankel``  the transforms H_l and H_l^{-1} of Sec. I (the paper's
    definitions, with the factors 4 pi (-i)^l and i^l / (2 pi^2)) evaluated
    with FFTLog (Hamilton 2000): on a log-spaced grid the input times r^3
    (or k^3) is a sum of complex powers, each of which the spherical Bessel
    kernel maps in closed form through its Mellin transform
    int_0^inf t^(s-1) j_l(t) dt = sqrt(pi) 2^(s-2) Gamma((l+s)/2) / Gamma((3+l-s)/2).

``template_plain``  the window-convolved multipoles of the linear tidal
    alignment model used for the emulator: P_lin = (sigma8/sigma8_fid)^2
    P_fid, P_+ = (A^2/4)(1-mu^2)^2 P_lin (no RSD on shapes) and
    P_gd = -(A/2)(1-mu^2)(b + f mu^2) P_lin, whose multipoles are
    P_+^(0,2,4) = A^2 {2/15, -4/21, 2/35} P_lin and P_gd^(2,4) =
    -A {(7b+f)/42, f/105} P_lin; each is taken to xi by H^{-1}, multiplied by
    Q^X_{l l'}(r) of eq. def_of_Q_llp and taken back by H_l
    (eq. window_convolution_X_hankel), then interpolated (linear in ln k) to
    the output wavenumbers.  The shot noise s_N 2 sigma_gamma^2 / nbar is
    added to P~_+^(0) unconvolved.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, Tuple

import numpy as np
from scipy.special import loggamma

from . import geometry, mesh, special

# ---------------------------------------------------------------------------
# window multipoles on the mesh


def _multinomial_monomials(j: int):
    """{(a, b, c): multinomial(j; a, b, c)} for a + b + c = j."""
    out = {}
    for a in range(j + 1):
        for b in range(j - a + 1):
            c = j - a - b
            out[(a, b, c)] = math.factorial(j) // (math.factorial(a) * math.factorial(b) * math.factorial(c))
    return out


def r_thresholds(n: int, box: float, n_rbins: int, rmax: float) -> np.ndarray:
    """Integer thresholds on q = |n|^2 (n the minimum-image offset in cells):
    bin b holds T_b <= q < T_{b+1}, with T_b = ceil((b u)(b u)), u = (rmax /
    n_rbins) / (box / n), evaluated in FP64 in this order."""
    u = (rmax / n_rbins) / (box / n)
    return np.array([math.ceil((b * u) * (b * u)) for b in range(n_rbins + 1)], dtype=np.int64)


def window_multipoles(ran, alpha: float, n: int, box: float, origin, observer, assignment: int,
                      interlacing: int, compensate: int, lmax: int, n_rbins: int, rmax: float) -> Dict:
    pos = ran.pos()
    w = alpha * ran.w
    xh = geometry.los(pos, observer)
    comp = mesh.compensation(n, assignment) if compensate else np.ones((n,) * 3)
    phase = mesh.interlace_phase(n) if interlacing else None

    def transform(values):
        F = mesh.fftn(mesh.deposit(pos, values, n, box, origin, assignment))
        if interlacing:
            F2 = mesh.fftn(mesh.deposit(pos, values, n, box, origin, assignment, shift=0.5))
            F = 0.5 * (F + phase * F2)
        return F / comp

    F0 = transform(w)
    m = mesh.signed_modes(n).astype(np.float64)
    rx, ry, rz = np.meshgrid(m, m, m, indexing="ij")
    q = (rx * rx + ry * ry + rz * rz).astype(np.int64)
    rr = np.sqrt(q.astype(np.float64))
    inv = np.where(rr > 0, 1.0 / np.where(rr > 0, rr, 1.0), 0.0)
    rh = (rx * inv, ry * inv, rz * inv)
    T = r_thresholds(n, box, n_rbins, rmax)
    bidx = np.searchsorted(T, q, side="right") - 1
    bidx[(q <= 0) | (q >= T[-1])] = -1
    sel = bidx >= 0
    counts = np.bincount(bidx[sel], minlength=n_rbins)
    h = box / n
    rsum = np.bincount(bidx[sel], weights=rr[sel] * h, minlength=n_rbins)
    I = alpha * float(np.sum(ran.w ** 2 * ran.nbar))
    vcell = h ** 3
    ells = list(range(0, lmax + 1, 2))
    cache = {}
    Q = np.zeros((len(ells), n_rbins))
    for i, l in enumerate(ells):
        G = np.zeros((n,) * 3)
        for j, c in enumerate(special.legendre(l)):
            if c == 0:
                continue
            for a, mult in _multinomial_monomials(j).items():
                if a not in cache:
                    Fa = transform(w * xh[:, 0] ** a[0] * xh[:, 1] ** a[1] * xh[:, 2] ** a[2])
                    cache[a] = np.real(mesh.ifftn(np.conj(Fa) * F0))
                G += float(c) * mult * rh[0] ** a[0] * rh[1] ** a[1] * rh[2] ** a[2] * cache[a]
        s = np.bincount(bidx[sel], weights=G[sel], minlength=n_rbins)
        Q[i] = (2 * l + 1) * s / (np.where(counts > 0, counts, 1) * vcell * I)
    r_eff = np.where(counts > 0, rsum / np.where(counts > 0, counts, 1), 0.0)
    return dict(ells=ells, Q=Q, counts=counts, r_eff=r_eff, norm_I=I, thresholds=T)


# ---------------------------------------------------------------------------
# FFTLog Hankel transforms


def mellin_jl(l: int, s: np.ndarray) -> np.ndarray:
    """int_0^inf t^(s-1) j_l(t) dt for complex s with -l < Re s < 2."""
    return np.exp(math.log(math.sqrt(math.pi)) + (s - 2.0) * math.log(2.0) + loggamma(0.5 * (l + s))
                  - loggamma(0.5 * (3.0 + l - s)))


def log_grid(xmin: float, xmax: float, n: int) -> np.ndarray:
    return np.exp(np.linspace(math.log(xmin), math.log(xmax), n))


def fftlog_integral(x: np.ndarray, fx: np.ndarray, l: int, q: float, kr: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """y_j and G(y_j) = int_0^inf f(x) j_l(x y) x^2 dx on the reciprocal log
    grid y_j = kr / x_{N-1-j}, for f sampled at log-spaced x (FFTLog, bias q).

    With u_n = f(x_n) x_n^(3-q) and c_m its DFT, f(x) x^3 = x^q (1/N) sum_m
    c_m (x/x_0)^(i w_m), w_m = 2 pi m / (N d), d the log spacing.  Each term
    integrates in closed form, int x^(q+iw) j_l(xy) dx/x = y^(-q-iw) M(q+iw),
    and y_j = y_0 e^(j d) turns the sum over m into a second DFT."""
    n = x.size
    d = math.log(x[-1] / x[0]) / (n - 1)
    u = fx * x ** (3.0 - q)
    c = np.fft.fft(u)
    w = np.fft.fftfreq(n, d=d) * 2.0 * math.pi
    y = kr / x[::-1]
    t = c * mellin_jl(l, q + 1j * w) * (x[0] * y[0]) ** (-1j * w) / n
    return y, np.fft.fft(t).real * y ** (-q)


def hankel(x: np.ndarray, fx: np.ndarray, l: int, inverse: bool, q: float = None) -> Tuple[np.ndarray, np.ndarray]:
    """The paper's H_l (inverse=False: r -> k, 4 pi (-i)^l int r^2 dr j_l(kr) g)
    or H_l^{-1} (inverse=True: k -> r, i^l int k^2 dk / (2 pi^2) j_l(kr) g)
    for even l, on log grids.  q: FFTLog bias; the default (1.5 for k -> r;
    1.0 for r -> k at l = 0, 0.5 at l >= 2) keeps x^(3-q) f small at both
    ends of the grid for the template path's integrands (P ~ k at small k,
    damped at large k; xi finite at small r, windowed at large r), which the
    quadrature pins confirm."""
    if l % 2:
        raise ValueError("even multipoles only")
    sign = (-1) ** (l // 2)
    if q is None:
        q = 1.5 if inverse else (1.0 if l == 0 else 0.5)
    y, G = fftlog_integral(x, fx, l, q)
    if inverse:
        return y, sign * G / (2.0 * math.pi ** 2)
    return y, sign * 4.0 * math.pi * G


# ---------------------------------------------------------------------------
# model, sigma8 and the plain template path

PLUS_XI = {0: Fraction(2, 15), 2: Fraction(-4, 21), 4: Fraction(2, 35)}
MINUS_XI = {4: Fraction(1, 420)}


def gd_moments(b: float, f: float) -> Dict[int, float]:
    """m=2 moments of -(1/2)(1-mu^2)(b+f mu^2) (per unit A and P_lin)."""
    return {2: -(7.0 * b + f) / 42.0, 4: -f / 105.0}


def dd_moments(b: float, f: float) -> Dict[int, float]:
    """Legendre moments of the Kaiser spectrum (b + f mu^2)^2 (per unit P_lin)."""
    return {0: b * b + 2.0 * b * f / 3.0 + f * f / 5.0, 2: 4.0 * b * f / 3.0 + 4.0 * f * f / 7.0,
            4: 8.0 * f * f / 35.0}


def sigma8(k: np.ndarray, pk: np.ndarray) -> float:
    """Top-hat R = 8 Mpc/h rms of P(k) on a log grid (trapezoid in ln k)."""
    x = 8.0 * k
    wth = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    integrand = k ** 3 * pk * wth ** 2 / (2.0 * math.pi ** 2)
    lnk = np.log(k)
    return math.sqrt(float(np.sum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(lnk))))


def q_on_grid(r_q: np.ndarray, Q: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Tabulated Q_l(r) -> grid r: linear in r, Q(0) = (1, 0, 0, ...), zero beyond the table."""
    out = np.zeros((Q.shape[0], r.size))
    xs = np.concatenate([[0.0], r_q])
    for i in range(Q.shape[0]):
        ys = np.concatenate([[1.0 if i == 0 else 0.0], Q[i]])
        out[i] = np.interp(r, xs, ys, right=0.0)
    return out


def interp_lnk(k: np.ndarray, v: np.ndarray, kout: np.ndarray) -> np.ndarray:
    return np.interp(np.log(kout), np.log(k), v)


# (family, m of its window mixing, multipoles l of the output = model multipoles l')
FAMILIES = {"dd": (0, (0, 2, 4)), "gd": (2, (2, 4)), "plus": (0, (0, 2, 4)), "minus": (4, (4,))}


def template_families(k: np.ndarray, pfid: np.ndarray, r_q: np.ndarray, Q: np.ndarray, params: np.ndarray,
                      kout: np.ndarray, nbar: float, sigma_gamma: float, families, sigma8_fid: float = None) -> np.ndarray:
    """Window-convolved multipoles of the listed families at kout for every
    parameter point (A, b, f, sigma8, s_N): shape (n_pts, rows, n_k), the rows
    being each family's multipoles in order (dd l = 0, 2, 4; gd L = 2, 4;
    plus l = 0, 2, 4; minus L = 4).  Model, with P_lin = (sigma8/sigma8_fid)^2
    P_fid: P_dd = (b + f mu^2)^2 P_lin (Kaiser), P_gd = -(A/2)(1-mu^2)(b+f mu^2)
    P_lin, P_+ = P_- = (A^2/4)(1-mu^2)^2 P_lin (no RSD on shapes).  For each
    output multipole l of family X: xi^(l') = H^{-1}_{l'}[P_X^(l')] for each
    model multipole l', times Q^X_{l l'}(r) (eq. def_of_Q_llp, m of the
    family), summed, and H_l of the sum (eq. window_convolution_X_hankel),
    interpolated linearly in ln k; the shot noise s_N 2 sigma_gamma^2 / nbar
    is added to P~_+^(0).  k: the log grid of pfid (also the FFTLog grid);
    Q: Q_0..Q_8 at r_q."""
    s8f = sigma8(k, pfid) if sigma8_fid is None else sigma8_fid
    r = 1.0 / k[::-1]
    Qg = q_on_grid(r_q, Q, r)
    rows = [(X, l) for X in families for l in FAMILIES[X][1]]
    wc = {}
    for X, l in rows:
        mX, lps = FAMILIES[X]
        for lp in lps:
            c = np.array([float(special.window_coef(mX, l, lp, lpp)) for lpp in (0, 2, 4, 6, 8)])
            wc[(X, l, lp)] = np.tensordot(c, Qg, axes=(0, 0))
    out = np.zeros((params.shape[0], len(rows), kout.size))
    damp = np.exp(-(k / 10.0) ** 2)  # keeps k^3 P(k) localised on the grid; negligible for k <= 0.3
    for p_i, (A, b, f, s8, sN) in enumerate(params):
        plin = (s8 / s8f) ** 2 * pfid * damp
        amp = {"dd": dd_moments(b, f), "gd": {L: A * v for L, v in gd_moments(b, f).items()},
               "plus": {l: A * A * float(c) for l, c in PLUS_XI.items()},
               "minus": {L: A * A * float(c) for L, c in MINUS_XI.items()}}
        xi = {(X, lp): hankel(k, amp[X][lp] * plin, lp, inverse=True)[1] for X in families for lp in FAMILIES[X][1]}
        for row, (X, l) in enumerate(rows):
            g = np.zeros_like(r)
            for lp in FAMILIES[X][1]:
                g += wc[(X, l, lp)] * xi[(X, lp)]
            kk, P = hankel(r, g, l, inverse=False)
            out[p_i, row] = interp_lnk(kk, P, kout)
            if X == "plus" and l == 0:
                out[p_i, row] += sN * 2.0 * sigma_gamma ** 2 / nbar
    return out


def template_plain(k: np.ndarray, pfid: np.ndarray, r_q: np.ndarray, Q: np.ndarray, params: np.ndarray,
                   kout: np.ndarray, nbar: float, sigma_gamma: float, sigma8_fid: float = None) -> np.ndarray:
    """Window-convolved P~_+^(0,2,4) and P~_Ed^(2,4) at kout for every
    parameter point (A, b, f, sigma8, s_N): shape (n_pts, 5, n_k)."""
    return template_families(k, pfid, r_q, Q, params, kout, nbar, sigma_gamma, ("plus", "gd"), sigma8_fid)


def template_multipoles(k: np.ndarray, pfid: np.ndarray, r_q: np.ndarray, Q: np.ndarray, params: np.ndarray,
                        kout: np.ndarray, nbar: float, sigma_gamma: float, sigma8_fid: float = None) -> np.ndarray:
    """All four families, rows DD_l0,2,4, GD_L2,4, PLUS_l0,2,4, MINUS_L4:
    shape (n_pts, 9, n_k)."""
    return template_families(k, pfid, r_q, Q, params, kout, nbar, sigma_gamma, ("dd", "gd", "plus", "minus"),
                             sigma8_fid)


# ---------------------------------------------------------------------------
# window multipoles by pair counting


def window_pairs(ran, alpha: float, norm_I: float, observer, los: str, lmax: int, n_rbins: int, rmax: float,
                 chunk: int = 256) -> Dict:
    """Q_l(r)/I of eq. windowQ_ell by a direct sum over the ordered pairs
    (i, j), i != j, of the catalog: each pair separated by r = x_j - x_i adds
    alpha^2 w_i w_j L_l(rhat . dhat) to the shell b with (b dr)^2 <= |r|^2 <
    ((b+1) dr)^2, dr = rmax / n_rbins (|r|^2 = dx*dx + dy*dy + dz*dz in FP64;
    r = 0 in no shell), and Q_l = (2l+1) * sum / (V_b I), V_b the shell's
    volume.  The pair's line of sight dhat points from the observer to its
    midpoint (los = "midpoint": the paper's direction toward the pair) or to
    its first point x_i (los = "endpoint")."""
    pos = ran.pos()
    w = ran.w
    obs = np.asarray(observer, dtype=np.float64)
    n = pos.shape[0]
    dr = rmax / n_rbins
    T = np.array([(b * dr) * (b * dr) for b in range(n_rbins + 1)])
    ells = list(range(0, lmax + 1, 2))
    S = np.zeros((len(ells), n_rbins))
    counts = np.zeros(n_rbins, dtype=np.int64)
    rsum = np.zeros(n_rbins)
    for i0 in range(0, n, chunk):
        xi = pos[i0:i0 + chunk]
        d = pos[None, :, :] - xi[:, None, :]                      # r = x_j - x_i
        r2 = d[:, :, 0] * d[:, :, 0] + d[:, :, 1] * d[:, :, 1] + d[:, :, 2] * d[:, :, 2]
        ii = np.arange(i0, i0 + xi.shape[0])
        keep = (r2 < T[-1]) & (r2 > 0.0)
        keep[np.arange(xi.shape[0]), ii] = False
        b = np.searchsorted(T, r2, side="right") - 1
        r = np.sqrt(r2)
        if los == "midpoint":
            dv = xi[:, None, :] + 0.5 * d - obs[None, None, :]
        elif los == "endpoint":
            dv = np.broadcast_to(xi[:, None, :] - obs[None, None, :], d.shape)
        else:
            raise ValueError("los must be 'midpoint' or 'endpoint'")
        mu = np.einsum("ijk,ijk->ij", d, dv) / (np.where(r > 0, r, 1.0) * np.linalg.norm(dv, axis=2))
        ww = (w[i0:i0 + chunk][:, None] * w[None, :])
        bk = b[keep]
        counts += np.bincount(bk, minlength=n_rbins)
        rsum += np.bincount(bk, weights=r[keep], minlength=n_rbins)
        for k, l in enumerate(ells):
            S[k] += np.bincount(bk, weights=(ww * special.peval(special.legendre(l), mu))[keep], minlength=n_rbins)
    vb = 4.0 * math.pi / 3.0 * np.array([((b + 1) ** 3 - b ** 3) * dr ** 3 for b in range(n_rbins)])
    Q = np.array([(2 * l + 1) * alpha ** 2 * S[k] / (vb * norm_I) for k, l in enumerate(ells)])
    r_eff = np.where(counts > 0, rsum / np.where(counts > 0, counts, 1), 0.0)
    return dict(ells=ells, Q=Q, counts=counts, r_eff=r_eff)
