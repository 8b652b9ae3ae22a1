"""Exact-rational special functions used by the estimator (oracle side).

Polynomials are lists of ``fractions.Fraction`` coefficients, lowest power
first.  Everything here follows Sec. II.D of the paper:
  * Legendre polynomials L_l(mu) (Rodrigues' formula);
  * associated Legendre L^m_L(mu) = (-1)^m (1-mu^2)^(m/2) d^m L_L/dmu^m
    (eq. def_of_asso, Condon-Shortley phase included);
  * the reduced kernels R^m_L(mu) = L^m_L(mu) / (1-mu^2)^(m/2), which are
    polynomials (the cancellation the paper uses to make the estimators
    FFT-able, eqs. def_of_Xiij and def_of_Xiijkl);
  * multipole prefactors (2L+1)(L-m)!/(L+m)! (eqs. multipole_cross_def,
    Hankel_trs_-);
  * C_{lL} = (2l+1) int dmu/2 L^4_L(mu) L_l(mu), the Legendre content of the
    m=4 basis used to read P_EE / P_BB off P_+ and P_- (eq. relation_pm_EB).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import numpy as np


def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pderiv(a, m=1):
    for _ in range(m):
        a = [a[i] * i for i in range(1, len(a))] or [Fraction(0)]
    return a


def _ppow(a, n):
    out = [Fraction(1)]
    for _ in range(n):
        out = _pmul(out, a)
    return out


@lru_cache(maxsize=None)
def legendre(l: int):
    """Coefficients of L_l(mu) via Rodrigues: L_l = 1/(2^l l!) d^l/dmu^l (mu^2-1)^l."""
    base = _ppow([Fraction(-1), Fraction(0), Fraction(1)], l)
    d = _pderiv(base, l)
    s = Fraction(1, 2 ** l * factorial(l))
    return tuple(c * s for c in d)


@lru_cache(maxsize=None)
def reduced_assoc(m: int, L: int):
    """R^m_L(mu) = L^m_L / (1-mu^2)^(m/2) = (-1)^m d^m L_L/dmu^m (a polynomial)."""
    d = _pderiv(list(legendre(L)), m)
    sgn = -1 if m % 2 else 1
    return tuple(c * sgn for c in d)


def peval(coefs, x):
    """Evaluate a polynomial with Fraction coefficients at float/array x (Horner, fp64)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for c in reversed(coefs):
        out = out * x + float(c)
    return out


def assoc_legendre(m: int, L: int, mu):
    """L^m_L(mu) with the Condon-Shortley phase, eq. def_of_asso (fp64)."""
    mu = np.asarray(mu, dtype=np.float64)
    return (1.0 - mu * mu) ** (m / 2.0) * peval(reduced_assoc(m, L), mu)


def _integrate_sym(coefs):
    """int_{-1}^{1} dmu/2 p(mu) for a Fraction polynomial."""
    s = Fraction(0)
    for i, c in enumerate(coefs):
        if i % 2 == 0:
            s += c / (i + 1)
    return s


def assoc_norm(m: int, L: int) -> Fraction:
    """int dmu/2 (L^m_L)^2 computed by exact integration (eq. ortho_asso_legendre)."""
    r = list(reduced_assoc(m, L))
    w = _ppow([Fraction(1), Fraction(0), Fraction(-1)], m)  # (1-mu^2)^m
    return _integrate_sym(_pmul(_pmul(r, r), w))


def prefactor(m: int, L: int) -> Fraction:
    """(2L+1)(L-m)!/(L+m)!: the multipole prefactor of the m-basis (m=0: 2l+1)."""
    return Fraction((2 * L + 1) * factorial(L - m), factorial(L + m))


def cmap_minus_to_legendre(l: int, L: int) -> Fraction:
    """C_{lL} = (2l+1) int dmu/2 L^4_L(mu) L_l(mu)."""
    r = list(reduced_assoc(4, L))
    w = _ppow([Fraction(1), Fraction(0), Fraction(-1)], 2)
    p = _pmul(_pmul(r, w), list(legendre(l)))
    return (2 * l + 1) * _integrate_sym(p)


# ---------------------------------------------------------------------------
# Wigner 3j symbols and the window mixing matrix (Sec. III.B eq. def_of_Q_llp)

def wigner3j(j1, j2, j3, m1, m2, m3):
    """Exact Wigner 3j symbol (sympy); returned as a sympy number."""
    from sympy.physics.wigner import wigner_3j
    return wigner_3j(j1, j2, j3, m1, m2, m3)


def window_coef(mX: int, l: int, lp: int, lpp: int):
    """Coefficient of Q_{l''} in Q^X_{l l'} (eq. def_of_Q_llp), exact (sympy)."""
    import sympy as sp
    if l < mX or lp < mX:
        return sp.Integer(0)
    f = sp.sqrt(sp.Rational(factorial(l - mX), factorial(l + mX)) *
                sp.Rational(factorial(lp + mX), factorial(lp - mX)))
    v = (2 * l + 1) * f * wigner3j(lpp, l, lp, 0, 0, 0) * wigner3j(lpp, l, lp, 0, mX, -mX)
    return sp.nsimplify(sp.simplify(v))


def binom(n, k):
    return comb(n, k)
