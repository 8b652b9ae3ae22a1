"""Pins of the oracle's special functions against closed forms, a library
routine (scipy's lpmv) and the exact rationals the paper prints."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import lpmv, eval_legendre

from oracle import special as S, geometry as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_legendre_closed_forms():
    mu = np.linspace(-1, 1, 41)
    assert np.allclose(S.peval(S.legendre(2), mu), 0.5 * (3 * mu ** 2 - 1), atol=1e-15)
    assert np.allclose(S.peval(S.legendre(4), mu), (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8, atol=1e-15)
    for l in range(9):
        assert np.allclose(S.peval(S.legendre(l), mu), eval_legendre(l, mu), atol=1e-13)


@pytest.mark.parametrize("m,L", [(2, 2), (2, 4), (2, 6), (4, 4), (4, 6), (4, 8), (1, 3), (3, 5)])
def test_assoc_legendre_matches_scipy(m, L):
    # scipy's lpmv includes the Condon-Shortley phase, as eq. def_of_asso does
    mu = np.linspace(-0.999, 0.999, 57)
    assert np.allclose(S.assoc_legendre(m, L, mu), lpmv(m, L, mu), rtol=1e-11, atol=1e-11)


def test_reduced_kernels_closed_forms():
    # R^2_L = L^2_L/(1-mu^2) and R^4_L = L^4_L/(1-mu^2)^2 (Sec. III.A) are polynomials
    assert S.reduced_assoc(2, 2) == (Fraction(3),)
    assert S.reduced_assoc(2, 4) == (Fraction(-15, 2), 0, Fraction(105, 2))
    assert S.reduced_assoc(4, 4) == (Fraction(105),)
    assert S.reduced_assoc(4, 6) == (Fraction(-945, 2), 0, Fraction(10395, 2))
    r48 = S.reduced_assoc(4, 8)
    assert r48 == (Fraction(10395, 8), 0, Fraction(-10395 * 26, 8), 0, Fraction(10395 * 65, 8))


@pytest.mark.parametrize("m", [0, 2, 4])
def test_orthogonality_normalisation(m):
    # eq. ortho_asso_legendre: int dmu/2 L^m_L L^m_L' = (L+m)!/((2L+1)(L-m)!) delta_LL'
    from math import factorial
    for L in range(m, 10):
        assert S.assoc_norm(m, L) == Fraction(factorial(L + m), (2 * L + 1) * factorial(L - m))
    # off-diagonal vanishes (numerical quadrature, independent of the exact route)
    x, w = np.polynomial.legendre.leggauss(40)
    for L in range(max(m, 1), 8):
        for Lp in range(L + 1, 9):
            v = 0.5 * np.sum(w * S.assoc_legendre(m, L, x) * S.assoc_legendre(m, Lp, x))
            assert abs(v) < 1e-9


def test_prefactors_and_minus_map():
    assert S.prefactor(2, 2) == Fraction(5, 24)
    assert S.prefactor(2, 4) == Fraction(1, 40)
    assert S.prefactor(2, 6) == Fraction(13, 1680)
    assert S.prefactor(4, 4) == Fraction(1, 4480)
    assert [S.cmap_minus_to_legendre(l, 4) for l in (0, 2, 4, 6)] == [56, -80, 24, 0]
    # C_{lL} reproduces L^4_L in the Legendre basis: sum_l C_{lL} L_l(mu) = L^4_L(mu)
    mu = np.linspace(-1, 1, 21)
    for L in (4, 6, 8):
        rec = sum(float(S.cmap_minus_to_legendre(l, L)) * eval_legendre(l, mu) for l in range(0, L + 1, 2))
        assert np.allclose(rec, S.assoc_legendre(4, L, mu), atol=1e-9)


def test_xi_relation_coefficients():
    """Multipoles of the validation spectra P_gd = (1/2)(1-mu^2)P, P_+ = P_- = (1/4)(1-mu^2)^2 P
    (Sec. IV.A eq. power_for_validation) give the paper's eq.
    xi_relations_normalization_coefficients: 1/6, {2/15, -4/21, 2/35}, 1/420."""
    half = [Fraction(1, 2), 0, Fraction(-1, 2)]
    quarter = [Fraction(1, 4), 0, Fraction(-1, 2), 0, Fraction(1, 4)]

    def moment(m, L, model):
        # (2L+1)(L-m)!/(L+m)! int dmu/2 P(mu) L^m_L(mu), with L^m_L = (1-mu^2)^{m/2} R^m_L
        r = list(S.reduced_assoc(m, L)) if m else list(S.legendre(L))
        w = S._ppow([Fraction(1), 0, Fraction(-1)], m // 2)
        p = S._pmul(S._pmul(model, r), w)
        return S.prefactor(m, L) * S._integrate_sym(p)

    gold = json.load(open(os.path.join(GOLD, "window_coefficients.json")))["xi_relations"]
    assert moment(2, 2, half) == Fraction(gold["gd_L2"])
    assert moment(0, 0, quarter) == Fraction(gold["plus_l0"])
    assert moment(0, 2, quarter) == Fraction(gold["plus_l2"])
    assert moment(0, 4, quarter) == Fraction(gold["plus_l4"])
    assert moment(4, 4, quarter) == Fraction(gold["minus_L4"])
    assert moment(2, 4, half) == 0


def test_window_coefficients_match_paper():
    gold = json.load(open(os.path.join(GOLD, "window_coefficients.json")))
    for e in gold["entries"]:
        got = [S.window_coef(e["mX"], e["l"], e["lp"], lpp) for lpp in (0, 2, 4, 6, 8)]
        want = [Fraction(q) for q in e["q"]]
        assert [Fraction(str(g)) for g in got] == want, e["cite"]


def test_standard_rotation_and_helicity_identities():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((200, 3))
    xh = v / np.linalg.norm(v, axis=1)[:, None]
    S_ = G.standard_rotation(xh)
    assert np.allclose(np.einsum("nji,njk->nik", S_, S_), np.eye(3)[None], atol=1e-14)
    assert np.allclose(S_[:, :, 2], xh, atol=1e-15)
    assert np.allclose(np.linalg.det(S_), 1.0)
    _, et, ep = G.basis(v + 0.0, (0.0, 0.0, 0.0))
    e = G.e_tensor(et, ep)
    # Sec. II.B: e_ii = e_ij e_ij = 0, e_ij e*_ij = 1, e_ij xhat_j = 0
    assert np.allclose(np.einsum("nii->n", e), 0, atol=1e-15)
    assert np.allclose(np.einsum("nij,nij->n", e, e), 0, atol=1e-15)
    assert np.allclose(np.einsum("nij,nij->n", e, np.conj(e)), 1, atol=1e-14)
    assert np.allclose(np.einsum("nij,nj->ni", e, xh), 0, atol=1e-15)
    # eq. def_of_phase_factor: |2 e_ij k_i k_j| / (1 - mu^2) = 1 for any khat
    k = rng.standard_normal((200, 3))
    k /= np.linalg.norm(k, axis=1)[:, None]
    mu = np.sum(k * xh, axis=1)
    ph = 2 * np.einsum("ni,nij,nj->n", k, e, k) / (1 - mu ** 2)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-12)
    # the phase is exp(2 i psi), psi the angle of k_perp from e_theta
    psi = np.arctan2(np.sum(k * ep, axis=1), np.sum(k * et, axis=1))
    assert np.allclose(ph, np.exp(2j * psi), atol=1e-12)
