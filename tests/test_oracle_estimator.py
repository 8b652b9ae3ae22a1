"""Pins of the oracle estimator: the mesh definitions (assignment weights,
mass conservation, mode counts by brute-force enumeration), Parseval, and the
agreement of two independent routes (defining double sum vs. the FFT route
with Cartesian tensors) on tiny inputs."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import estimator as E, mesh as M
from synth import Catalog, box_uniform


def _cats(rng, ng, nr, origin, box, noise=1.0):
    gp = box_uniform(ng, rng, origin, box)
    rp = box_uniform(nr, rng, origin, box)
    g = Catalog(gp[:, 0], gp[:, 1], gp[:, 2], rng.random(ng) + 0.5, np.full(ng, 2e-3),
                noise * rng.standard_normal(ng), noise * rng.standard_normal(ng))
    r = Catalog(rp[:, 0], rp[:, 1], rp[:, 2], rng.random(nr) + 0.5, np.full(nr, 2e-3))
    return g, r


@pytest.mark.parametrize("p", [1, 2, 3])
def test_assignment_weights_sum_to_one_and_closed_forms(p):
    u = np.linspace(0.0, 5.0, 101)
    c, w = M.stencil_1d(u, p)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-15)
    # first moment is preserved by CIC and TSC (sum w c = u)
    if p > 1:
        assert np.allclose((w * c).sum(axis=1), u, atol=1e-13)
    if p == 3:  # TSC at a node: (1/8, 3/4, 1/8); halfway between nodes 2 and 3: (1/2, 1/2, 0) at nodes 2, 3, 4
        c0, w0 = M.stencil_1d(np.array([2.0, 2.5]), 3)
        assert np.allclose(w0[0], [0.125, 0.75, 0.125]) and list(c0[0]) == [1, 2, 3]
        assert np.allclose(w0[1], [0.5, 0.5, 0.0]) and list(c0[1]) == [2, 3, 4]


def test_deposit_mass_conservation():
    rng = np.random.default_rng(0)
    pos = box_uniform(3000, rng, (10.0, -5.0, 7.0), 64.0)
    v = rng.random(3000) + 1j * rng.random(3000)
    for p in (1, 2, 3):
        for sh in (0.0, 0.5):
            d = M.deposit(pos, v, 16, 64.0, (10.0, -5.0, 7.0), p, shift=sh)
            assert abs(d.sum() - v.sum()) < 1e-10


def _bins_by_enumeration(n, nb, num, den):
    """Bin of each integer mode by exact comparison |n| in [b dn, (b+1) dn)."""
    dn = Fraction(num, den)
    counts = [0] * nb
    half = n // 2
    rng_ = [i if i < half else i - n for i in range(n)]
    for a in rng_:
        for b in rng_:
            for c in rng_:
                q = a * a + b * b + c * c
                if q == 0:
                    continue
                for j in range(nb):
                    lo2, hi2 = (j * dn) ** 2, ((j + 1) * dn) ** 2
                    if lo2 <= q < hi2:
                        counts[j] += 1
                        break
    return counts


@pytest.mark.parametrize("n,nb,dn", [(8, 4, None), (12, 5, None), (16, 10, (16, 20)), (10, 3, (7, 5))])
def test_mode_counts_bit_exact(n, nb, dn):
    num, den = dn if dn else M.default_dn(n, nb)
    got = M.mode_counts(n, nb, num, den)
    assert list(got) == _bins_by_enumeration(n, nb, num, den)


def test_default_bin_width_rationals():
    # Delta k / k_f for the workloads: 32^3/16 -> 1, 512^3/50 -> 128/25, 256^3/50 -> 64/25, 1024^3/80 -> 32/5
    assert M.default_dn(32, 16) == (1, 1)
    assert M.default_dn(512, 50) == (128, 25)
    assert M.default_dn(256, 50) == (64, 25)
    assert M.default_dn(1024, 80) == (32, 5)


@pytest.mark.parametrize("p,il,comp", [(1, 0, 0), (2, 0, 1), (3, 1, 1), (2, 1, 0)])
def test_brute_definition_equals_fft_route(p, il, comp):
    rng = np.random.default_rng(10 + p + il)
    origin, box = (300.0, 200.0, 250.0), 100.0
    g, r = _cats(rng, 150, 500, origin, box)
    cfg = E.Config(mesh=8, box=box, origin=origin, assignment=p, interlacing=il, compensate=comp,
                   n_kbins=4, lmax=4)
    a = E.brute(g, r, cfg)
    b = E.mesh64(g, r, cfg)
    assert list(a["n_modes"]) == list(b["n_modes"])
    scale = np.abs(a["re"]).max(axis=1, keepdims=True)
    assert np.all(np.abs(a["re"] - b["re"]) <= 1e-11 * scale)
    assert np.all(np.abs(a["im"] - b["im"]) <= 1e-11 * scale)


def test_brute_equals_fft_route_lmax8_near_observer():
    # the higher multipoles (L = 6, 8) and a wide-angle geometry (observer near the box)
    rng = np.random.default_rng(77)
    origin, box = (20.0, -30.0, 10.0), 60.0
    g, r = _cats(rng, 100, 300, origin, box)
    cfg = E.Config(mesh=8, box=box, origin=origin, assignment=2, interlacing=1, n_kbins=4, lmax=8)
    a = E.brute(g, r, cfg)
    b = E.mesh64(g, r, cfg)
    scale = np.abs(a["re"]).max(axis=1, keepdims=True)
    assert np.all(np.abs(a["re"] - b["re"]) <= 1e-10 * scale)


def test_parseval_monopole_normalisation():
    """sum_b N_b (P_dd^(0) + N_dd) I = sum_{k binned} |F(k)|^2 and, with bins covering
    every non-zero mode, = N^3 sum_c D_c^2 - |F(0)|^2 (NGP, no compensation)."""
    rng = np.random.default_rng(5)
    origin, box, n = (0.0, 0.0, 0.0), 50.0, 8
    g, r = _cats(rng, 300, 900, origin, box)
    # dn = 1 with 12 bins reaches |n|^2 < 144 > 3 * 16: every mode is binned
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=1, interlacing=0, compensate=0,
                   n_kbins=12, dn=(1, 1), lmax=0, families=("DD",))
    res = E.mesh64(g, r, cfg)
    assert res["n_modes"].sum() == n ** 3 - 1
    lhs = np.sum(res["n_modes"] * (res["re"][0] + res["shot_dd"])) * res["norm_I"]
    sc = E.scalars(g, r)
    D = M.deposit(np.concatenate([g.pos(), r.pos()]), np.concatenate([g.w, -sc["alpha"] * r.w]),
                  n, box, origin, 1)
    rhs = n ** 3 * np.sum(D ** 2) - abs(D.sum()) ** 2
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_scalars_closed_forms():
    rng = np.random.default_rng(2)
    g, r = _cats(rng, 100, 400, (0, 0, 0), 10.0)
    sc = E.scalars(g, r)
    alpha = g.w.sum() / r.w.sum()
    I = alpha * np.sum(r.w ** 2 * r.nbar)
    assert math.isclose(sc["alpha"], alpha) and math.isclose(sc["norm_I"], I)
    assert math.isclose(sc["shot_plus"], np.sum(g.w ** 2 * (g.g1 ** 2 + g.g2 ** 2)) / I)
    assert math.isclose(sc["shot_dd"], (np.sum(g.w ** 2) + alpha ** 2 * np.sum(r.w ** 2)) / I)


def test_invariance_under_basis_rotation():
    """Rotating every object's (e_theta, e_phi) by psi multiplies gamma by exp(-2 i psi)
    and e_ij by exp(2 i psi): the products gamma e*_ij, hence all spectra, are unchanged.
    Checked by rotating the whole configuration about the observer's z axis, which
    moves positions and re-expresses the same physical shapes in the new local basis
    (the basis of eq. def_standard_rotation rotates rigidly about z)."""
    rng = np.random.default_rng(9)
    origin, box = (100.0, 120.0, 40.0), 40.0
    g, r = _cats(rng, 120, 400, origin, box)
    cfg = E.Config(mesh=8, box=box, origin=origin, assignment=2, interlacing=0, n_kbins=4, lmax=4)
    a = E.mesh64(g, r, cfg)
    # rotate by 90 degrees about z: (x, y) -> (-y, x); the mesh maps onto itself when the box is
    # rotated with it, so rotate the box origin too and keep modes' bins (|n| is invariant)
    def rot(c):
        return Catalog(-c.y, c.x, c.z, c.w, c.nbar, c.g1, c.g2)
    o2 = (-(origin[1] + box), origin[0], origin[2])
    g2, r2 = rot(g), rot(r)
    # keep objects off the mesh boundary ambiguity: shift by a tiny amount inside the box
    cfg2 = E.Config(mesh=8, box=box, origin=o2, assignment=2, interlacing=0, n_kbins=4, lmax=4)
    b = E.mesh64(g2, r2, cfg2)
    scale = np.abs(a["re"]).max(axis=1, keepdims=True)
    # the rotated mesh is the original mesh up to a one-cell reindexing of the x axis; the
    # binned spectra of a rigidly rotated configuration agree up to that node offset
    assert np.all(np.abs(a["re"] - b["re"]) <= 1e-9 * scale)
