"""Physics pins of the oracle (what the paper fixes, independent of any code path):

* LPP -> GPP: for a distant observer the local-plane-parallel estimators agree
  with the global-plane-parallel ones (Sec. III.A, eqs. lpp_dens, gpp_dens and
  Sec. IV.B case (c)).
* Known-spectrum recovery from a Gaussian tidal field with the validation
  spectra of Sec. IV.A (eq. power_for_validation), including the closed-form
  amplitudes 1/6, {2/15, -4/21, 2/35}, 1/420 and vanishing gd L=4, dd l=2,4.
* Closed-form shot noise: only the monopole of P_+ carries shape noise
  (Sec. V); its expectation is sum w^2 |gamma|^2 / I.
* B-modes of a pure linear tidal field vanish (Sec. II.C eq. relation_pm_EB).
"""
import numpy as np
import pytest

from oracle import estimator as E, mesh as M, special as S
from synth import lattice_catalogs, pure_noise_catalogs, Catalog, box_uniform
from physics_expect import _expected_lattice


def test_lpp_equals_gpp_for_distant_observer():
    rng = np.random.default_rng(21)
    nhat = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    box = 80.0
    D = 2.0e7
    centre = D * nhat
    origin = tuple(centre - box / 2)
    gp = box_uniform(400, rng, origin, box)
    rp = box_uniform(1200, rng, origin, box)
    g = Catalog(gp[:, 0], gp[:, 1], gp[:, 2], np.ones(400), np.full(400, 1e-3),
                rng.standard_normal(400), rng.standard_normal(400))
    r = Catalog(rp[:, 0], rp[:, 1], rp[:, 2], np.ones(1200), np.full(1200, 1e-3))
    cfg = E.Config(mesh=8, box=box, origin=origin, observer=(0.0, 0.0, 0.0), assignment=2,
                   interlacing=1, n_kbins=4, lmax=4)
    a = E.mesh64(g, r, cfg)
    b = E.gpp(g, r, cfg, nhat)
    assert a["series"] == b["series"]
    # scale: auto-power of the two fields in each product (before shot-noise subtraction)
    names = a["series"]
    pdd = a["re"][names.index("DD_l0")] + a["shot_dd"]
    ppp = a["re"][names.index("PLUS_l0")] + a["shot_plus"]
    for i, s in enumerate(names):
        scale = pdd if s.startswith("DD") else (np.sqrt(np.abs(pdd * ppp)) if s.startswith("GD") else ppp)
        sel = a["n_modes"] > 0
        assert np.all(np.abs(a["re"][i] - b["re"][i])[sel] <= 1e-4 * np.abs(scale[sel])), s
        assert np.all(np.abs(a["im"][i] - b["im"][i])[sel] <= 1e-4 * np.abs(scale[sel])), s


@pytest.mark.slow
def test_known_spectrum_recovery_tidal_field():
    n, box = 16, 800.0
    nhat = np.array([0.6, 0.48, 0.64])
    D = 1.0e7
    origin = tuple(D * nhat - box / 2)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=(0.0, 0.0, 0.0), assignment=1,
                   interlacing=0, compensate=0, n_kbins=8, lmax=4)
    amp = 0.5
    runs = []
    for seed in range(24):
        g, r, s = lattice_catalogs(n, box, origin, (0.0, 0.0, 0.0), seed, delta_rms=0.1, amp=amp)
        res = E.mesh64(g, r, cfg)
        v = dict(zip(res["series"], res["re"]))
        v["DD_l0"] = v["DD_l0"] + res["shot_dd"]      # the lattice has no Poisson noise
        v["PLUS_l0"] = v["PLUS_l0"] + res["shot_plus"]
        runs.append((v, s, res["alpha"]))
    s2 = np.mean([x[1] ** 2 / x[2] for x in runs])
    exp = _expected_lattice(cfg, s2, amp, nhat)
    ok = res["n_modes"] >= 20
    for key in ("DD_l0", "DD_l2", "DD_l4", "GD_L2", "GD_L4", "PLUS_l0", "PLUS_l2", "PLUS_l4", "MINUS_L4"):
        arr = np.array([x[0][key] * (s2 / (x[1] ** 2 / x[2])) for x in runs])
        mean = arr.mean(axis=0)
        err = arr.std(axis=0, ddof=1) / np.sqrt(len(runs))
        scale = np.abs(exp["DD_l0"]) * (amp if key.startswith("GD") else (amp ** 2 if key[0] in "PM" else 1))
        dev = np.abs(mean - exp[key])
        assert np.all(dev[ok] <= 4.0 * err[ok] + 1e-3 * scale[ok]), (key, dev[ok], err[ok])


def test_shell_expectation_approaches_paper_amplitudes():
    """The exact discrete-shell expectation used above tends to the continuum
    amplitudes of eq. xi_relations_normalization_coefficients on shells with
    many modes (1/6 for gd L=2, 2/15, -4/21, 2/35 for +, 1/420 for -)."""
    n, box = 32, 800.0
    nhat = np.array([0.6, 0.48, 0.64])
    cfg = E.Config(mesh=n, box=box, origin=(0.0, 0.0, 0.0), assignment=1, interlacing=0, compensate=0,
                   n_kbins=8, lmax=4)
    amp = 1.0
    exp = _expected_lattice(cfg, 1.0, amp, nhat)
    big = M.mode_counts(n, 8, *cfg.bin_width()) > 2000
    for key, c, tol in (("GD_L2", -1 / 6, 0.01), ("PLUS_l0", 2 / 15, 0.01), ("PLUS_l2", -4 / 21, 0.01),
                        ("PLUS_l4", 2 / 35, 0.08), ("MINUS_L4", 1 / 420, 0.01)):
        assert np.allclose(exp[key][big], c * exp["DD_l0"][big], rtol=tol), key
    assert np.all(np.abs(exp["GD_L4"][big]) < 0.01 * np.abs(exp["GD_L2"][big]))
    assert np.all(np.abs(exp["DD_l2"][big]) < 0.01 * exp["DD_l0"][big])


def test_shot_noise_closed_form_pure_noise():
    """Uniform positions with pure shape noise: after subtracting N_+ the P_+ monopole
    and every other shape moment average to zero."""
    n, box, sigma = 12, 200.0, 0.3
    origin = (500.0, 300.0, 200.0)
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=2, interlacing=1, n_kbins=6, lmax=4,
                   families=("GD", "PLUS", "MINUS"))
    vals = {k: [] for k in ("PLUS_l0", "PLUS_l2", "MINUS_L4", "GD_L2")}
    for seed in range(16):
        g, r = pure_noise_catalogs(3000, 6000, origin, box, sigma, seed)
        res = E.mesh64(g, r, cfg)
        d = dict(zip(res["series"], res["re"]))
        for k in vals:
            vals[k].append(d[k])
        npl = res["shot_plus"]
        assert abs(npl - 2 * sigma ** 2 * np.sum(g.w ** 2) / res["norm_I"]) < 0.1 * npl
    for k, v in vals.items():
        v = np.array(v)[:, 1:]      # bin 0 holds only the DC mode
        m = v.mean()
        err = v.std(ddof=1) / np.sqrt(v.size)
        assert abs(m) < 4 * err + 1e-3 * npl, (k, m, err)


@pytest.mark.slow
def test_b_modes_vanish_for_linear_tidal_field():
    n, box = 16, 800.0
    nhat = np.array([0.0, 0.6, 0.8])
    D = 1.0e7
    origin = tuple(D * nhat - box / 2)
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=1, interlacing=0, compensate=0,
                   n_kbins=8, lmax=4, families=("PLUS", "MINUS"))
    bb, ee = [], []
    for seed in range(6):
        g, r, s = lattice_catalogs(n, box, origin, (0.0, 0.0, 0.0), 100 + seed, amp=1.0)
        res = E.mesh64(g, r, cfg)
        d = dict(zip(res["series"], res["re"]))
        d["PLUS_l0"] = d["PLUS_l0"] + res["shot_plus"]
        # recompute EE/BB monopole with the noise-free P_+ monopole
        b0 = 0.5 * (d["PLUS_l0"] - 56 * d["MINUS_L4"])
        e0 = 0.5 * (d["PLUS_l0"] + 56 * d["MINUS_L4"])
        bb.append(b0)
        ee.append(e0)
    bb, ee = np.array(bb), np.array(ee)
    big = res["n_modes"] > 400
    # realisation by realisation: P_+ = P_- per mode for a pure E field, so BB is only the
    # discreteness of the shell average (the mu-moments of a finite mode set)
    assert np.all(np.abs(bb[:, big]) < 0.05 * np.abs(ee[:, big]))
