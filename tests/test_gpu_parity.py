"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 path <= 1e-9 of the per-bin scale; FP32 path <= 1e-4 of the
per-bin scale, where the scale of a series is the auto power of the fields
in its product before shot-noise subtraction (DD: P_dd^(0) + N_dd; PLUS,
MINUS, EE, BB: P_+^(0) + N_+; GD: their geometric mean).  In addition the
real part (the spectrum) of every series is held to the same tolerance
relative to its own value, on every bin where that value is at least
OWN_FLOOR (1e-2) of the scale: a weak series (an l = 4 moment, MINUS_L4, a
B-mode) is then checked against itself and not only against the auto power.
Mode counts are compared bit-exactly.
"""
import numpy as np
import pytest

from oracle import estimator as E, mesh as M
from synth import Catalog, box_uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lpp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2202_11839_amd as pkg
    pkg.load()
    return pkg


def _cats(seed, ng, nr, origin, box, wfun=True, margin=0.0):
    rng = np.random.default_rng(seed)
    o = np.asarray(origin) + margin
    gp = box_uniform(ng, rng, o, box - 2 * margin)
    rp = box_uniform(nr, rng, o, box - 2 * margin)
    w_g = rng.random(ng) + 0.5 if wfun else np.ones(ng)
    w_r = rng.random(nr) + 0.5 if wfun else np.ones(nr)
    g = Catalog(gp[:, 0], gp[:, 1], gp[:, 2], w_g, np.full(ng, 2e-3), 0.3 * rng.standard_normal(ng),
                0.3 * rng.standard_normal(ng))
    r = Catalog(rp[:, 0], rp[:, 1], rp[:, 2], w_r, np.full(nr, 2e-3))
    return g, r


def _scales(ref):
    s = ref["series"]
    dd = ref["re"][s.index("DD_l0")] + ref["shot_dd"] if "DD_l0" in s else None
    pp = ref["re"][s.index("PLUS_l0")] + ref["shot_plus"] if "PLUS_l0" in s else None
    out = []
    for name in s:
        if name.startswith("DD"):
            out.append(np.abs(dd))
        elif name.startswith("GD"):
            out.append(np.sqrt(np.abs(dd * pp)))
        else:
            out.append(np.abs(pp))
    return np.array(out)


def _compare(got, ref, tol):
    assert got["series"] == ref["series"]
    assert list(got["n_modes"]) == list(ref["n_modes"]), (got["n_modes"], ref["n_modes"])
    for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran"):
        assert abs(got[k] - ref[k]) <= 1e-10 * abs(ref[k]), k
    np.testing.assert_allclose(got["k_lo"], ref["k_lo"], rtol=1e-13)
    sel = ref["n_modes"] > 0
    # k_eff is an FP64 sum of |k| over up to ~2e6 modes of a shell at 512^3,
    # summed in another order on the device: relative rounding up to ~N u
    np.testing.assert_allclose(got["k_eff"][sel], ref["k_eff"][sel], rtol=1e-10)
    sc = _scales(ref)
    err_re = np.abs(got["re"] - ref["re"])[:, sel] / sc[:, sel]
    err_im = np.abs(got["im"] - ref["im"])[:, sel] / sc[:, sel]
    worst = max(err_re.max(), err_im.max())
    if worst > tol:
        i, b = np.unravel_index(np.argmax(np.maximum(err_re, err_im)), err_re.shape)
        raise AssertionError(f"series {ref['series'][i]} bin {b}: rel err {worst:.3e} > {tol:.1e}")
    own = _own_errors(got, ref)
    bad = {k: v for k, v in own.items() if v > tol}
    if bad:
        raise AssertionError(f"error relative to the series' own value above {tol:.1e}: {bad}")
    return worst


OWN_FLOOR = 1e-2


def _own_errors(got, ref):
    """Largest |GPU - oracle| / |oracle| of each series' real part over the
    bins with modes where |oracle| >= OWN_FLOOR * scale (0 if there is none)."""
    sc = _scales(ref)
    sel = ref["n_modes"] > 0
    out = {}
    for i, name in enumerate(ref["series"]):
        r = np.asarray(ref["re"][i])
        m = sel & (np.abs(r) >= OWN_FLOOR * sc[i])
        out[name] = float((np.abs(np.asarray(got["re"][i]) - r)[m] / np.abs(r[m])).max()) if m.any() else 0.0
    return out


# ---------------------------------------------------------------------------
# building blocks

@pytest.mark.parametrize("n", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fft3d_matches_numpy(lpp, n, prec):
    import torch
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    dt = torch.complex128 if prec == "f64" else torch.complex64
    t = torch.tensor(a, dtype=dt, device="cuda").contiguous()
    plan = lpp.Plan(n, 1.0, (0.0, 0.0, 0.0), (-1.0, -1.0, -1.0), precision=prec, n_kbins=1)
    plan.fft3d(t)
    want = np.fft.fftn(a)
    got = t.cpu().numpy()
    rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert rel < (1e-12 if prec == "f64" else 3e-6), rel


def _to_zblocked(t, n):
    """[z][y][x] tensor -> the estimator's z-blocked order ((z/8 N + y) N + x) 8 + z%8."""
    return t.reshape(n // 8, 8, n, n).permute(0, 2, 3, 1).contiguous()


def _from_zblocked(t, n):
    return t.permute(0, 3, 1, 2).reshape(n, n, n).contiguous()


@pytest.mark.parametrize("n,prec", [(512, "f64"), (512, "f32")])
def test_fft3d_zblocked_matches_scipy(lpp, n, prec):
    """The estimator's z-blocked 3D transform (x, y and z passes of
    fft_zb_kernel with the estimator's launch shapes, nothing pruned) on a
    random 512^3 mesh against scipy's FP64 FFT."""
    import scipy.fft as sfft
    import torch
    rng = np.random.default_rng(n + 1)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    dt = torch.complex128 if prec == "f64" else torch.complex64
    t = _to_zblocked(torch.tensor(a, dtype=dt, device="cuda"), n)
    plan = lpp.Plan(n, 1.0, (0.0, 0.0, 0.0), (-1.0, -1.0, -1.0), precision=prec, n_kbins=1)
    plan.fft3d_zblocked(t)
    got = _from_zblocked(t, n).cpu().numpy()
    del t
    want = sfft.fftn(a, workers=16)
    rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert rel < (1e-12 if prec == "f64" else 3e-6), rel


def test_fft3d_zblocked_1024_matches_plain_layout(lpp):
    """At 1024^3 (FP32) the z-blocked transform against the plain-layout one
    (fft_axis_kernel, itself checked against numpy above): two different
    kernels and memory orders, the same DFT."""
    import torch
    n = 1024
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1024)
    plain = torch.complex(torch.randn((n, n, n), generator=gen, device="cuda"),
                          torch.randn((n, n, n), generator=gen, device="cuda"))
    zb = _to_zblocked(plain, n)
    plan = lpp.Plan(n, 1.0, (0.0, 0.0, 0.0), (-1.0, -1.0, -1.0), precision="f32", n_kbins=1)
    plan.fft3d(plain)
    plan.fft3d_zblocked(zb)
    back = _from_zblocked(zb, n)
    del zb
    diff = float((back - plain).abs().max())
    scale = float(plain.abs().max())
    assert diff <= 3e-6 * scale, diff / scale


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("il", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_deposit_matches_oracle(lpp, p, il, prec):
    import torch
    n, box, origin = 32, 64.0, (-7.0, 3.0, 11.0)
    g, _ = _cats(100 + p, 5000, 10, origin, box)
    plan = lpp.Plan(n, box, origin, (-100.0, -100.0, -100.0), assignment=p, interlacing=il, precision=prec,
                    n_kbins=4)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    mesh = torch.empty((n, n, n), dtype=dt, device="cuda")
    plan.deposit_weights(g, -0.75, mesh)
    got = mesh.cpu().numpy().transpose(2, 1, 0)  # [z, y, x] -> [x, y, z]
    pos = g.pos()
    want = M.deposit(pos, -0.75 * g.w, n, box, origin, p)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert np.max(np.abs(got.real - want)) <= tol * np.max(np.abs(want))
    if il:
        want2 = M.deposit(pos, -0.75 * g.w, n, box, origin, p, shift=0.5)
        assert np.max(np.abs(got.imag - want2)) <= tol * np.max(np.abs(want2))
    else:
        assert np.all(got.imag == 0)


@pytest.mark.parametrize("p,il,prec", [(3, 1, "f32"), (2, 0, "f32"), (3, 1, "f64"), (2, 0, "f64"), (1, 1, "f64")])
def test_dense_deposit_in_chunks_matches_oracle(lpp, p, il, prec):
    """About 15 objects per cell: a tile's region holds ~12,000 objects,
    which the deposit stages in ~24 chunks, every region row giving each
    chunk an equal share of its objects; the mesh against the oracle's.
    (NGP in FP32 is left out: the staged region coordinate, cell plus offset
    in one float, resolves the half-cell boundary of the nearest node to
    ~1e-6 of a cell, and among 60,000 objects one lies that close to it.)"""
    import torch
    n, box, origin = 16, 64.0, (5.0, -9.0, 2.0)
    g, _ = _cats(200 + p, 60000, 10, origin, box)
    plan = lpp.Plan(n, box, origin, (-100.0, -100.0, -100.0), assignment=p, interlacing=il, precision=prec,
                    n_kbins=4)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    mesh = torch.empty((n, n, n), dtype=dt, device="cuda")
    plan.deposit_weights(g, 0.5, mesh)
    got = mesh.cpu().numpy().transpose(2, 1, 0)
    pos = g.pos()
    want = M.deposit(pos, 0.5 * g.w, n, box, origin, p)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert np.max(np.abs(got.real - want)) <= tol * np.max(np.abs(want))
    if il:
        want2 = M.deposit(pos, 0.5 * g.w, n, box, origin, p, shift=0.5)
        assert np.max(np.abs(got.imag - want2)) <= tol * np.max(np.abs(want2))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_maximum_shell_count_matches_oracle(lpp, prec):
    """The largest number of k-shells (256, of width 1/8 of the fundamental
    mode on a 64^3 mesh, up to its Nyquist frequency): the shell sums of a
    launch then hold 2 n 256 rows per wavefront, which limits a launch to
    four fields; counts bit-exact and every series against the oracle."""
    n, box, origin, obs = 64, 400.0, (300.0, 200.0, 250.0), (0.0, 0.0, 0.0)
    g, r = _cats(37, 3000, 9000, origin, box)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=obs, assignment=3, interlacing=1, n_kbins=256,
                   dn=(1, 8), lmax=4)
    ref = E.mesh64(g, r, cfg)
    plan = lpp.Plan(n, box, origin, obs, assignment=3, interlacing=1, precision=prec, lmax=4, n_kbins=256,
                    dn=(1, 8))
    _compare(plan.estimate(g, r), ref, 1e-9 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dense_estimate_matches_oracle(lpp, prec):
    """A dense catalog pair (2,000 galaxies and 40,000 randoms on a 16^3
    mesh, ~10 density objects per cell, so the density passes stage each tile
    in several chunks): every series against the oracle."""
    n, box, origin, obs = 16, 100.0, (300.0, 200.0, 250.0), (0.0, 0.0, 0.0)
    g, r = _cats(31, 2000, 40000, origin, box)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=obs, assignment=3, interlacing=1, n_kbins=6, lmax=4)
    ref = E.mesh64(g, r, cfg)
    plan = lpp.Plan(n, box, origin, obs, assignment=3, interlacing=1, precision=prec, lmax=4, n_kbins=6)
    _compare(plan.estimate(g, r), ref, 1e-9 if prec == "f64" else 1e-4)


# ---------------------------------------------------------------------------
# the whole estimator

CASES = [
    # (mesh, box, origin, observer, p, il, comp, lmax, nb, ng, nr)
    (16, 100.0, (300.0, 200.0, 250.0), (0.0, 0.0, 0.0), 3, 1, 1, 4, 6, 800, 3000),
    (32, 150.0, (300.0, 200.0, 250.0), (0.0, 0.0, 0.0), 2, 0, 1, 4, 10, 3000, 9001),
    (32, 80.0, (20.0, -30.0, 10.0), (0.0, 0.0, 0.0), 3, 1, 1, 4, 16, 2001, 7003),   # wide angle, near observer
    (16, 60.0, (-30.0, -30.0, 5.0), (0.0, 0.0, 0.0), 1, 0, 0, 4, 8, 500, 1500),     # NGP, no compensation
    (16, 60.0, (40.0, -70.0, -20.0), (0.0, 0.0, 0.0), 2, 1, 1, 8, 8, 700, 2100),    # lmax = 8
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_estimate_matches_oracle(lpp, case, prec):
    n, box, origin, obs, p, il, comp, lmax, nb, ng, nr = CASES[case]
    g, r = _cats(7 + case, ng, nr, origin, box)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=obs, assignment=p, interlacing=il, compensate=comp,
                   lmax=lmax, n_kbins=nb)
    ref = E.mesh64(g, r, cfg)
    plan = lpp.Plan(n, box, origin, obs, assignment=p, interlacing=il, compensate=comp, precision=prec, lmax=lmax,
                    n_kbins=nb)
    got = plan.estimate(g, r)
    _compare(got, ref, 1e-9 if prec == "f64" else 1e-4)


def _footprint_cats(seed, ng, nr, pts):
    rng = np.random.default_rng(seed)
    gp, rp = pts(ng, rng), pts(nr, rng)
    g = Catalog(gp[:, 0], gp[:, 1], gp[:, 2], rng.random(ng) + 0.5, np.full(ng, 2e-3), 0.3 * rng.standard_normal(ng),
                0.3 * rng.standard_normal(ng))
    r = Catalog(rp[:, 0], rp[:, 1], rp[:, 2], rng.random(nr) + 0.5, np.full(nr, 2e-3))
    return g, r


_FOOTPRINT_REF = {}


def _footprint_case(layout):
    """(catalogs, plan arguments, oracle result) of a compact-footprint case, cached."""
    from synth import wedge_uniform
    if layout not in _FOOTPRINT_REF:
        if layout == "wedge":
            n, box, origin, p, il = 64, 400.0, (20.0, 20.0, 0.0), 3, 1
            pts = lambda k, rng: wedge_uniform(k, rng, (10.0, 60.0), (5.0, 35.0), (300.0, 420.0))
        else:
            n, box, origin, p, il = 32, 200.0, (300.0, 100.0, 150.0), 2, 1

            def pts(k, rng):
                u = box_uniform(k, rng, (0.0, 0.0, 0.0), 1.0)
                y = np.where(u[:, 1] < 0.5, 2.0 * u[:, 1] * 9.0, box - 2.0 * (u[:, 1] - 0.5) * 9.0 - 1e-9)
                return np.stack([origin[0] + 20.0 + 60.0 * u[:, 0], origin[1] + y,
                                 origin[2] + 40.0 + 100.0 * u[:, 2]], axis=1)
        g, r = _footprint_cats(11, 2500, 9000, pts)
        cfg = E.Config(mesh=n, box=box, origin=origin, assignment=p, interlacing=il, lmax=4, n_kbins=12)
        _FOOTPRINT_REF[layout] = (g, r, dict(mesh_n=n, box_size=box, box_origin=origin, assignment=p,
                                             interlacing=il, lmax=4, n_kbins=12), E.mesh64(g, r, cfg))
    return _FOOTPRINT_REF[layout]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_distant_observer_matches_global_plane_parallel(lpp, prec):
    """A physics pin of the GPU path that does not go through the oracle's LPP
    code: for an observer 2e7 Mpc/h away the local lines of sight are all
    parallel to nhat, and the LPP multipoles equal the global-plane-parallel
    ones computed from Gamma = gamma exp(-2 i phi_{k,n}) (Sec. III.A, eqs.
    lpp_dens and gpp_dens; Sec. IV.B case (c)), to 1e-4 of each series' scale
    (the endpoint directions differ from nhat by < 1e-5)."""
    nhat = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    box, n = 80.0, 16
    origin = tuple(2.0e7 * nhat - box / 2)
    g, r = _cats(21, 600, 1800, origin, box, wfun=False)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=(0.0, 0.0, 0.0), assignment=2, interlacing=1,
                   n_kbins=6, lmax=4)
    ref = E.gpp(g, r, cfg, nhat)
    plan = lpp.Plan(n, box, origin, (0.0, 0.0, 0.0), assignment=2, interlacing=1, precision=prec, lmax=4,
                    n_kbins=6)
    got = plan.estimate(g, r)
    assert got["series"][:len(ref["series"])] == ref["series"]
    assert list(got["n_modes"]) == list(ref["n_modes"])
    sc = _scales(ref)
    sel = ref["n_modes"] > 0
    for i, name in enumerate(ref["series"]):
        for part in ("re", "im"):
            err = np.abs(np.asarray(got[part][i]) - ref[part][i])[sel] / sc[i][sel]
            assert err.max() <= 1e-4, (name, part, err.max())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_objects_on_the_pole_axis_match_oracle(lpp, prec):
    """The pole edge case of the line-of-sight basis: a fifth of the galaxies
    lie on the z-axis through the observer (sin theta = 0 exactly, half of
    them above it, theta = 0, half below, theta = pi), where phi is taken as
    0, so their shapes are read in the basis (e_theta, e_phi) = (+-x, y)
    (App. E, eq. def_standard_rotation).  The axis is a cell boundary of the
    mesh (x = y = 0 with the origin at -50 and H = 6.25), so that the
    device's position, rebuilt from the cell and the offset in it, is exactly
    on the axis too; every series against the oracle."""
    box, n = 100.0, 16
    origin = (-50.0, -50.0, -50.0)
    obs = (0.0, 0.0, 0.0)
    g, r = _cats(29, 600, 2000, origin, box)
    rng = np.random.default_rng(290)
    on = rng.choice(g.n, size=g.n // 5, replace=False)
    g.x[on] = 0.0
    g.y[on] = 0.0
    g.z[on] = rng.uniform(5.0, 45.0, on.size) * np.where(np.arange(on.size) % 2 == 0, 1.0, -1.0)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=obs, assignment=3, interlacing=1, n_kbins=6, lmax=4)
    ref = E.mesh64(g, r, cfg)
    plan = lpp.Plan(n, box, origin, obs, assignment=3, interlacing=1, precision=prec, lmax=4, n_kbins=6)
    _compare(plan.estimate(g, r), ref, 1e-9 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_global_line_of_sight_matches_oracle_gpp(lpp, prec):
    """The plan's global-line-of-sight mode against the oracle's
    global-plane-parallel estimator (Sec. II.C), with the observer inside the
    box and one galaxy placed exactly on it: the observer plays no part."""
    nhat = np.array([2.0, -1.0, 2.0]) / 3.0
    box, n = 120.0, 16
    origin = (10.0, -20.0, 30.0)
    g, r = _cats(23, 700, 2100, origin, box)
    obs = np.asarray(origin) + box / 2
    g.x[0], g.y[0], g.z[0] = obs
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=tuple(obs), assignment=3, interlacing=1,
                   n_kbins=6, lmax=4)
    ref = E.gpp(g, r, cfg, nhat)
    plan = lpp.Plan(n, box, origin, tuple(obs), assignment=3, interlacing=1, precision=prec, lmax=4,
                    n_kbins=6, los=tuple(3.0 * nhat))
    got = plan.estimate(g, r)
    assert got["series"][:len(ref["series"])] == ref["series"]
    assert list(got["n_modes"]) == list(ref["n_modes"])
    sc = _scales(ref)
    sel = ref["n_modes"] > 0
    tol = 1e-9 if prec == "f64" else 1e-4
    for i, name in enumerate(ref["series"]):
        for part in ("re", "im"):
            err = np.abs(np.asarray(got[part][i]) - ref[part][i])[sel] / sc[i][sel]
            assert err.max() <= tol, (name, part, err.max())
    # the same catalogs with each object's own line of sight are refused (a galaxy at the observer)
    local = lpp.Plan(n, box, origin, tuple(obs), assignment=3, interlacing=1, precision=prec, lmax=4, n_kbins=6)
    with pytest.raises(lpp.LppError) as e:
        local.estimate(g, r)
    assert e.value.status == 4  # LPP_E_AT_OBSERVER


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["wedge", "wrapped_slabs"])
def test_estimate_compact_footprint(lpp, layout, prec):
    """Catalogs that cover a small part of the box, so that most node rows,
    tile-rows and planes are outside the footprint and skipped by the
    deposit and the transforms: a survey wedge (RA 10-60, Dec 5-35 deg,
    r 300-420) in a 64^3 box, and two thin slabs at both ends of the y range
    whose stencils wrap around the periodic boundary."""
    g, r, kw, ref = _footprint_case(layout)
    plan = lpp.Plan(precision=prec, **kw)
    got = plan.estimate(g, r)
    worst = _compare(got, ref, 1e-9 if prec == "f64" else 1e-4)
    print(f"{layout} {prec}: worst rel err {worst:.2e}")


def test_estimate_spectra_subsets(lpp):
    n, box, origin = 16, 90.0, (100.0, 50.0, -40.0)
    g, r = _cats(55, 900, 2500, origin, box)
    for fams, mask in ((("DD",), 1), (("GD",), 2), (("PLUS",), 4), (("PLUS", "MINUS"), 12), (("DD", "GD"), 3)):
        cfg = E.Config(mesh=n, box=box, origin=origin, assignment=3, interlacing=1, lmax=4, n_kbins=6,
                       families=fams)
        ref = E.mesh64(g, r, cfg)
        plan = lpp.Plan(n, box, origin, assignment=3, interlacing=1, precision="f64", lmax=4, n_kbins=6, spectra=mask)
        got = plan.estimate(g, r)
        assert got["series"] == ref["series"]
        sel = ref["n_modes"] > 0
        for i, s in enumerate(ref["series"]):
            sc = np.abs(ref["re"][i][sel]).max() + 1e-300
            assert np.max(np.abs(got["re"][i] - ref["re"][i])[sel]) <= 1e-9 * sc, (fams, s)


def test_c1_workload_fp64_and_fp32(lpp):
    """The 32^3 plain-estimator workload (5,000 galaxies from a GRF with tidal shapes,
    50,000 randoms, CIC, l <= 4, 16 bins) against the oracle."""
    from synth import WORKLOADS, make_catalogs
    wl = WORKLOADS["c1"]
    g, r = make_catalogs(wl, mock=0)
    cfg = E.Config(mesh=wl["mesh"], box=wl["box"], origin=wl["origin"], observer=wl["observer"],
                   assignment=wl["assignment"], interlacing=wl["interlacing"], lmax=4, n_kbins=wl["n_kbins"])
    ref = E.mesh64(g, r, cfg)
    for prec, tol in (("f64", 1e-9), ("f32", 1e-4)):
        plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                        interlacing=wl["interlacing"], precision=prec, lmax=4, n_kbins=wl["n_kbins"])
        got = plan.estimate(g, r)
        worst = _compare(got, ref, tol)
        print(f"c1 {prec}: worst rel err {worst:.2e}")


def _series_errors(got, ref):
    """Largest |GPU - oracle| / scale of each series over the shells with modes (re and im)."""
    sc = _scales(ref)
    sel = ref["n_modes"] > 0
    return {name: float(max((np.abs(np.asarray(got[part][i]) - ref[part][i])[sel] / sc[i][sel]).max()
                            for part in ("re", "im")))
            for i, name in enumerate(ref["series"])}


def test_per_multipole_error_table(lpp):
    """The error of every multipole against the oracle, per precision, on the
    32^3 workload and the 64^3 wedge: each within its tolerance (FP64 1e-9,
    FP32 1e-4) relative to the series' scale, and relative to its own value
    on the bins where that is at least OWN_FLOOR of the scale (the columns
    ending in _own).  The table is printed (pytest -s) and, if LPP_ERROR_TABLE
    names a file, written there as JSON."""
    import json
    import os
    from synth import WORKLOADS, make_catalogs
    wl = WORKLOADS["c1"]
    g, r = make_catalogs(wl, mock=0)
    cfg = E.Config(mesh=wl["mesh"], box=wl["box"], origin=wl["origin"], observer=wl["observer"],
                   assignment=wl["assignment"], interlacing=wl["interlacing"], lmax=4, n_kbins=wl["n_kbins"])
    cases = {"c1": (g, r, dict(mesh_n=wl["mesh"], box_size=wl["box"], box_origin=wl["origin"],
                               observer=wl["observer"], assignment=wl["assignment"], interlacing=wl["interlacing"],
                               lmax=4, n_kbins=wl["n_kbins"]), E.mesh64(g, r, cfg))}
    cases["wedge64"] = _footprint_case("wedge")
    table = {}
    for case, (gc, rc, kw, ref) in cases.items():
        for prec, tol in (("f64", 1e-9), ("f32", 1e-4)):
            got = lpp.Plan(precision=prec, **kw).estimate(gc, rc)
            errs = _series_errors(got, ref)
            own = _own_errors(got, ref)
            table[f"{case}_{prec}"] = errs
            table[f"{case}_{prec}_own"] = own
            for e in (errs, own):
                worst = max(e, key=e.get)
                assert e[worst] <= tol, (case, prec, worst, e[worst])
    cols = list(table)
    print("\n| series | " + " | ".join(cols) + " |")
    for name in table[cols[0]]:
        print(f"| {name} | " + " | ".join(f"{table[c][name]:.1e}" for c in cols) + " |")
    out = os.environ.get("LPP_ERROR_TABLE")
    if out:
        with open(out, "w") as f:
            json.dump(table, f, indent=1)


def test_device_catalogs_and_reuse(lpp):
    """Device-resident catalogs (torch tensors) give the same result as host ones, and a
    plan can be reused for catalogs of different sizes (workspace regrowth)."""
    import torch
    n, box, origin = 32, 120.0, (200.0, 100.0, 300.0)
    plan = lpp.Plan(n, box, origin, assignment=3, interlacing=1, precision="f32", lmax=4, n_kbins=8)
    for seed, (ng, nr) in enumerate([(500, 1500), (4000, 20000), (1000, 3000)]):
        g, r = _cats(200 + seed, ng, nr, origin, box)
        host = plan.estimate(g, r)
        to_dev = lambda c: Catalog(*[None if v is None else torch.tensor(v, dtype=torch.float32, device="cuda")
                                     for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])
        dev = plan.estimate(to_dev(g), to_dev(r))
        sc = _scales(host)
        sel = host["n_modes"] > 0
        # float32 columns vs float64 columns: positions rounded to float32 on the device side
        assert np.all(np.abs(dev["re"] - host["re"])[:, sel] <= 2e-4 * sc[:, sel])


def test_error_paths_leave_plan_usable(lpp):
    n, box, origin = 16, 50.0, (10.0, 10.0, 10.0)
    plan = lpp.Plan(n, box, origin, (0.0, 0.0, 0.0), assignment=2, interlacing=0, precision="f64", lmax=4, n_kbins=4)
    g, r = _cats(3, 300, 900, origin, box)

    def bad(mut, code, which="g"):
        gg, rr = _cats(3, 300, 900, origin, box)
        mut(gg if which == "g" else rr)
        with pytest.raises(lpp.LppError) as e:
            plan.estimate(gg, rr)
        assert e.value.status == code, (e.value, code)

    def nan(c):
        c.x[5] = np.nan

    def outside(c):
        c.y[7] = origin[1] + box + 1.0

    def zero_w(c):
        c.w[:] = 0.0

    def nan_shape(c):
        c.g2[3] = np.inf

    bad(nan, 2)
    bad(nan_shape, 2)
    bad(outside, 3)
    bad(outside, 3, which="r")
    bad(zero_w, 5, which="r")
    # an object at the observer (observer inside the box)
    plan2 = lpp.Plan(n, box, origin, (30.0, 30.0, 30.0), assignment=2, interlacing=0, precision="f64", lmax=4,
                     n_kbins=4)
    g2, r2 = _cats(4, 300, 900, origin, box)
    g2.x[0], g2.y[0], g2.z[0] = 30.0, 30.0, 30.0
    with pytest.raises(lpp.LppError) as e:
        plan2.estimate(g2, r2)
    assert e.value.status == 4
    # the plan still works
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=2, interlacing=0, lmax=4, n_kbins=4)
    ref = E.mesh64(g, r, cfg)
    _compare(plan.estimate(g, r), ref, 1e-9)


def test_batch_statuses(lpp):
    n, box, origin = 16, 70.0, (100.0, 100.0, 100.0)
    plan = lpp.Plan(n, box, origin, assignment=3, interlacing=1, precision="f64", lmax=4, n_kbins=5)
    cats = [_cats(30 + i, 200 + 150 * i, 700 + 300 * i, origin, box) for i in range(4)]
    cats[2][0].x[0] = np.nan
    outs = plan.estimate_batch([c[0] for c in cats], [c[1] for c in cats])
    assert isinstance(outs[2], lpp.LppError) and outs[2].status == 2
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=3, interlacing=1, lmax=4, n_kbins=5)
    for i in (0, 1, 3):
        _compare(outs[i], E.mesh64(cats[i][0], cats[i][1], cfg), 1e-9)


def _to_dev(c, dtype):
    import torch
    return Catalog(*[None if v is None else torch.tensor(v, dtype=dtype, device="cuda")
                     for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_graph_matches_oracle_and_replays(lpp, prec):
    """A batch of device-resident mocks of different sizes goes through one
    captured graph; every catalog matches the oracle; a second call on the
    same buffers replays the graph (no new capture), also after the buffers
    were refilled with other mocks of the same sizes, with eager estimates in
    between; an invalid catalog gets its own status and leaves the rest
    alone."""
    import torch
    n, box, origin = 32, 150.0, (300.0, 200.0, 250.0)
    tol = 1e-9 if prec == "f64" else 1e-4
    plan = lpp.Plan(n, box, origin, assignment=3, interlacing=1, precision=prec, lmax=4, n_kbins=10)
    cfg = E.Config(mesh=n, box=box, origin=origin, assignment=3, interlacing=1, lmax=4, n_kbins=10)
    sizes = [(700, 2500), (2000, 9000), (400, 5000)]
    cats = [_cats(500 + i, ng, nr, origin, box) for i, (ng, nr) in enumerate(sizes)]
    dev = [(_to_dev(g, torch.float64), _to_dev(r, torch.float64)) for g, r in cats]
    outs = plan.estimate_batch([d[0] for d in dev], [d[1] for d in dev])
    assert plan.batch_stats() == (1, 1)
    for (g, r), o in zip(cats, outs):
        _compare(o, E.mesh64(g, r, cfg), tol)
    # eager work in between, then the same buffers refilled with other mocks
    single = plan.estimate(*cats[1])
    _compare(single, E.mesh64(*cats[1], cfg), tol)
    cats2 = [_cats(900 + i, ng, nr, origin, box) for i, (ng, nr) in enumerate(sizes)]
    for (d_g, d_r), (g, r) in zip(dev, cats2):
        for dst, src in ((d_g, g), (d_r, r)):
            for name in ("x", "y", "z", "w", "nbar", "g1", "g2"):
                t = getattr(dst, name)
                if t is not None:
                    t.copy_(torch.tensor(getattr(src, name), dtype=torch.float64))
    for rep in range(2):
        outs2 = plan.estimate_batch([d[0] for d in dev], [d[1] for d in dev])
        assert plan.batch_stats() == (1, 2 + rep)
        for (g, r), o in zip(cats2, outs2):
            _compare(o, E.mesh64(g, r, cfg), tol)
    # an invalid catalog: its own status; the graph is captured again for the valid ones
    dev[1][0].x[5] = float("nan")
    outs3 = plan.estimate_batch([d[0] for d in dev], [d[1] for d in dev])
    assert isinstance(outs3[1], lpp.LppError) and outs3[1].status == 2
    for i in (0, 2):
        _compare(outs3[i], E.mesh64(*cats2[i], cfg), tol)
    assert plan.batch_stats()[0] == 2


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tuning_variants_match_oracle(lpp, prec):
    """Every launch shape gives the oracle's result: rows per x-pass workgroup,
    columns per strided workgroup, shell-sum workgroups and fields per deposit
    pass, on the compact wedge footprint (64^3)."""
    g, r, kw, ref = _footprint_case("wedge")
    plan = lpp.Plan(precision=prec, **kw)
    tol = 1e-9 if prec == "f64" else 1e-4
    variants = [dict(fft_rows_x=16), dict(fft_cols_y=8), dict(fft_cols_y=16), dict(fft_cols_z=8), dict(fft_cols_z=16),
                dict(bin_blocks=64), dict(bin_blocks=8192), dict(gather_density=1), dict(gather_density=3),
                dict(gather_shape=1), dict(gather_shape=2), dict(serial=1), dict(fft_streaming=8),
                dict(fft_streaming=13), dict(unfused=1), dict(unfused=1, gather_shape=3)]
    if prec == "f32":
        variants += [dict(gather_shape=3), dict(gather_density=4), dict(gather_density=6)]
    base = plan.tuning()
    for v in variants:
        plan.set_tuning(**{**base, **v})
        _compare(plan.estimate(g, r), ref, tol)


def test_overlapped_deposits_match_serial_order(lpp):
    """The default pipeline deposits the next gather pass on a second stream
    while the current pass is transformed (two work-mesh sets); the result is
    bitwise the serial pipeline's, for several estimates in a row on the same
    plan."""
    g, r, kw, ref = _footprint_case("wedge")
    plan = lpp.Plan(precision="f64", **kw)
    base = plan.tuning()
    plan.set_tuning(**{**base, "serial": 1})
    serial = plan.estimate(g, r)
    plan.set_tuning(**{**base, "serial": 0})
    for _ in range(3):
        over = plan.estimate(g, r)
        assert list(over["n_modes"]) == list(serial["n_modes"])
        for part in ("re", "im", "k_eff"):
            assert np.array_equal(np.asarray(over[part]), np.asarray(serial[part])), part
    _compare(over, ref, 1e-9)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_two_runs_are_bitwise_equal(lpp, prec):
    """Every step is reproducible bit for bit: the counting sort puts the
    objects of each cell in index order before the (atomic-free) gather, the
    shell sums go through one LDS row set per wavefront added in a fixed
    order, and every cross-block reduction has a fixed shape.  Two plans,
    same catalogs: identical estimates and window multipoles."""
    g, r, kw, _ = _footprint_case("wedge")
    a = lpp.Plan(precision=prec, **kw).estimate(g, r)
    b = lpp.Plan(precision=prec, **kw).estimate(g, r)
    for part in ("re", "im", "k_eff"):
        assert np.array_equal(np.asarray(a[part]), np.asarray(b[part])), part
    wa = lpp.Plan(precision=prec, **kw).window_multipoles(r, 0.25, lmax=4, n_rbins=12, rmax=40.0)
    wb = lpp.Plan(precision=prec, **kw).window_multipoles(r, 0.25, lmax=4, n_rbins=12, rmax=40.0)
    assert np.array_equal(wa["Q"], wb["Q"])


def test_autotune_writes_cache_and_keeps_parity(lpp, tmp_path):
    g, r, kw, ref = _footprint_case("wedge")
    plan = lpp.Plan(precision="f32", **kw)
    path = tmp_path / "tune.jsonl"
    chosen = plan.autotune(g, r, cache_path=str(path))
    line = path.read_text().strip().splitlines()
    assert len(line) == 1 and '"key": "N64_f32_p3_il1"' in line[0]
    for k, v in chosen.items():
        assert f'"{k}": {v}' in line[0]
    _compare(plan.estimate(g, r), ref, 1e-4)


_WINDOW_REF = {}


def _window_case(name):
    """Randoms of a survey wedge seen from a near observer (wide angles) in a
    box twice the wedge's extent; the oracle's Q_l at l <= lmax."""
    from oracle import window as OW
    from synth import wedge_uniform
    if name not in _WINDOW_REF:
        if name == "wedge_l8":
            n, box, origin, p, il, lmax, nb, rmax, nr = 32, 600.0, (-80.0, -80.0, -80.0), 3, 1, 8, 12, 240.0, 40000
            pts = lambda k, rng: wedge_uniform(k, rng, (5.0, 80.0), (5.0, 60.0), (60.0, 200.0))
        else:
            n, box, origin, p, il, lmax, nb, rmax, nr = 32, 500.0, (100.0, -50.0, 20.0), 2, 0, 4, 10, 200.0, 30000
            pts = lambda k, rng: box_uniform(k, rng, (180.0, 40.0, 90.0), 160.0)
        rng = np.random.default_rng(77)
        rp = pts(nr, rng)
        ran = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), rng.random(nr) + 0.5, np.full(nr, 3e-4))
        alpha = 0.05
        ref = OW.window_multipoles(ran, alpha, n, box, origin, (0.0, 0.0, 0.0), p, il, 1, lmax, nb, rmax)
        _WINDOW_REF[name] = (ran, alpha, dict(mesh_n=n, box_size=box, box_origin=origin, assignment=p,
                                              interlacing=il, lmax=4, n_kbins=8), (lmax, nb, rmax), ref)
    return _WINDOW_REF[name]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["wedge_l8", "box_l4"])
def test_window_multipoles_match_oracle(lpp, name, prec):
    ran, alpha, kw, (lmax, nb, rmax), ref = _window_case(name)
    plan = lpp.Plan(precision=prec, **kw)
    got = plan.window_multipoles(ran, alpha, lmax=lmax, n_rbins=nb, rmax=rmax)
    assert list(got["counts"]) == list(ref["counts"])
    assert abs(got["norm_I"] - ref["norm_I"]) <= 1e-12 * ref["norm_I"]
    sel = ref["counts"] > 0
    np.testing.assert_allclose(got["r_eff"][sel], ref["r_eff"][sel], rtol=1e-12)
    scale = np.max(np.abs(ref["Q"][0][sel]))
    tol = 1e-9 if prec == "f64" else 1e-4
    err = np.max(np.abs(got["Q"][:, sel] - ref["Q"][:, sel])) / scale
    assert err <= tol, (name, prec, err)


@pytest.mark.parametrize("cols", ["host_f64", "dev_f64", "dev_f32"])
def test_window_pairs_match_oracle(lpp, cols):
    """Pair-counted window multipoles (midpoint and end-point lines of sight)
    of a near-observer wedge (3,000 randoms, unequal weights, l <= 8, 12
    shells) against the oracle's direct FP64 sum over the same pairs: ordered
    pair counts exact, Q_l and the mean separations at 1e-11 (FP64 with a
    different summation order); FP32 device columns are compared with the
    oracle on the same FP32-rounded values."""
    import torch
    from oracle import window as OW
    from synth import wedge_uniform
    rng = np.random.default_rng(41)
    n = 3000
    rp = wedge_uniform(n, rng, (5.0, 80.0), (5.0, 60.0), (60.0, 200.0))
    ran = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), 0.5 + rng.random(n), np.full(n, 1e-3))
    if cols == "dev_f32":
        ran = _rounded_f32(ran)
    alpha, norm_I, lmax, nb, rmax = 0.07, 3.5e-4, 8, 12, 240.0
    if cols == "host_f64":
        arg = ran
    else:
        dt = torch.float32 if cols == "dev_f32" else torch.float64
        arg = Catalog(*[None if v is None else torch.tensor(v, dtype=dt, device="cuda")
                        for v in (ran.x, ran.y, ran.z, ran.w, ran.nbar, ran.g1, ran.g2)])
    for los in ("midpoint", "endpoint"):
        ref = OW.window_pairs(ran, alpha, norm_I, (0.0, 0.0, 0.0), los, lmax, nb, rmax)
        got = lpp.window_pairs(arg, alpha, norm_I, (0.0, 0.0, 0.0), los, lmax, nb, rmax)
        assert list(got["counts"]) == list(ref["counts"]), los
        scale = np.max(np.abs(ref["Q"][0]))
        assert np.max(np.abs(got["Q"] - ref["Q"])) <= 1e-11 * scale, (los, np.max(np.abs(got["Q"] - ref["Q"])) / scale)
        sel = ref["counts"] > 0
        np.testing.assert_allclose(got["r_eff"][sel], ref["r_eff"][sel], rtol=1e-12)


def test_template_plain_matches_oracle(lpp):
    """The plain template path (FFTLog on the GPU, FP64) against the oracle's
    numpy FFTLog, for a smooth window table and a few parameter points, host
    and device I/O."""
    import torch
    from oracle import window as OW
    k = OW.log_grid(1e-5, 1e3, 4096)
    pfid = 2e4 * (k / 0.02) / (1 + (k / 0.02) ** 2) ** 1.4
    r_q = np.linspace(5.0, 3000.0, 300)
    Q = np.vstack([np.exp(-r_q / 900.0) * (1.0 if i == 0 else 0.3 * (-1) ** i / (i + 1)) *
                   (1 + 0.2 * np.sin(r_q / 300.0 + i)) for i in range(5)])
    kout = np.arange(1, 31) * 0.01
    pars = np.array([[0.03, 2.0, 0.7, 0.8, 1.0], [0.01, 1.2, 0.9, 0.65, 0.5], [0.045, 2.8, 0.55, 0.95, 1.8]])
    ref = OW.template_plain(k, pfid, r_q, Q, pars, kout, nbar=1.4e-3, sigma_gamma=0.2)
    got = lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, pars, kout, 1.4e-3, 0.2)
    for o in range(5):
        scale = np.max(np.abs(ref[:, o]))
        assert np.max(np.abs(got[:, o] - ref[:, o])) <= 1e-9 * scale, (o, np.max(np.abs(got[:, o] - ref[:, o])) / scale)
    dp = torch.tensor(pars, device="cuda")
    do = torch.zeros((3, 5, 30), dtype=torch.float64, device="cuda")
    lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, dp, kout, 1.4e-3, 0.2, out=do)
    assert np.array_equal(do.cpu().numpy(), got)


def test_template_multipoles_matches_oracle(lpp):
    """All four template families (density auto with its leakage quadrupole,
    shape-density cross, plus, minus) on the GPU against the oracle's FFTLog
    path, host I/O, and the plus and cross rows against lpp_template_plain
    (same kernels per point)."""
    from oracle import window as OW
    k = OW.log_grid(1e-5, 1e3, 4096)
    pfid = 2e4 * (k / 0.02) / (1 + (k / 0.02) ** 2) ** 1.4
    r_q = np.linspace(5.0, 3000.0, 300)
    Q = np.vstack([np.exp(-r_q / 900.0) * (1.0 if i == 0 else 0.3 * (-1) ** i / (i + 1)) *
                   (1 + 0.2 * np.sin(r_q / 300.0 + i)) for i in range(5)])
    kout = np.arange(1, 31) * 0.01
    pars = np.array([[0.03, 2.0, 0.7, 0.8, 1.0], [-1.0, 1.0, 0.0, 0.9, 0.0], [0.045, 2.8, 0.55, 0.95, 1.8]])
    ref = OW.template_multipoles(k, pfid, r_q, Q, pars, kout, nbar=1.4e-3, sigma_gamma=0.2)
    got = lpp.template_multipoles(pfid, 1e-5, 1e3, r_q, Q, pars, kout, 1.4e-3, 0.2)
    assert got.shape == (3, 9, 30)
    for o in range(9):
        scale = np.max(np.abs(ref[:, o]))
        assert np.max(np.abs(got[:, o] - ref[:, o])) <= 1e-9 * scale, (lpp.TEMPLATE_SERIES[o],
                                                                       np.max(np.abs(got[:, o] - ref[:, o])) / scale)
    plain = lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, pars, kout, 1.4e-3, 0.2)
    for o5, o9 in ((0, 5), (1, 6), (2, 7), (3, 3), (4, 4)):
        scale = np.max(np.abs(plain[:, o5]))
        assert np.max(np.abs(got[:, o9] - plain[:, o5])) <= 1e-13 * scale


# ---------------------------------------------------------------------------
# the emulator network

EMU_WIDTHS = [5, 256, 256, 256, 150]


def _emu_setup(seed=5, B=300):
    import torch
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (B, 5))
    T = np.sin(X @ rng.standard_normal((5, 150))) + 0.1 * rng.standard_normal((B, 150))
    return (X, T, torch.tensor(X, dtype=torch.float32, device="cuda"),
            torch.tensor(T, dtype=torch.float32, device="cuda"))


def test_mlp_forward_matches_oracle(lpp):
    """Forward pass (BF16 MFMA, FP32 accumulation) of the 5-256-256-256-150
    network against the FP64 oracle with the same BF16 operand rounding, on
    300 rows (partial 32-row tiles).  Tolerance 3e-3 of the output scale: a
    BF16 rounding decision taken on an FP32 vs an FP64 sum can differ by one
    BF16 unit (2^-8 relative) on a few activations."""
    import torch
    from oracle import mlp as OM
    net = lpp.Mlp(EMU_WIDTHS, max_batch=512, seed=11)
    p = net.params()
    X, T, Xd, Td = _emu_setup()
    Y = torch.zeros((X.shape[0], 150), dtype=torch.float32, device="cuda")
    net.forward(Xd, Y)
    ref = OM.forward(p.astype(np.float64), EMU_WIDTHS, X.astype(np.float32).astype(np.float64), bf16=True)
    err = np.max(np.abs(Y.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 3e-3, err


def _bf16_forward_bound(params, widths, X):
    """Exact FP64 forward of the network and two a-priori figures for how far
    a forward pass with BF16 weights, BF16 hi + lo layer inputs and FP32
    accumulation can lie from it, per output:

    * a worst-case bound, carried layer by layer with absolute values:
      BF16 weights (round to nearest even: relative error at most u = 2^-8),
      inputs split as hi + lo = bf16(a) + bf16(a - hi) (error at most
      2^-16 |a|), FP32 accumulation of the 2K products and the bias (at most
      (2K + 1) 2^-24 of the sum of their magnitudes), SiLU in FP32
      (Lipschitz constant 1.1, 2^-20 relative evaluation error).  It holds
      for any parameters but is loose by the growth of |W| sums;
    * the standard deviation of the same error under the usual model of
      rounding errors as independent, zero-mean and uniformly distributed
      (variance at most (u |W|)^2 / 3 per weight, and likewise for the input
      split), propagated to first order through the layers with the exact
      SiLU derivative."""
    from oracle import mlp as OM
    layers = OM.unpack(np.asarray(params, dtype=np.float64), widths)
    a = np.asarray(X, dtype=np.float64)
    e = np.zeros_like(a)
    v = np.zeros_like(a)
    u8, u16, u24 = 2.0 ** -8, 2.0 ** -16, 2.0 ** -24
    for l, (Wm, b) in enumerate(layers):
        K = Wm.shape[1]
        aW = np.abs(Wm).T
        z = a @ Wm.T + b
        a_in = u16 * (np.abs(a) + e) + e               # |split(a_dev) - a|
        mag = (np.abs(a) + a_in) @ ((1 + u8) * aW) + np.abs(b)
        ez = a_in @ ((1 + u8) * aW) + u8 * (np.abs(a) @ aW) + (2 * K + 1) * u24 * mag
        vz = (a * a) @ (Wm.T ** 2) * (u8 * u8 / 3.0 + u16 * u16 / 3.0) + v @ (Wm.T ** 2)
        if l + 1 < len(layers):
            sg = 1.0 / (1.0 + np.exp(-z))
            a = z * sg
            e = 1.1 * ez + 2.0 ** -20 * (np.abs(a) + 1.1 * ez)
            v = vz * (sg * (1.0 + z * (1.0 - sg))) ** 2
        else:
            return z, ez, np.sqrt(vz)


def test_mlp_forward_within_bf16_bound_of_fp64(lpp):
    """The device's forward pass (BF16 MFMA, FP32 accumulation) against the
    plain FP64 network (no BF16 rounding anywhere): every output lies within
    the worst-case bound of _bf16_forward_bound, within 6 standard deviations
    of its rounding-error model, and the errors' rms over all outputs is
    0.3-2 standard deviations (the model neither misses a systematic error
    nor is vacuous)."""
    import torch
    net = lpp.Mlp(EMU_WIDTHS, max_batch=512, seed=11)
    p = net.params().astype(np.float64)
    X, T, Xd, Td = _emu_setup(8)
    Y = torch.zeros((X.shape[0], 150), dtype=torch.float32, device="cuda")
    net.forward(Xd, Y)
    ref, bound, sd = _bf16_forward_bound(p, EMU_WIDTHS, X.astype(np.float32).astype(np.float64))
    got = Y.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    z = err / sd
    assert z.max() < 6.0, z.max()
    rms = float(np.sqrt(np.mean(z * z)))
    assert 0.3 < rms < 2.0, rms
    print(f"\nBF16 forward vs FP64: max err {err.max():.2e} (output scale {np.max(np.abs(ref)):.2e}), "
          f"max err/sd {z.max():.2f}, rms err/sd {rms:.2f}, max err/worst-case bound {np.max(err / bound):.1e}")


def test_mlp_gradients_and_adam_match_oracle(lpp):
    """One training step: the loss and the gradients (BF16 backward products)
    against the oracle's chain rule with the same roundings, then Adam's
    update against the oracle's Adam applied to the device's own gradients."""
    from oracle import mlp as OM
    net = lpp.Mlp(EMU_WIDTHS, max_batch=512, seed=12)
    p0 = net.params().astype(np.float64)
    X, T, Xd, Td = _emu_setup(6)
    Xf = X.astype(np.float32).astype(np.float64)
    Tf = T.astype(np.float32).astype(np.float64)
    loss = net.train_step(Xd, Td, lr=1e-3)
    p1, g = net.params(grads=True)
    ref_loss, ref_g = OM.loss_and_grads(p0, EMU_WIDTHS, Xf, Tf, bf16=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    off = 0
    for l in range(4):
        n_w = EMU_WIDTHS[l] * EMU_WIDTHS[l + 1]
        for seg in (slice(off, off + n_w), slice(off + n_w, off + n_w + EMU_WIDTHS[l + 1])):
            scale = np.max(np.abs(ref_g[seg]))
            assert np.max(np.abs(g[seg] - ref_g[seg])) <= 2e-2 * scale, (l, seg)
        off += n_w + EMU_WIDTHS[l + 1]
    want, _, _ = OM.adam_step(p0, g.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    assert np.max(np.abs(p1 - want)) <= 1e-6


def test_mlp_fit_learns_and_is_deterministic(lpp):
    """Graph-replayed training lowers the loss of a smooth map (plus noise of
    variance 0.01) by over 85% in 30 epochs, and two fits from the same seeds
    end with identical parameters."""
    import torch
    X, T, Xd, Td = _emu_setup(7, B=2048)
    losses, params = [], []
    for _ in range(2):
        net = lpp.Mlp(EMU_WIDTHS, max_batch=2048, seed=3)
        Y = torch.zeros((2048, 150), dtype=torch.float32, device="cuda")
        net.forward(Xd, Y)
        before = float(torch.mean((Y - Td) ** 2))
        net.fit(Xd, Td, batch=256, epochs=30, lr0=2e-3, lr1=1e-5, seed=9)
        net.forward(Xd, Y)
        losses.append((before, float(torch.mean((Y - Td) ** 2))))
        params.append(net.params())
    assert losses[0][1] < 0.15 * losses[0][0], losses
    assert np.array_equal(params[0], params[1])


def test_emulator_round_trip_on_template_design(lpp):
    """The emulator's encoding and decoding around the network: trained for a
    few hundred epochs on 3,000 plain-path templates of a smooth window, its
    held-out predictions stay within 2 % of the plain path (the 1 % bar is
    measured on the full 20,000-point design by bench.py), and it evaluates
    them faster than the plain path does (bench.py times both at 2,000
    points; here at least 3x at 300, where launch latency weighs most)."""
    import torch
    from paper_2202_11839_amd.emulator import Emulator, accuracy
    from synth import EMU_RANGES, latin_hypercube, power_spectrum
    k = np.exp(np.linspace(np.log(1e-5), np.log(1e3), 4096))
    r_q = np.linspace(5.0, 2000.0, 200)
    Q = np.vstack([np.exp(-r_q / 700.0) * (1.0 if i == 0 else 0.2 / (i + 1)) for i in range(5)])
    pts = latin_hypercube(3300, EMU_RANGES, seed=4)
    P = torch.tensor(pts, dtype=torch.float64, device="cuda")
    Y = torch.zeros((3300, 5, 30), dtype=torch.float64, device="cuda")
    lpp.template_plain(power_spectrum(k), 1e-5, 1e3, r_q, Q, P, np.arange(1, 31) * 0.01, 1.4e-3, 0.2, out=Y)
    emu = Emulator(EMU_RANGES, n_k=30, max_batch=512, seed=1)
    emu.fit(P[:3000], Y[:3000], 1.4e-3, 0.2, epochs=200, batch=128, lr0=2e-3, lr1=1e-5, seed=3)
    E = torch.zeros((300, 5, 30), dtype=torch.float64, device="cuda")
    emu.predict(P[3000:], E)
    rel, _ = accuracy(E.cpu().numpy(), Y[3000:].cpu().numpy())
    assert np.all(np.isfinite(rel)) and rel.max() < 0.02, rel.max(axis=0)
    # what the network gains: the same 300 points through the plain path
    # (FFTLog per point) and through the network, best of five, same GPU
    import time

    def best(f):
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return min(ts)
    Yp = torch.zeros((300, 5, 30), dtype=torch.float64, device="cuda")
    t_plain = best(lambda: lpp.template_plain(power_spectrum(k), 1e-5, 1e3, r_q, Q, P[3000:], np.arange(1, 31) * 0.01,
                                              1.4e-3, 0.2, out=Yp))
    t_emu = best(lambda: emu.predict(P[3000:], E))
    assert t_emu * 3 < t_plain, (t_emu, t_plain)


def test_full_size_512_workload_sampled_outputs(lpp):
    """The 512^3 workload (1.5M galaxies + 15M randoms, TSC + interlacing,
    50 shells) in bench.py's launch configuration (device-resident catalogs,
    FP32): mode counts bit-exact and the scalars at 1e-10 against the oracle,
    and the two monopoles the oracle computes at full size in FP64 (DD_l0 and
    PLUS_l0: one deposit and one numpy FFT per grid) at the FP32 tolerance."""
    import torch
    from oracle import mesh as OM
    from synth import WORKLOADS, make_catalogs
    wl = WORKLOADS["c2"]
    gal, ran = make_catalogs(wl, mock=0)
    dev = lambda c: Catalog(*[None if v is None else torch.tensor(v, device="cuda")
                              for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision="f32", lmax=4, n_kbins=wl["n_kbins"])
    got = plan.estimate(dev(gal), dev(ran))
    cfg = E.Config(mesh=wl["mesh"], box=wl["box"], origin=wl["origin"], observer=wl["observer"],
                   assignment=wl["assignment"], interlacing=wl["interlacing"], lmax=4, n_kbins=wl["n_kbins"])
    sc = E.scalars(gal, ran)
    for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran"):
        assert abs(got[k] - sc[k]) <= 1e-10 * abs(sc[k]), k
    num, den = cfg.bin_width()
    counts = OM.mode_counts(cfg.mesh, cfg.n_kbins, num, den)
    assert list(got["n_modes"]) == list(counts)
    bidx = OM.bin_index(cfg.mesh, cfg.n_kbins, num, den)
    comp = OM.compensation(cfg.mesh, cfg.assignment)
    phase = OM.interlace_phase(cfg.mesh)
    safe = np.where(counts > 0, counts, 1)
    allpos = np.concatenate([gal.pos(), ran.pos()])
    Fd = E._transform(cfg, allpos, np.concatenate([gal.w, -sc["alpha"] * ran.w]), comp, phase)
    dd0 = E._bin_sums(cfg, bidx, Fd * np.conj(Fd)).real / (sc["norm_I"] * safe) - sc["shot_dd"]
    del Fd
    Fg = E._transform(cfg, gal.pos(), gal.w * (gal.g1 + 1j * gal.g2), comp, phase)
    pp0 = E._bin_sums(cfg, bidx, Fg * np.conj(Fg)).real / (sc["norm_I"] * safe) - sc["shot_plus"]
    del Fg
    s = got["series"]
    for name, ref, shot in (("DD_l0", dd0, sc["shot_dd"]), ("PLUS_l0", pp0, sc["shot_plus"])):
        g = got["re"][s.index(name)]
        scale = np.abs(ref) + shot  # the auto power before shot-noise subtraction
        assert np.max(np.abs(g - ref) / scale) <= 1e-4, name


def test_full_size_512_all_series_against_stored_oracle(lpp):
    """Every series of the 512^3 wedge workload's estimator settings (TSC +
    interlacing, compensation, l <= 4, 50 shells), FP32, device-resident
    catalogs as bench.py times it, against the FP64 oracle (mesh64, the
    paper's Cartesian-tensor FFT route) on a 60,000 + 600,000 subsample of the
    workload, stored in tests/golden/c2_subsample_512.json by
    tests/golden/make_c2_subsample.py (which calls only oracle/ and synth/):
    all 15 series per shell at 1e-4 (of the scale and of the series' own
    value), mode counts bit-exact, scalars at 1e-10."""
    import json
    import os
    import sys
    import torch
    gold_path = os.path.join(os.path.dirname(__file__), "golden", "c2_subsample_512.json")
    gold = json.load(open(gold_path))
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_c2_subsample as MK
    g, r = MK.catalogs()
    cs = MK.checksums(g, r)
    for k, v in gold["checksums"].items():
        assert abs(cs[k] - v) <= 1e-12 * max(1.0, abs(v)), ("the catalog generator changed", k, cs[k], v)
    ref = dict(gold)
    for k in ("n_modes", "k_eff", "k_lo", "re", "im"):
        ref[k] = np.asarray(gold[k])
    wl = MK.WORKLOADS["c2"]
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision="f32", lmax=4, n_kbins=wl["n_kbins"])
    got = plan.estimate(_device_catalog(g, torch), _device_catalog(r, torch))
    worst = _compare(got, ref, 1e-4)
    own = _own_errors(got, ref)
    print(f"\n512^3 subsample, FP32 vs FP64 oracle: worst {worst:.2e} of the scale; own-value "
          + ", ".join(f"{k} {v:.1e}" for k, v in own.items()))


def test_batch_256_mock_against_stored_oracle(lpp):
    """One mock of the 256^3 batch workload's settings (TSC + interlacing,
    l <= 4, 50 shells), a 30,000 + 300,000 subsample, through the batch path
    (lpp_estimate_batch: one captured graph, then a replay) next to two other
    mocks, against the FP64 oracle stored in tests/golden/c3_subsample_256.json
    by tests/golden/make_c3_subsample.py: every series at 1e-4 (scale and own
    value), counts bit-exact, on the capture and on the replay."""
    import json
    import os
    import sys
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_subsample_256.json")))
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_c3_subsample as MK
    g, r = MK.catalogs()
    cs = MK.checksums(g, r)
    for k, v in gold["checksums"].items():
        assert abs(cs[k] - v) <= 1e-12 * max(1.0, abs(v)), ("the catalog generator changed", k, cs[k], v)
    ref = dict(gold)
    for k in ("n_modes", "k_eff", "k_lo", "re", "im"):
        ref[k] = np.asarray(gold[k])
    wl = MK.WORKLOADS["c3"]
    others = [MK.make_catalogs(wl, mock=m, n_gal=20000 + 5000 * m, n_ran=200000) for m in (6, 7)]
    gals = [_device_catalog(g, torch)] + [_device_catalog(o[0], torch) for o in others]
    rans = [_device_catalog(r, torch)] + [_device_catalog(o[1], torch) for o in others]
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision="f32", lmax=4, n_kbins=wl["n_kbins"])
    for _ in range(2):
        outs = plan.estimate_batch(gals, rans)
        assert all(not isinstance(o, Exception) for o in outs), outs
        _compare(outs[0], ref, 1e-4)
    assert plan.batch_stats() == (1, 2)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_shell_sums_match_the_unfused_path(lpp, prec):
    """The shape fields' z pass fused with their shell sums against the same
    z pass as launches of its own followed by the shell-sum kernel (tuning
    field unfused = 1), on the 256^3 batch workload's settings (a 30,000 +
    300,000 subsample, TSC + interlacing, l <= 4, 50 shells): both transform,
    combine and weigh every mode with the same operations, so the series may
    differ only by the order of the FP64 shell sums (1e-10 of each series'
    scale); counts bit-exact."""
    import os
    import sys
    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_c3_subsample as MK
    g, r = MK.catalogs()
    wl = MK.WORKLOADS["c3"]
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision=prec, lmax=4, n_kbins=wl["n_kbins"])
    dt = torch.float32 if prec == "f32" else torch.float64
    gd, rd = _device_catalog(g, torch, dt), _device_catalog(r, torch, dt)
    fused = plan.estimate(gd, rd)
    plan.set_tuning(unfused=1)
    assert plan.tuning()["unfused"] == 1
    sep = plan.estimate(gd, rd)
    assert list(fused["n_modes"]) == list(sep["n_modes"])
    scales = _series_scale(sep)
    for i, name in enumerate(sep["series"]):
        for part in ("re", "im"):
            d = np.abs(np.asarray(fused[part][i]) - np.asarray(sep[part][i]))
            assert np.all(d <= 1e-10 * scales[i] + 1e-300), (name, part, float((d / scales[i]).max()))


def _device_catalog(c, torch, dtype=None):
    return Catalog(*[None if v is None else torch.tensor(v, device="cuda", dtype=dtype)
                     for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])


def _rounded_f32(c):
    """The catalog as the device sees FP32 columns (each value rounded to FP32)."""
    return Catalog(*[None if v is None else np.asarray(v, dtype=np.float32).astype(np.float64)
                     for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])


def _series_scale(r):
    """Each series' scale (the auto power of its fields before shot-noise
    subtraction) from a result of the library."""
    s = r["series"]
    dd = np.abs(np.asarray(r["re"][s.index("DD_l0")]) + r["shot_dd"])
    pp = np.abs(np.asarray(r["re"][s.index("PLUS_l0")]) + r["shot_plus"])
    return [dd if n.startswith("DD") else (np.sqrt(dd * pp) if n.startswith("GD") else pp) for n in s]


def test_full_size_1024_workload_counts_scalars_and_precisions(lpp):
    """The 1024^3 workload (10M galaxies + 50M randoms, TSC + interlacing, 80
    shells) in the launch configuration bench.py times for it (device-resident
    FP32 catalogs): mode counts bit-exact and the scalars at 1e-10 against the
    oracle (on the same FP32 columns), and every multipole of the FP32 path within 1e-4 of its scale of
    the FP64 path on the same catalogs (the oracle's own FP64 transforms at
    this size are beyond a test's time)."""
    import gc
    import torch
    from oracle import mesh as OM
    from synth import WORKLOADS, make_catalogs
    wl = WORKLOADS["c4"]
    print(f"[1024^3] generating catalogs", flush=True)
    gal, ran = make_catalogs(wl, mock=0, grf_mesh=512)
    dg, dr = _device_catalog(gal, torch, torch.float32), _device_catalog(ran, torch, torch.float32)
    mk = lambda prec: lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                               interlacing=wl["interlacing"], precision=prec, lmax=4, n_kbins=wl["n_kbins"])
    res = {}
    for prec in ("f32", "f64"):
        print(f"[1024^3] estimate {prec}", flush=True)
        plan = mk(prec)
        res[prec] = plan.estimate(dg, dr)
        del plan
        gc.collect()
        torch.cuda.empty_cache()
    sc = E.scalars(_rounded_f32(gal), _rounded_f32(ran))  # the columns the device read
    for prec in ("f32", "f64"):
        for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran"):
            assert abs(res[prec][k] - sc[k]) <= 1e-10 * abs(sc[k]), (prec, k)
    print(f"[1024^3] oracle mode counts", flush=True)
    num, den = OM.default_dn(wl["mesh"], wl["n_kbins"])
    counts = OM.mode_counts(wl["mesh"], wl["n_kbins"], num, den)
    for prec in ("f32", "f64"):
        assert list(res[prec]["n_modes"]) == list(counts), prec
    r32, r64 = res["f32"], res["f64"]
    assert r32["series"] == r64["series"]
    sel = counts > 0
    for i, (name, sc_i) in enumerate(zip(r64["series"], _series_scale(r64))):
        for part in ("re", "im"):
            err = np.abs(np.asarray(r32[part][i]) - np.asarray(r64[part][i]))[sel] / sc_i[sel]
            assert err.max() <= 1e-4, (name, part, err.max())


def test_full_size_256_batch_matches_single_estimates(lpp):
    """bench.py's batch at 256^3 (8 of the 64 mocks over the 0.2M-2M galaxy
    ladder, 10x randoms, device-resident FP32) through one captured graph:
    each mock's scalars at 1e-10 and mode counts bit-exactly against the
    oracle, and every multipole equal to the same mock's single estimate
    within 1e-6 of its scale (the two differ only in where the randoms'
    weight scale is read)."""
    import torch
    from oracle import mesh as OM
    from synth import WORKLOADS, c3_sizes, make_catalogs
    wl = WORKLOADS["c3"]
    ladder = c3_sizes(64)
    pick = sorted(set(int(round(x)) for x in np.linspace(0, 63, 8)))
    cats = [make_catalogs(wl, mock=i, n_gal=ladder[i], n_ran=10 * ladder[i]) for i in pick]
    dev = [(_device_catalog(g, torch, torch.float32), _device_catalog(r, torch, torch.float32)) for g, r in cats]
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision="f32", lmax=4, n_kbins=wl["n_kbins"])
    outs = plan.estimate_batch([d[0] for d in dev], [d[1] for d in dev])
    num, den = OM.default_dn(wl["mesh"], wl["n_kbins"])
    counts = OM.mode_counts(wl["mesh"], wl["n_kbins"], num, den)
    sel = counts > 0
    for (g, r), (dg, dr), o in zip(cats, dev, outs):
        assert not isinstance(o, Exception), o
        sc = E.scalars(_rounded_f32(g), _rounded_f32(r))  # the columns the device read
        for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran"):
            assert abs(o[k] - sc[k]) <= 1e-10 * abs(sc[k]), k
        assert list(o["n_modes"]) == list(counts)
        single = plan.estimate(dg, dr)
        for i, (name, sc_i) in enumerate(zip(single["series"], _series_scale(single))):
            for part in ("re", "im"):
                err = np.abs(np.asarray(o[part][i]) - np.asarray(single[part][i]))[sel] / sc_i[sel]
                assert err.max() <= 1e-6, (name, part, err.max())


def test_known_spectrum_recovery_on_the_gpu(lpp):
    """The GPU estimator against the paper's closed forms rather than the
    oracle: lattice catalogs of a Gaussian field with tidal shapes
    gamma = -(A/2)(1 - mu^2) delta (Sec. IV.A eq. power_for_validation) at a
    distant observer; the mean over 32 realisations of every multipole
    matches the exact discrete-shell expectation within 4 sigma of the
    realisation scatter (plus 1e-3 of the scale).  On shells with many modes
    that expectation tends to the amplitudes -1/6 (GD L=2), 2/15, -4/21, 2/35
    (PLUS l=0,2,4) and 1/420 (MINUS L=4) times P (checked on the CPU)."""
    from physics_expect import _expected_lattice
    from synth import lattice_catalogs
    n, box = 16, 800.0
    nhat = np.array([0.6, 0.48, 0.64])
    origin = tuple(1.0e7 * nhat - box / 2)
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=(0.0, 0.0, 0.0), assignment=1, interlacing=0,
                   compensate=0, n_kbins=8, lmax=4)
    plan = lpp.Plan(n, box, origin, (0.0, 0.0, 0.0), assignment=1, interlacing=0, compensate=0, precision="f32",
                    lmax=4, n_kbins=8)
    amp = 0.5
    runs = []
    for seed in range(32):
        g, r, s = lattice_catalogs(n, box, origin, (0.0, 0.0, 0.0), 1000 + seed, delta_rms=0.1, amp=amp)
        res = plan.estimate(g, r)
        v = dict(zip(res["series"], np.asarray(res["re"])))
        v["DD_l0"] = v["DD_l0"] + res["shot_dd"]      # the lattice has no Poisson noise
        v["PLUS_l0"] = v["PLUS_l0"] + res["shot_plus"]
        runs.append((v, s, res["alpha"]))
    s2 = np.mean([x[1] ** 2 / x[2] for x in runs])
    exp = _expected_lattice(cfg, s2, amp, nhat)
    ok = np.asarray(res["n_modes"]) >= 20
    for key in ("DD_l0", "DD_l2", "DD_l4", "GD_L2", "GD_L4", "PLUS_l0", "PLUS_l2", "PLUS_l4", "MINUS_L4"):
        arr = np.array([x[0][key] * (s2 / (x[1] ** 2 / x[2])) for x in runs])
        mean = arr.mean(axis=0)
        err = arr.std(axis=0, ddof=1) / np.sqrt(len(runs))
        scale = np.abs(exp["DD_l0"]) * (amp if key.startswith("GD") else (amp ** 2 if key[0] in "PM" else 1))
        dev = np.abs(mean - exp[key])
        assert np.all(dev[ok] <= 4.0 * err[ok] + 1e-3 * scale[ok]), (key, dev[ok], err[ok])


def test_shot_noise_closed_form_on_the_gpu(lpp):
    """Uniform positions with pure shape noise (Sec. V): N_+ equals
    2 sigma^2 sum w^2 / I, and after its subtraction the P_+ monopole and
    every other shape moment average to zero over 16 realisations."""
    from synth import pure_noise_catalogs
    n, box, sigma = 16, 200.0, 0.3
    origin = (500.0, 300.0, 200.0)
    plan = lpp.Plan(n, box, origin, (0.0, 0.0, 0.0), assignment=2, interlacing=1, precision="f32", lmax=4,
                    n_kbins=6)
    vals = {k: [] for k in ("PLUS_l0", "PLUS_l2", "MINUS_L4", "GD_L2")}
    for seed in range(16):
        g, r = pure_noise_catalogs(3000, 6000, origin, box, sigma, 500 + seed)
        res = plan.estimate(g, r)
        d = dict(zip(res["series"], np.asarray(res["re"])))
        for k in vals:
            vals[k].append(d[k])
        npl = res["shot_plus"]
        assert abs(npl - 2 * sigma ** 2 * np.sum(g.w ** 2) / res["norm_I"]) < 0.1 * npl
    for k, v in vals.items():
        v = np.array(v)[:, 1:]      # bin 0 holds only the DC mode
        m = v.mean()
        err = v.std(ddof=1) / np.sqrt(v.size)
        assert abs(m) < 4 * err + 1e-3 * npl, (k, m, err)


def test_emulator_predict_fused_network_matches_layered_forward(lpp):
    """lpp_emulator_predict runs the network as one fused launch per batch;
    its outputs equal the layer-by-layer lpp_mlp_forward's (same bits) after
    the same decoding, here on 700 points (ragged 16-row blocks, two batches
    of at most 512) of an untrained network."""
    import torch
    from paper_2202_11839_amd.emulator import Emulator
    from synth import EMU_RANGES, latin_hypercube
    n, n_k = 700, 30
    pts = latin_hypercube(n, EMU_RANGES, seed=11)
    emu = Emulator(EMU_RANGES, n_k=n_k, max_batch=512, seed=5)
    emu.nbar, emu.sigma_gamma = 1.4e-3, 0.2
    rng = np.random.default_rng(3)
    mean_h, sd_h = rng.normal(size=5 * n_k), 0.5 + rng.random(5 * n_k)
    emu.mean = torch.tensor(mean_h, dtype=torch.float64, device="cuda")
    emu.sd = torch.tensor(sd_h, dtype=torch.float64, device="cuda")
    P = torch.tensor(pts, dtype=torch.float64, device="cuda")
    E = torch.zeros((n, 5, n_k), dtype=torch.float64, device="cuda")
    emu.predict(P, E)
    torch.cuda.synchronize()
    lo = np.array([r[0] for r in EMU_RANGES]); hi = np.array([r[1] for r in EMU_RANGES])
    X = (2.0 * (pts - lo) / (hi - lo) - 1.0).astype(np.float32)
    Yl = np.zeros((n, 5 * n_k), dtype=np.float32)
    for r0 in range(0, n, 512):
        Xd = torch.tensor(X[r0:r0 + 512], device="cuda")
        Yd = torch.zeros((Xd.shape[0], 5 * n_k), dtype=torch.float32, device="cuda")
        emu.net.forward(Xd, Yd)
        torch.cuda.synchronize()
        Yl[r0:r0 + 512] = Yd.cpu().numpy()
    assert np.all(np.isfinite(Yl))
    pref = np.where(np.arange(5)[None, :] < 3, (pts[:, 0] ** 2 * pts[:, 3] ** 2)[:, None],
                    (pts[:, 0] * pts[:, 3] ** 2)[:, None])
    want = (Yl.astype(np.float64) * sd_h + mean_h).reshape(n, 5, n_k) * pref[:, :, None]
    scale = np.abs(want)
    shot = 2.0 * 0.2 ** 2 / 1.4e-3 * pts[:, 4][:, None]
    want[:, 0, :] += shot
    scale[:, 0, :] += np.abs(shot)
    got = E.cpu().numpy()
    # a one-ulp change of any FP32 network output moves its decoded value by
    # about 6e-8 of its size; the decoding itself (FP64, device vs host,
    # fused or separate roundings) by about 1e-16 of the terms' size
    assert np.max(np.abs(got - want) / scale) < 1e-12


def test_emulator_rejects_degenerate_points_and_ranges(lpp):
    """lpp_emulator_encode refuses a training point whose prefactor is zero
    (A = 0 lies inside the amplitude range but has no shape to learn: its
    standardised shapes would be inf/NaN and spoil every column's
    statistics), and lpp_emulator_predict refuses a range with hi <= lo (the
    encoding would divide by zero)."""
    import torch
    from paper_2202_11839_amd.emulator import Emulator
    from synth import EMU_RANGES, latin_hypercube
    n_k = 30
    pts = latin_hypercube(64, EMU_RANGES, seed=2)
    pts[17, 0] = 0.0
    P = torch.tensor(pts, dtype=torch.float64, device="cuda")
    Y = torch.ones((64, 5, n_k), dtype=torch.float64, device="cuda")
    emu = Emulator(EMU_RANGES, n_k=n_k, max_batch=64, seed=1)
    with pytest.raises(lpp.LppError) as e:
        emu.fit(P, Y, 1.4e-3, 0.2, epochs=1, batch=32)
    assert e.value.status == 1
    pts[17, 0] = 0.01
    P = torch.tensor(pts, dtype=torch.float64, device="cuda")
    emu.fit(P, Y, 1.4e-3, 0.2, epochs=1, batch=32)
    out = torch.zeros((64, 5, n_k), dtype=torch.float64, device="cuda")
    emu.predict(P, out)
    bad = list(EMU_RANGES)
    bad[2] = (1.0, 1.0)
    emu.ranges = [float(v) for r in bad for v in r]
    with pytest.raises(lpp.LppError) as e:
        emu.predict(P, out)
    assert e.value.status == 1


def test_field_level_validation_cases(lpp):
    """The paper's validation in small (Sec. IV.A-C): field-level mocks in its
    BOSS-NGC-like window on a 256^3 mesh of its 3000 Mpc/h box (8 mocks).
    Case (a), LPP with each node's own line of sight, and case (c), GPP of a
    field projected along one direction, agree with their window-convolved
    templates (lpp_template_multipoles on the window's FFT multipoles) for the
    lowest moments GD_L2 and PLUS_l0 at 0.02 <= k <= 0.1 within 4 sigma + 3 %;
    case (b), GPP of the locally projected field, misses the GD_L2 template
    by more than 20 % at every such k."""
    import math
    import torch
    from synth import power_spectrum
    from synth.fieldmocks import FieldMocks
    n, box, nb, dn = 256, 3000.0, 12, (4, 1)
    fm = FieldMocks(n=n, box=box)
    common = dict(assignment=1, interlacing=0, compensate=0, precision="f32", lmax=4, n_kbins=nb, dn=dn)
    pl = lpp.Plan(n, box, tuple(fm.origin), tuple(fm.observer), **common)
    pg = lpp.Plan(n, box, tuple(fm.origin), tuple(fm.observer), los=tuple(fm.nhat), **common)
    s = pl.series
    runs = {c: [] for c in "abc"}
    res = None
    for mock in range(8):
        gl, gg, ran = fm.realise(1000 + mock)
        for case, plan, gal in (("a", pl, gl), ("b", pg, gl), ("c", pg, gg)):
            res = plan.estimate(gal, ran)
            v = np.array(res["re"])
            v[s.index("PLUS_l0")] += res["shot_plus"]
            runs[case].append(v)
    del pl, pg
    torch.cuda.empty_cache()
    kgrid = np.exp(np.linspace(np.log(1e-5), np.log(1e3), 4096))
    pfid = power_spectrum(kgrid)
    from oracle import window as OW   # sigma8 of the fiducial spectrum, as the template path computes it
    par = np.array([[-1.0, 1.0, 0.0, OW.sigma8(kgrid, pfid), 0.0]])
    keff = np.asarray(res["k_eff"])
    sel = (keff >= 0.02) & (keff <= 0.1)

    def template(los):
        w = lpp.Plan(2 * n, 2 * box, tuple(fm.origin - box / 2), tuple(fm.observer), assignment=1, interlacing=0,
                     compensate=0, precision="f32", lmax=4, n_kbins=8, los=los)
        win = w.window_multipoles(ran, 1.0, lmax=8, n_rbins=250, rmax=box)
        ok = win["counts"] > 0
        return lpp.template_multipoles(pfid, 1e-5, 1e3, win["r_eff"][ok], win["Q"][:, ok], par, keff[sel], 1.0,
                                       0.0)[0]
    ta, tc = template(None), template(tuple(fm.nhat))
    names = list(lpp.TEMPLATE_SERIES)
    for case, T in (("a", ta), ("c", tc)):
        v = np.stack(runs[case])
        mean, err = v.mean(axis=0), v.std(axis=0, ddof=1) / math.sqrt(v.shape[0])
        for nm in ("GD_L2", "PLUS_l0"):
            t = T[names.index(nm)]
            d = np.abs(mean[s.index(nm)][sel] - t)
            assert np.all(d <= 4 * err[s.index(nm)][sel] + 0.03 * np.abs(t)), (case, nm, d / np.abs(t))
    vb = np.stack(runs["b"]).mean(axis=0)[s.index("GD_L2")][sel]
    t = ta[names.index("GD_L2")]
    assert np.all(np.abs(vb - t) > 0.2 * np.abs(t)), np.abs(vb - t) / np.abs(t)
