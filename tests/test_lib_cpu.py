"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function include/lpp.h declares, validates configurations, and its tables
(series names, k-shell thresholds) agree with the oracle's definitions."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpp.h")


def _lib():
    import paper_2202_11839_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("liblpp.so not built (run __graft_entry__.build())")
    return pkg


def test_exports_match_header():
    pkg = _lib()
    lib = pkg.load()
    decl = re.findall(r"^(?:lpp_status|const char\*)\s+(lpp_\w+)\s*\(", open(HEADER).read(), re.M)
    assert len(decl) >= 13
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(decl) == sorted(pkg.EXPORTS)
    assert "gfx950" in pkg.version()


def _cfg(**kw):
    from paper_2202_11839_amd._lib import Config
    c = Config()
    c.mesh_n = kw.get("mesh_n", 32)
    c.box_size = kw.get("box_size", 100.0)
    c.box_origin = (C.c_double * 3)(0.0, 0.0, 0.0)
    c.observer = (C.c_double * 3)(-10.0, -10.0, -10.0)
    c.assignment = kw.get("assignment", 3)
    c.interlacing = kw.get("interlacing", 1)
    c.compensate = 1
    c.precision = kw.get("precision", 0)
    c.lmax = kw.get("lmax", 4)
    c.spectra = kw.get("spectra", 15)
    c.n_kbins = kw.get("n_kbins", 8)
    c.dn_num, c.dn_den = kw.get("dn", (0, 0))
    c.global_los = kw.get("global_los", 0)
    c.los = (C.c_double * 3)(*kw.get("los", (0.0, 0.0, 0.0)))
    return c


@pytest.mark.parametrize("bad", [dict(mesh_n=48), dict(mesh_n=8), dict(mesh_n=2048), dict(box_size=-1.0),
                                 dict(assignment=4), dict(interlacing=2), dict(precision=3), dict(lmax=3),
                                 dict(lmax=10), dict(spectra=0), dict(spectra=16), dict(n_kbins=0),
                                 dict(dn=(17, 1), n_kbins=1), dict(dn=(-1, 2)), dict(lmax=2, spectra=8),
                                 dict(lmax=0, spectra=2), dict(global_los=2, los=(0.0, 0.0, 1.0)),
                                 dict(global_los=1), dict(global_los=1, los=(0.0, float("nan"), 1.0))])
def test_plan_validation(bad):
    pkg = _lib()
    lib = pkg.load()
    h = C.c_void_p()
    st = lib.lpp_plan_create(C.byref(_cfg(**bad)), C.byref(h))
    assert st == 1  # LPP_E_INVALID
    assert not h.value


def test_global_line_of_sight_config():
    """A global line of sight of any positive length is accepted (and the
    observer ignored); its series are those of the local-LOS plan."""
    pkg = _lib()
    lib = pkg.load()
    for los in ((0.0, 0.0, 1.0), (3.0, -4.0, 12.0), (1e-200, 0.0, 0.0), (1e300, 1e300, 0.0)):
        h = C.c_void_p()
        assert lib.lpp_plan_create(C.byref(_cfg(global_los=1, los=los)), C.byref(h)) == 0
        assert lib.lpp_plan_destroy(h) == 0
    a = pkg.Plan(32, 100.0, (0.0, 0.0, 0.0), (-5.0, -5.0, -5.0), n_kbins=7)
    b = pkg.Plan(32, 100.0, (0.0, 0.0, 0.0), (-5.0, -5.0, -5.0), n_kbins=7, los=(0.0, 1.0, 1.0))
    assert a.series == b.series


def test_plan_tables_match_oracle():
    pkg = _lib()
    from oracle import estimator as E, mesh as M
    for lmax in (0, 2, 4, 6, 8):
        for fams, mask in ((("DD", "GD", "PLUS", "MINUS"), 15), (("DD",), 1), (("PLUS", "MINUS"), 12)):
            if lmax < 4 and "MINUS" in fams or lmax < 2 and "GD" in fams:
                continue
            p = pkg.Plan(32, 100.0, (0.0, 0.0, 0.0), (-5.0, -5.0, -5.0), lmax=lmax, spectra=mask, n_kbins=7)
            assert p.series == E.series_names(lmax, fams)
    # null arguments and out-of-range names
    lib = pkg.load()
    assert lib.lpp_plan_create(None, None) == 1
    p = pkg.Plan(64, 100.0, (0.0, 0.0, 0.0), n_kbins=10)
    assert lib.lpp_series_name(p.handle, 99) is None
    assert lib.lpp_series_name(p.handle, -1) is None
    sz = C.c_size_t()
    assert lib.lpp_workspace_size(p.handle, 1000, 5000, C.byref(sz)) == 0
    assert sz.value > 4 * 64 ** 3 * 8  # at least the four complex meshes
    assert lib.lpp_workspace_size(p.handle, 0, 5000, C.byref(sz)) == 1
    assert pkg.load().lpp_status_string(6) == b"workspace too small"


def test_workspace_too_small_is_reported():
    pkg = _lib()
    lib = pkg.load()
    p = pkg.Plan(32, 100.0, (0.0, 0.0, 0.0), n_kbins=4)
    # a misaligned pointer is rejected without touching a device
    assert lib.lpp_set_workspace(p.handle, C.c_void_p(0x1001), 1 << 20) == 1


def test_tuning_defaults_validation_and_cache(tmp_path, monkeypatch):
    """Launch shapes: defaults resolve without a device, unsupported values are
    rejected and leave the plan unchanged, and a plan created while
    LPP_AUTOTUNE_CACHE names a cache file starts from its record."""
    pkg = _lib()
    monkeypatch.delenv("LPP_AUTOTUNE_CACHE", raising=False)
    plan = pkg.Plan(512, 1700.0, (-50.0, -50.0, -50.0), precision="f32", lmax=4, n_kbins=50)
    t = plan.tuning()
    # FP32 up to N = 512: ten shape fields per pass (the node-parallel deposit)
    assert t == {"fft_rows_x": 8, "fft_cols_y": 16, "fft_cols_z": 8, "bin_blocks": 8192, "gather_density": 8,
                 "gather_shape": 10, "serial": 0, "fft_streaming": 15, "unfused": 0}
    for bad in (dict(fft_rows_x=3), dict(fft_rows_x=4), dict(fft_rows_x=64), dict(fft_cols_y=32), dict(fft_cols_z=4),
                dict(bin_blocks=10), dict(bin_blocks=100000), dict(gather_density=9), dict(gather_shape=11),
                dict(serial=2), dict(fft_streaming=7), dict(fft_streaming=16), dict(unfused=2), dict(unfused=-1)):
        with pytest.raises(pkg.LppError):
            plan.set_tuning(**bad)
        assert plan.tuning() == t
    plan.set_tuning(fft_cols_y=8, gather_density=2)
    assert plan.tuning()["fft_cols_y"] == 8 and plan.tuning()["gather_density"] == 2
    # the y pass streams by default only when its runs fill 128-byte lines:
    # not with 8 FP32 lines (64-byte runs), always in FP64 (0 = the default)
    assert plan.tuning()["fft_streaming"] == 15
    plan.set_tuning(fft_streaming=0)
    assert plan.tuning()["fft_streaming"] == 8 | 1 | 4
    plan.set_tuning(fft_streaming=8 | 2)
    assert plan.tuning()["fft_streaming"] == 10
    # FP64: the default strided block holds one z-group of one column; more
    # lines than 1024 threads or one CU's LDS allow are refused
    p64 = pkg.Plan(1024, 1700.0, (-50.0, -50.0, -50.0), precision="f64", lmax=4, n_kbins=50)
    assert p64.tuning()["fft_cols_y"] == 8 and p64.tuning()["fft_cols_z"] == 8 and p64.tuning()["fft_rows_x"] == 8
    assert p64.tuning()["fft_streaming"] == 15
    p1k = pkg.Plan(1024, 1700.0, (-50.0, -50.0, -50.0), precision="f32", lmax=4, n_kbins=50)
    assert p1k.tuning()["fft_streaming"] == 13
    # a mesh of at most 256 MiB stays in the Infinity Cache between passes: only the z pass streams
    p256 = pkg.Plan(256, 1700.0, (-50.0, -50.0, -50.0), precision="f32", lmax=4, n_kbins=50)
    assert p256.tuning()["fft_streaming"] == 8 | 4
    # four shape fields per pass at 1024^3 (two sets of twenty meshes would not fit)
    assert p1k.tuning()["gather_shape"] == 4 and p1k.tuning()["gather_density"] == 8
    with pytest.raises(pkg.LppError):
        p1k.set_tuning(gather_shape=5)
    for bad in (dict(fft_cols_y=16), dict(fft_cols_z=16)):
        with pytest.raises(pkg.LppError):
            p64.set_tuning(**bad)
    with pytest.raises(pkg.LppError):
        p64.set_tuning(fft_rows_x=16)
    # FP64 at N = 1024: at most four density and two shape fields per deposit
    # pass (two sets of four 17 GB work meshes); up to N = 512 eight and four
    assert p64.tuning()["gather_shape"] == 2 and p64.tuning()["gather_density"] == 4
    p64s = pkg.Plan(512, 1700.0, (-50.0, -50.0, -50.0), precision="f64", lmax=4, n_kbins=50)
    assert p64s.tuning()["gather_shape"] == 4 and p64s.tuning()["gather_density"] == 8
    with pytest.raises(pkg.LppError):
        p64.set_tuning(gather_shape=3)
    with pytest.raises(pkg.LppError):
        p64.set_tuning(gather_density=5)
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"key": "N256_f32_p3_il1", "fft_rows_x": 8, "fft_cols_y": 8, "bin_blocks": 1024, '
                     '"gather_density": 3, "gather_shape": 1}\n'
                     '{"key": "N512_f32_p3_il1", "fft_rows_x": 16, "fft_cols_y": 8, "fft_cols_z": 16, '
                     '"bin_blocks": 4096, '
                     '"gather_density": 2, "gather_shape": 1}\n')
    monkeypatch.setenv("LPP_AUTOTUNE_CACHE", str(cache))
    tuned = pkg.Plan(512, 1700.0, (-50.0, -50.0, -50.0), precision="f32", lmax=4, n_kbins=50)
    assert tuned.tuning() == {"fft_rows_x": 16, "fft_cols_y": 8, "fft_cols_z": 16, "bin_blocks": 4096,
                              "gather_density": 2, "gather_shape": 1, "serial": 0, "fft_streaming": 13,
                              "unfused": 0}
    other = pkg.Plan(512, 1700.0, (-50.0, -50.0, -50.0), precision="f32", assignment=2, lmax=4, n_kbins=50)
    assert other.tuning() == t


def test_window_coefficients_of_the_library_match_the_paper_and_the_oracle():
    """The library's host-side Q^X_{l l'} coefficients (used by the template
    path) against the values printed in the paper and the oracle's exact ones."""
    import json
    from fractions import Fraction
    from oracle import special as S
    pkg = _lib()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "window_coefficients.json")))
    for e in gold["entries"]:
        for lpp_, q in zip((0, 2, 4, 6, 8), e["q"]):
            assert abs(pkg.window_coefficient(e["mX"], e["l"], e["lp"], lpp_) - float(Fraction(q))) < 1e-14, e
    for mX in (0, 2, 4):
        for l in range(mX, 9, 2):
            for lp in range(mX, 9, 2):
                for lpp_ in range(0, 17, 2):
                    want = float(S.window_coef(mX, l, lp, lpp_))
                    assert abs(pkg.window_coefficient(mX, l, lp, lpp_) - want) < 1e-13, (mX, l, lp, lpp_)


def test_bench_traffic_record_applies_only_to_its_kernels():
    """The committed counter record of the strided FFT passes is attached to a
    bench line only when the timed y and z kernels match its kernel pattern
    (another mesh size or line count gets none) and its hashed sources are
    the current ones."""
    import hashlib
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "fft_zb_strided_c2_traffic.json")))
    default = bench.strided_kernel_name(512, {"fft_streaming": 15, "fft_cols_y": 16, "fft_cols_z": 8}, names_only=True)
    assert default == ["fft_zb_kernel<float, 512, 16, false, true>", "fft_zb_kernel<float, 512, 8, false, true>"]
    assert all(re.fullmatch(rec["kernel"], k) for k in default)
    current = all(hashlib.sha256(open(os.path.join(ROOT, "paper_2202_11839_amd", "csrc", f), "rb").read()).hexdigest()
                  == h for f, h in rec["sources_sha256"].items())
    assert bench.committed_traffic(default) == (rec["bytes_per_launch"] if current else None)
    for n, t in ((1024, {"fft_streaming": 13, "fft_cols_y": 8, "fft_cols_z": 8}),
                 (512, {"fft_streaming": 13, "fft_cols_y": 8, "fft_cols_z": 8}),
                 (256, {"fft_streaming": 15, "fft_cols_y": 16, "fft_cols_z": 8})):
        assert bench.committed_traffic(bench.strided_kernel_name(n, t, names_only=True)) is None, (n, t)
    assert bench.committed_traffic([]) is None
    assert rec["bytes_per_launch"] == rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
