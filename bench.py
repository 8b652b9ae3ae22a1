#!/usr/bin/env python
"""Throughput of the LPP multipole estimator on one MI355X.

One step = one full estimate (Sec. III.A): a galaxy catalog with shapes and
its random catalog, already resident in HBM, in; every multipole series
(DD l<=4, GD L=2,4, PLUS l<=4, MINUS L=4, EE/BB), the normalisation and the
shot noise per k-shell out.  The default workload is the 512^3 single mock:
wedge footprint RA 0-90 deg, Dec 0-40 deg, comoving distance 1000-1600 Mpc/h,
1.5M galaxies drawn from a 512^3 Gaussian random field with tidal shapes,
15M randoms, TSC with interlacing, 50 shells.

Prints ONE JSON line (rank 0) with estimates/s, the roofline of the dominant
kernel from live HIP-event timings, the FP64-path rate and the CPU oracle
baseline timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def to_device(cat, torch):
    from synth import Catalog
    f = lambda a: None if a is None else torch.from_numpy(a).to("cuda", non_blocking=False).contiguous()
    return Catalog(f(cat.x), f(cat.y), f(cat.z), f(cat.w), f(cat.nbar), f(cat.g1), f(cat.g2))


SERIAL = 0  # --serial: deposits and transforms one after the other on one stream


def plan_for(lpp, wl, precision):
    plan = lpp.Plan(wl["mesh"], wl["box"], wl["origin"], wl["observer"], assignment=wl["assignment"],
                    interlacing=wl["interlacing"], precision=precision, lmax=wl["lmax"], n_kbins=wl["n_kbins"])
    if SERIAL:
        plan.set_tuning(serial=1)
    return plan


def time_steps(plan, gdev, rdev, steps, warmup, torch, profile=False):
    for _ in range(warmup):
        plan.estimate(gdev, rdev)
    torch.cuda.synchronize()
    plan.set_profiling(profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for i in range(steps):
        res = plan.estimate(gdev, rdev)
        log(f"step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile() if profile else None
    plan.set_profiling(False)
    return (t1 - t0), res, prof


def fp32_errors(r32, r64):
    """Largest error of each FP32 multipole against the FP64 path on the same
    catalogs, over the shells with modes, relative to the series' scale: the
    auto power of the fields in its product before shot-noise subtraction
    (DD: P_dd^(0) + N_dd; PLUS, MINUS, EE, BB: P_+^(0) + N_+; GD: their
    geometric mean), the scale the parity tests use."""
    import numpy as np
    s = r64["series"]
    dd = np.abs(np.asarray(r64["re"][s.index("DD_l0")]) + r64["shot_dd"])
    pp = np.abs(np.asarray(r64["re"][s.index("PLUS_l0")]) + r64["shot_plus"])
    sel = np.asarray(r64["n_modes"]) > 0
    out = {}
    for i, name in enumerate(s):
        sc = dd if name.startswith("DD") else (np.sqrt(dd * pp) if name.startswith("GD") else pp)
        e = max(np.max(np.abs(np.asarray(r32[p][i]) - np.asarray(r64[p][i]))[sel] / sc[sel]) for p in ("re", "im"))
        out[name] = float(f"{e:.3g}")
    return out


def launches_per_set(res):
    """Transforms per estimate at l <= 4 with interlacing: the density set has
    15 fields (one packed mesh each), the shape set 38 (two interlaced meshes
    each): 1 + 5 + 9 plus-type, 5 + 9 cross, 9 minus.  Every transform runs
    one y pass of the strided kernel; the z pass runs as its own launch for
    the density meshes and the two meshes of the shape set's base only (the
    other shape fields take it inside the fused shell-sum kernel).  Returns
    (density meshes, shape meshes, shape meshes with a z-pass launch)."""
    assert len(res["series"]) == 15, res["series"]
    return 15, 76, 2


def strided_pass_bytes(pos, wl):
    """HBM bytes (y, z) that the y pass and the z pass of one transform move,
    given the footprint of the object set (complex float32 nodes):
      y pass: read every flagged node row, write the (kx, ky) inside the last
              shell in every flagged plane;
      z pass: read the flagged planes of the (kx, ky) columns inside the last
              shell, write the modes inside the last shell.
    Flags follow the deposit's reach: node row (y, z) is flagged when a cell
    row (y + dy, z + dz), dy, dz in -2..1, holds an object."""
    import numpy as np
    n, box = wl["mesh"], wl["box"]
    c = np.floor((pos - np.asarray(wl["origin"])[None, :]) / (box / n)).astype(np.int64)
    c = np.clip(c, 0, n - 1)
    occ = np.zeros((n, n), dtype=bool)
    occ[c[:, 1], c[:, 2]] = True
    row = np.zeros_like(occ)
    for dy in range(-2, 2):
        for dz in range(-2, 2):
            row |= np.roll(np.roll(occ, -dy, axis=0), -dz, axis=1)
    planes = int(row.any(axis=0).sum())
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    qmax = (n // 2) ** 2
    circle = int((m[:, None] ** 2 + m[None, :] ** 2 < qmax).sum())
    sphere = int((m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2 < qmax).sum())
    y_bytes = 8 * (int(row.sum()) * n + planes * circle)
    z_bytes = 8 * (circle * planes + sphere)
    return y_bytes, z_bytes


def strided_kernel_name(n, tuning, names_only=False):
    """The instantiation(s) of the FFT kernel that run the y and z passes:
    <float, N, lines per workgroup, along-x = false, non-temporal accesses>."""
    st = tuning["fft_streaming"]
    y = (tuning["fft_cols_y"], bool(st & 8 and st & 2))
    z = (tuning["fft_cols_z"], bool(st & 8 and st & 4))
    name = lambda c: "fft_zb_kernel<float, %d, %d, false, %s>" % (n, c[0], "true" if c[1] else "false")
    if names_only:
        return [name(y), name(z)]
    if y == z:
        return name(y) + " (y and z passes)"
    return "%s (y pass), %s (z pass)" % (name(y), name(z))


def committed_traffic(kernel_names):
    """Counter-measured HBM bytes per launch of the strided FFT pass at the C2
    workload, from the committed rocprofv3 summary, if it was taken on the
    current sources (the SHA-256 of the kernel source and of the host code
    that sequences its launches are recorded in the summary) and on the
    kernels being timed (every name matches the summary's kernel pattern, so
    another mesh size or launch shape gets none)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "fft_zb_strided_c2_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        pattern = rec.get("kernel")
        if not pattern or not kernel_names or not all(re.fullmatch(pattern, k) for k in kernel_names):
            return None
        digests = rec.get("sources_sha256") or {}
        if not digests:
            return None
        for name, want in digests.items():
            with open(os.path.join(ROOT, "paper_2202_11839_amd", "csrc", name), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
    except OSError:
        return None
    return rec.get("bytes_per_launch")


def model_bytes_c2(wl, n_gal, n_ran):
    """The whole-estimate algorithmic byte model of the l <= 4 estimate: per
    field and interlaced copy a deposit write (1 M_c), a two-pass transform
    read and write (4 M_c) and a shell-sum read (1 M_c), plus one read of the
    field's base (1 M_c), the real density fields at half: (38 x 13 +
    15 x 6.5) M_c, M_c = N^3 x 8 B; plus one read of the FP64 catalog columns."""
    mc = 8.0 * wl["mesh"] ** 3
    return (38 * 13 + 15 * 6.5) * mc + 8.0 * (7 * n_gal + 5 * n_ran)


def committed_estimate_traffic():
    """Counter-measured HBM bytes of one whole estimate (every kernel's
    FETCH_SIZE and WRITE_SIZE, scaled by the calibration copy) from the
    committed record, if it was taken on the current kernel and host sources
    (their SHA-256 are in the record)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "estimate_c2_fp32_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        digests = rec.get("sources_sha256") or {}
        if not digests:
            return None
        for name, want in digests.items():
            with open(os.path.join(ROOT, "paper_2202_11839_amd", "csrc", name), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
    except OSError:
        return None
    return rec.get("bytes_per_estimate")


def batch_c3(lpp, torch, k, reps, tune_cache):
    """The 256^3 batch workload: k mocks of the 64-mock size ladder
    N_i = round(0.2e6 10^(i/63)) galaxies (10x randoms; k = 64 is the whole
    ladder), each with its own GRF, device-resident in float32, through
    lpp_estimate_batch (one captured graph, replayed) with the launch shapes
    lpp_autotune picks on the largest mock (cached in tune_cache), and, for
    comparison, through lpp_estimate one by one."""
    import numpy as np
    from synth import WORKLOADS, c3_sizes, make_catalogs
    wl = dict(WORKLOADS["c3"])
    ladder = c3_sizes(64)
    pick = sorted(set(int(round(x)) for x in np.linspace(0, 63, k)))
    t0 = time.perf_counter()
    gals, rans = [], []
    for i in pick:
        g, r = make_catalogs(wl, mock=i, n_gal=ladder[i], n_ran=10 * ladder[i])
        f = lambda c: type(c)(*[None if v is None else torch.tensor(v, dtype=torch.float32, device="cuda")
                                for v in (c.x, c.y, c.z, c.w, c.nbar, c.g1, c.g2)])
        gals.append(f(g))
        rans.append(f(r))
        if len(gals) % 16 == 0:
            log(f"batch: {len(gals)}/{len(pick)} mocks generated ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    ngal = sum(ladder[i] for i in pick)
    log(f"batch: {len(pick)} mocks generated in {time.perf_counter() - t0:.1f} s ({ngal} galaxies)")
    plan = plan_for(lpp, wl, "f32")
    default_shapes = plan.tuning()
    t0 = time.perf_counter()
    tuned = plan.autotune(gals[-1], rans[-1], tune_cache)
    t_tune = time.perf_counter() - t0
    log(f"batch: autotuned on the largest mock in {t_tune:.1f} s: {tuned}")
    outs = plan.estimate_batch(gals, rans)  # capture
    assert all(isinstance(o, dict) for o in outs), outs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.estimate_batch(gals, rans)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    for g, r in zip(gals, rans):  # warm-up of the eager path
        plan.estimate(g, r)
        break
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, r in zip(gals, rans):
        plan.estimate(g, r)
    torch.cuda.synchronize()
    de = time.perf_counter() - t0
    caps, launches = plan.batch_stats()
    # the batch's algorithmic bytes per mock from the whole-estimate model (two-pass transforms)
    mc = 8.0 * wl["mesh"] ** 3
    model_bytes = (38 * 13 + 15 * 6.5) * mc
    log(f"batch: {len(pick)} mocks in {1e3 * dt:.1f} ms per batch (graph), {1e3 * de:.1f} ms one by one")
    return {"workload": f"{len(pick)} mocks of the 256^3 wedge batch (mock indices {pick[0]}..{pick[-1]} of the "
                        f"0.2M-2M galaxy ladder, 10x randoms)", "mocks": len(pick), "galaxies": ngal,
            "mocks_per_s": round(len(pick) / dt, 3), "ms_per_batch": round(1e3 * dt, 2),
            "ms_per_mock": round(1e3 * dt / len(pick), 3),
            "model_frac_per_mock": round(model_bytes / (dt / len(pick)) / 1e9 / HBM_PEAK_GBS, 4),
            "eager_mocks_per_s": round(len(pick) / de, 3), "graph_captures": caps, "graph_launches": launches,
            "autotune_s": round(t_tune, 1), "tuning": tuned, "default_tuning": default_shapes}


def emulator_c5(lpp, torch, wl, ran, gal, rdev, epochs):
    """Window multipoles Q_l (l <= 8) of the 512^3 workload's randoms on a
    padded 3400 Mpc/h box (512^3, r <= 2000 Mpc/h in 200 shells), the plain
    template path (FFTLog, FP64) over a 22,000-point Latin hypercube of
    (A, b, f, sigma8, s_N), and the BF16 emulator trained on 20,000 of them;
    accuracy on the other 2,000 and the time per 2,000 points of each route,
    plus the separable evaluation (4 basis templates, a 4 x 150 map per point)."""
    import numpy as np
    from paper_2202_11839_amd.emulator import Emulator, accuracy
    from synth import EMU_RANGES, latin_hypercube, power_spectrum
    out = {}
    plan = lpp.Plan(512, 3400.0, (-50.0, -50.0, -50.0), wl["observer"], assignment=3, interlacing=1,
                    precision="f32", lmax=4, n_kbins=50)
    alpha = float(np.sum(gal.w) / np.sum(ran.w))
    plan.window_multipoles(rdev, alpha, lmax=8, n_rbins=200, rmax=2000.0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    win = plan.window_multipoles(rdev, alpha, lmax=8, n_rbins=200, rmax=2000.0)
    out["window_ms"] = round(1e3 * (time.perf_counter() - t0), 1)
    del plan
    torch.cuda.empty_cache()
    sel = win["counts"] > 0
    r_q, Q = win["r_eff"][sel], win["Q"][:, sel]
    kgrid = np.exp(np.linspace(np.log(1e-5), np.log(1e3), 4096))
    pfid = power_spectrum(kgrid)
    kout = np.arange(1, 31) * 0.01
    nbar = float(gal.nbar[0])  # constant over the catalog
    sig = float(wl["sigma"])
    pts = latin_hypercube(22000, EMU_RANGES, seed=0)
    P = torch.tensor(pts, dtype=torch.float64, device="cuda")
    Y = torch.zeros((22000, 5, 30), dtype=torch.float64, device="cuda")
    lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, P[:100], kout, nbar, sig, out=Y[:100])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, P, kout, nbar, sig, out=Y)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out["plain_ms_22000"] = round(1e3 * t_plain, 1)
    t0 = time.perf_counter()
    for _ in range(5):
        lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, P[20000:], kout, nbar, sig, out=Y[20000:])
    torch.cuda.synchronize()
    t_plain2k = (time.perf_counter() - t0) / 5
    emu = Emulator(EMU_RANGES, n_k=30, max_batch=4096, seed=1)
    t0 = time.perf_counter()
    loss = emu.fit(P[:20000], Y[:20000], nbar, sig, epochs=epochs, batch=128, lr0=5e-4, lr1=1e-5, seed=2)
    torch.cuda.synchronize()
    out["train_s"] = round(time.perf_counter() - t0, 2)
    out["train_loss"] = loss
    E = torch.zeros((2000, 5, 30), dtype=torch.float64, device="cuda")
    emu.predict(P[20000:], E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        emu.predict(P[20000:], E)
    torch.cuda.synchronize()
    t_emu = (time.perf_counter() - t0) / 10
    rel, perk = accuracy(E.cpu().numpy(), Y[20000:].cpu().numpy())
    names = ["P+_0", "P+_2", "P+_4", "Pgd_2", "Pgd_4"]
    out["heldout_max_rel_err"] = {n_: round(float(rel[:, i].max()), 5) for i, n_ in enumerate(names)}
    out["heldout_p99_rel_err"] = {n_: round(float(np.percentile(rel[:, i], 99)), 5) for i, n_ in enumerate(names)}
    out["heldout_max_perk_rel_err"] = {n_: round(float(perk[:, i].max()), 5) for i, n_ in enumerate(names)}
    out["within_1pct"] = bool(rel.max() <= 0.01)
    out["plain_ms_2000"] = round(1e3 * t_plain2k, 2)
    out["emulator_ms_2000"] = round(1e3 * t_emu, 3)
    out["speedup_vs_plain"] = round(t_plain2k / t_emu, 1)
    # separable evaluation: four basis templates from the plain path, then a 4 x 150 map per point
    basis_pts = np.array([[1.0, 1.0, 0.0, 1.0, 0.0], [1.0, 0.0, 1.0, 1.0, 0.0]])
    Bm = lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, basis_pts, kout, nbar, sig)
    plus = Bm[0, :3]                       # A^2 sigma8^2 = 1
    gd_b = Bm[0, 3:]                       # (7b + f) = 7, f = 0
    gd_f = Bm[1, 3:]                       # (7b + f) = 1, f = 1
    basis = np.stack([np.concatenate([plus.ravel(), np.zeros(60)]), np.concatenate([np.zeros(90), gd_b.ravel() / 7.0]),
                      np.concatenate([np.zeros(90), (gd_f - gd_b / 7.0).ravel()]),
                      np.concatenate([np.full(30, 2 * sig * sig / nbar), np.zeros(120)])])
    hp = pts[20000:]
    t0 = time.perf_counter()
    coef = np.stack([hp[:, 0] ** 2 * hp[:, 3] ** 2, hp[:, 0] * hp[:, 3] ** 2 * (7 * hp[:, 1] + hp[:, 2]),
                     hp[:, 0] * hp[:, 3] ** 2 * hp[:, 2], hp[:, 4]], axis=1)
    sepv = coef @ basis
    t_sep = time.perf_counter() - t0
    sep_rel, _ = accuracy(sepv.reshape(2000, 5, 30), Y[20000:].cpu().numpy())
    out["separable_ms_2000_host"] = round(1e3 * t_sep, 3)
    out["separable_max_rel_err"] = float(sep_rel.max())
    # the same separable map as one device matrix product (4 basis rows, FP64)
    coef_d = torch.tensor(coef, device="cuda")
    basis_d = torch.tensor(basis, device="cuda")
    (coef_d @ basis_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        sep_d = coef_d @ basis_d
    torch.cuda.synchronize()
    t_sep_d = (time.perf_counter() - t0) / 10
    out["separable_ms_2000_device"] = round(1e3 * t_sep_d, 4)
    out["speedup_vs_separable_host"] = round(t_sep / t_emu, 2)
    out["speedup_vs_separable_device"] = round(t_sep_d / t_emu, 2)
    del sep_d
    log(f"emulator: plain {1e3 * t_plain2k:.2f} ms / 2000 pts, emulator {1e3 * t_emu:.3f} ms, "
        f"max held-out err {rel.max():.4f}, separable {1e3 * t_sep:.3f} ms (err {sep_rel.max():.1e})")
    return out


def _shell_modes(n, n_kbins, dn):
    """Per k-shell the distinct |n|^2 of its modes and their multiplicities
    (the estimator's shells: T_b <= |n|^2 < T_{b+1}, T_b = ceil((b dn)^2),
    n != 0, |n_i| < N/2)."""
    import numpy as np
    num, den = dn
    T = [-((-(b * b * num * num)) // (den * den)) for b in range(n_kbins + 1)]
    h = int(math.isqrt(T[-1])) + 1
    m = np.arange(-h, h + 1)
    q = (m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2).ravel()
    cnt = np.bincount(q, minlength=T[-1] + 1)
    out = []
    for b in range(n_kbins):
        qs = np.arange(max(T[b], 1), T[b + 1])
        out.append((qs[cnt[qs] > 0], cnt[qs][cnt[qs] > 0]))
    return out


def validation_f2(lpp, torch, n_mocks):
    """The paper's validation (Sec. IV.A-C) at field level on its own
    geometry: Gaussian density fields on a 512^3 mesh of a 3000 Mpc/h periodic
    box, the tidal field projected at every mesh node inside the BOSS-NGC-like
    window (RA 120-260, Dec -5-70 deg, r 1000-1500 Mpc/h; 9.9M nodes) with
    each node's own line of sight, measured with the LPP estimator (case (a)),
    with the GPP estimator along the window's central direction (case (b),
    inconsistent lines of sight), and the field projected along that
    direction measured with GPP (case (c)).  The mean over the mocks is
    compared with the window-convolved templates of eq. all_convolutions
    (lpp_template_multipoles at A = -1, b = 1, f = 0, sigma8 = sigma8_fid:
    P_gd = (1-mu^2)P/2, P_+ = P_- = (1-mu^2)^2 P/4, eq. power_for_validation)
    averaged over each shell's modes, built from the window's Q_l: end-point
    FFT route on a padded 6000 Mpc/h box whose 1024^3 nodes contain the
    mock's (case (a)), midpoint and end-point pair counts of 200,000 random
    points in the window (case (a), the paper's route), and the FFT route
    about the global direction (case (c))."""
    import numpy as np
    from synth import power_spectrum
    from synth.fieldmocks import FieldMocks
    t0 = time.perf_counter()
    fm = FieldMocks()
    log(f"validation: {fm.count} window nodes ({time.perf_counter() - t0:.1f} s set-up)")
    n, box, nb, dn = 512, 3000.0, 24, (4, 1)
    common = dict(assignment=1, interlacing=0, compensate=0, precision="f32", lmax=4, n_kbins=nb, dn=dn)
    plan_l = lpp.Plan(n, box, tuple(fm.origin), tuple(fm.observer), **common)
    plan_g = lpp.Plan(n, box, tuple(fm.origin), tuple(fm.observer), los=tuple(fm.nhat), **common)
    series = plan_l.series
    sums = {c: [] for c in "abc"}
    kinfo = None
    t0 = time.perf_counter()
    t_est = 0.0
    for mock in range(n_mocks):
        gl, gg, ran = fm.realise(mock)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for case, plan, gal in (("a", plan_l, gl), ("b", plan_g, gl), ("c", plan_g, gg)):
            r = plan.estimate(gal, ran)
            v = np.array(r["re"])
            # field-level mocks carry no Poisson noise: add back what the estimator subtracted
            v[series.index("DD_l0")] += r["shot_dd"]
            v[series.index("PLUS_l0")] += r["shot_plus"]
            for name in ("EE_l0", "BB_l0"):
                v[series.index(name)] += 0.5 * r["shot_plus"]
            sums[case].append(v)
            kinfo = r
        t_est += time.perf_counter() - ts
        if (mock + 1) % 16 == 0:
            log(f"validation: {mock + 1}/{n_mocks} mocks ({time.perf_counter() - t0:.1f} s)")
    del plan_l, plan_g
    torch.cuda.empty_cache()
    # window multipoles
    alpha = 1.0
    wplan = lpp.Plan(1024, 2 * box, tuple(fm.origin - box / 2), tuple(fm.observer), assignment=1, interlacing=0,
                     compensate=0, precision="f32", lmax=4, n_kbins=8)
    win_a = wplan.window_multipoles(ran, alpha, lmax=8, n_rbins=250, rmax=box)
    del wplan
    torch.cuda.empty_cache()
    wplan = lpp.Plan(1024, 2 * box, tuple(fm.origin - box / 2), tuple(fm.observer), assignment=1, interlacing=0,
                     compensate=0, precision="f32", lmax=4, n_kbins=8, los=tuple(fm.nhat))
    win_c = wplan.window_multipoles(ran, alpha, lmax=8, n_rbins=250, rmax=box)
    del wplan
    torch.cuda.empty_cache()
    # pair counts of random points drawn uniformly in the window (the paper's
    # route): W = n W_window with n = 1/H^3 the nodes' density, so each of the
    # m points carries alpha = V_window / (m H^3)
    from synth import Catalog, seed_seq, wedge_uniform, wedge_volume
    from synth.fieldmocks import PAPER_WINDOW
    m_pts = 200_000
    rp = wedge_uniform(m_pts, seed_seq(6, 0, 3), PAPER_WINDOW["ra"], PAPER_WINDOW["dec"], PAPER_WINDOW["r"]) + \
        fm.observer[None, :]
    pts = Catalog(rp[:, 0].copy(), rp[:, 1].copy(), rp[:, 2].copy(), None, None)
    vol = wedge_volume(PAPER_WINDOW["ra"], PAPER_WINDOW["dec"], PAPER_WINDOW["r"])
    alpha_p = vol / (m_pts * fm.h ** 3)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    pairs_mid = lpp.window_pairs(pts, alpha_p, win_a["norm_I"], tuple(fm.observer), "midpoint", 8, 250, box)
    t_pairs = time.perf_counter() - tp
    pairs_end = lpp.window_pairs(pts, alpha_p, win_a["norm_I"], tuple(fm.observer), "endpoint", 8, 250, box)
    # templates, averaged over each shell's modes
    kgrid = np.exp(np.linspace(np.log(1e-5), np.log(1e3), 4096))
    pfid = power_spectrum(kgrid)
    x = 8.0 * kgrid
    wth = 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3
    s8 = math.sqrt(float(np.sum(0.5 * (np.diff(np.log(kgrid))) *
                              ((kgrid ** 3 * pfid * wth ** 2)[1:] + (kgrid ** 3 * pfid * wth ** 2)[:-1])) /
                       (2 * math.pi ** 2)))
    par = np.array([[-1.0, 1.0, 0.0, s8, 0.0]])
    kf = 2 * math.pi / box
    kfine = np.exp(np.linspace(np.log(0.5 * kf), np.log(1.2 * kf * nb * dn[0] / dn[1]), 256))
    shells = _shell_modes(n, nb, dn)

    def template(win):
        sel = win["counts"] > 0
        t = lpp.template_multipoles(pfid, 1e-5, 1e3, win["r_eff"][sel], win["Q"][:, sel], par, kfine, 1.0, 0.0)[0]
        out = np.zeros((9, nb))
        for b, (qs, mult) in enumerate(shells):
            kk = kf * np.sqrt(qs)
            for o in range(9):
                out[o, b] = np.sum(mult * np.interp(np.log(kk), np.log(kfine), t[o])) / np.sum(mult)
        return out
    tmpl = {"a_fft_endpoint": template(win_a), "a_pairs_midpoint": template(pairs_mid),
            "a_pairs_endpoint": template(pairs_end), "c_fft_global": template(win_c)}
    k_eff = np.asarray(kinfo["k_eff"])
    tnames = list(lpp.TEMPLATE_SERIES)
    rec = {"workload": (f"{n_mocks} field-level mocks, 512^3 mesh of a 3000 Mpc/h box, BOSS-NGC-like window "
                        f"RA 120-260 Dec -5-70 r 1000-1500 Mpc/h ({fm.count} nodes), NGP on the nodes, {nb} shells "
                        f"of width {dn[0] * kf:.5f} h/Mpc"),
           "mocks": n_mocks, "estimates_per_s": round(3 * n_mocks / t_est, 2),
           "window_pairs_s_200k_midpoint": round(t_pairs, 2), "k_eff": [round(v, 5) for v in k_eff],
           "n_modes": [int(v) for v in kinfo["n_modes"]]}

    def stats(case, names):
        v = np.stack(sums[case])
        mean = v.mean(axis=0)
        err = v.std(axis=0, ddof=1) / math.sqrt(v.shape[0])
        return {nm: (mean[series.index(nm)], err[series.index(nm)]) for nm in names}
    main = ["DD_l0", "GD_L2", "PLUS_l0", "PLUS_l2", "PLUS_l4", "MINUS_L4"]
    leak = ["DD_l2", "GD_L4"]
    out_cases = {}
    for case, tkey in (("a", "a_pairs_midpoint"), ("a", "a_pairs_endpoint"), ("a", "a_fft_endpoint"),
                       ("b", "a_pairs_midpoint"), ("c", "c_fft_global")):
        st = stats(case, main + leak)
        T = tmpl[tkey]
        d = {}
        for nm in main + leak:
            mean, err = st[nm]
            tv = T[tnames.index(nm)]
            ref = tv if nm in main else T[tnames.index("DD_l0" if nm == "DD_l2" else "GD_L2")]
            d[nm] = {"frac_diff": [round(float(v), 4) for v in (mean - tv) / np.abs(ref)],
                     "err_frac": [round(float(v), 4) for v in err / np.abs(ref)]}
        out_cases[f"case_{case}_vs_{tkey}"] = d
    rec["comparison"] = out_cases
    # the end-point vs midpoint difference of the window multipoles themselves
    sel = (pairs_mid["counts"] > 0) & (pairs_end["counts"] > 0)
    q0 = np.max(np.abs(pairs_mid["Q"][0][sel]))
    rec["window_endpoint_vs_midpoint_max_abs_dQ_over_Q0max"] = {
        f"l{2 * i}": round(float(np.max(np.abs(pairs_mid["Q"][i][sel] - pairs_end["Q"][i][sel])) / q0), 5)
        for i in range(5)}
    selw = sel & (win_a["counts"] > 0)
    rec["window_fft_vs_pairs_endpoint_max_abs_dQ_over_Q0max"] = {
        f"l{2 * i}": round(float(np.max(np.abs(win_a["Q"][i][selw] - pairs_end["Q"][i][selw])) / q0), 5)
        for i in range(5)}
    log(f"validation: {n_mocks} mocks x 3 estimates in {t_est:.1f} s; pairs {t_pairs:.2f} s")
    return rec


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, gal, ran):
    """The FP64 oracle (oracle.estimator.mesh64, the paper's Cartesian-tensor
    FFT route) timed on a bounded sample of the same workload, on the host
    threads scipy's FFT is given (oracle.mesh.workers()).

    The oracle's estimate is a sum of independent units, one per monomial of
    its Cartesian tensors: deposit the per-object coefficient on the grid and
    on the interlaced grid, transform both, combine, compensate, multiply by
    the monomial of khat and accumulate.  At l <= 4 it runs 23 such units on
    the density set (galaxies and randoms) and 59 on the shape set
    (galaxies), plus the shell sums.  The sample times one unit of each kind
    at the full mesh and one shell sum; the estimate's time is
    23 t_density + 59 t_shape + 15 t_shell."""
    import numpy as np
    from oracle import estimator as E, mesh as M
    n, box, origin, p = wl["mesh"], wl["box"], wl["origin"], wl["assignment"]
    cfg = E.Config(mesh=n, box=box, origin=origin, observer=wl["observer"], assignment=p,
                   interlacing=wl["interlacing"], n_kbins=wl["n_kbins"], lmax=4)
    kx, ky, kz, kk = E._khat(n)
    comp = M.compensation(n, p)
    phase = M.interlace_phase(n)
    gpos, rpos = gal.pos(), ran.pos()
    allpos = np.concatenate([gpos, rpos])
    alpha = gal.w.sum() / ran.w.sum()
    w = np.concatenate([gal.w, -alpha * ran.w])
    t0 = time.perf_counter()
    acc = kx * kx * E._transform(cfg, allpos, w, comp, phase)
    ta = time.perf_counter() - t0
    log(f"cpu baseline: one density-set unit {ta:.1f} s")
    t0 = time.perf_counter()
    acc = acc + kx * ky * E._transform(cfg, gpos, gal.w * (gal.g1 + 1j * gal.g2), comp, phase)
    tc = time.perf_counter() - t0
    log(f"cpu baseline: one shape-set unit {tc:.1f} s")
    num, den = cfg.bin_width()
    t0 = time.perf_counter()
    bidx = M.bin_index(n, cfg.n_kbins, num, den)
    E._bin_sums(cfg, bidx, acc * np.conj(acc))
    tb = time.perf_counter() - t0
    del acc, bidx, kx, ky, kz, kk
    t_est = 23 * ta + 59 * tc + 15 * tb
    return {"value": 1.0 / t_est, "unit": "estimates/s", "cores": M.workers(), "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus_visible": os.cpu_count(),
            "sample": (f"one unit of each kind of the FP64 oracle's FFT route at {n}^3 (deposit on both grids, two "
                       f"scipy FFTs, interlace combine, compensation, monomial product): density set of "
                       f"{gal.n + ran.n} objects {ta:.1f} s, shape set of {gal.n} objects {tc:.1f} s, one shell "
                       f"sum {tb:.1f} s; estimate = 23 + 59 units + 15 shell sums"),
            "seconds_sampled": round(ta + tc + tb, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--batch-mocks", type=int, default=64,
                    help="mocks of the 256^3 batch workload (spread over its 64-mock size ladder) "
                         "timed through the graph-captured batch path; 0 skips it")
    ap.add_argument("--lmax8", type=int, default=1,
                    help="1: also time the l <= 8 estimate of the same catalogs (FP32)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--emulator", type=int, default=1,
                    help="1: window multipoles of the 512^3 randoms, the plain template path over the 22,000-point "
                         "design and the emulator trained on 20,000 of them (accuracy on the other 2,000, speedup)")
    ap.add_argument("--emu-epochs", type=int, default=1500)
    ap.add_argument("--validation-mocks", type=int, default=64,
                    help="field-level mocks of the paper's validation (its 512^3, 3000 Mpc/h box and BOSS-NGC-like "
                         "window), LPP / inconsistent GPP / GPP estimates against the window-convolved templates; "
                         "0 skips it")
    ap.add_argument("--only", default="",
                    help="comma-separated legs to run alone (validation); the main estimate line is then not printed")
    ap.add_argument("--serial", type=int, default=0,
                    help="1: run each estimate's deposits and transforms on one stream (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference kernel "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    args = ap.parse_args()
    global SERIAL
    SERIAL = args.serial
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the field-parallel sharding is a design note, not code); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB done")
        return

    import paper_2202_11839_amd as lpp
    from synth import WORKLOADS, make_catalogs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.only:
        legs = set(args.only.split(","))
        rec = {}
        if "validation" in legs:
            rec["validation_f2"] = validation_f2(lpp, torch, args.validation_mocks)
        print(json.dumps(rec), flush=True)
        return
    wl = dict(WORKLOADS[args.workload])
    t0 = time.perf_counter()
    # above 512^3 the galaxies are drawn from a 512^3 GRF of the same box (the
    # clustering only shapes the footprint's occupancy; the mesh is the workload)
    gal, ran = make_catalogs(wl, mock=0, grf_mesh=min(wl["mesh"], 512))
    log(f"catalogs generated in {time.perf_counter() - t0:.1f} s: {gal.n} galaxies, {ran.n} randoms")
    gdev, rdev = to_device(gal, torch), to_device(ran, torch)
    torch.cuda.synchronize()

    plan = plan_for(lpp, wl, "f32")
    dt, res, _ = time_steps(plan, gdev, rdev, args.steps, args.warmup, torch)
    ms = 1e3 * dt / args.steps
    value = args.steps / dt
    log(f"fp32: {ms:.1f} ms/estimate, {value:.3f} estimates/s")
    # stage times and the strided pass's launch time from a profiled run
    # (profiling runs the deposits and the transforms one after the other, so
    # that every kernel's time is its own)
    psteps = max(1, min(args.steps, 2))
    _, _, prof = time_steps(plan, gdev, rdev, psteps, 0, torch, profile=True)

    # roofline of the dominant kernel: the strided (y and z) passes of the 3D transforms
    n = wl["mesh"]
    stages = {k: v for k, v in prof.items() if v[1] > 0}
    total_ms, launches = stages["fft_yz"]
    avg_ms = total_ms / launches
    nd_mesh, ns_mesh, ns_z = launches_per_set(res)
    yd, zd = strided_pass_bytes(np.concatenate([gal.pos(), ran.pos()]), wl)
    ys, zs = strided_pass_bytes(gal.pos(), wl)
    n_strided = 2 * nd_mesh + ns_mesh + ns_z
    assert launches == n_strided * psteps, (launches, n_strided)
    alg_bytes = (nd_mesh * (yd + zd) + ns_mesh * ys + ns_z * zs) / n_strided  # per launch
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = committed_traffic(strided_kernel_name(n, plan.tuning(), names_only=True))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "kernel": strided_kernel_name(n, plan.tuning()),
            "alg_bytes_per_launch": round(alg_bytes), "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "stage_ms_per_step": {k: round(v[0] / psteps, 3) for k, v in prof.items()},
            "stages_serial_ms_per_step": round(sum(v[0] for v in prof.values()) / psteps, 2)}
    # the whole estimate against the same peak: the algorithmic byte model, and
    # the counter-measured bytes of every kernel of one estimate
    mb = model_bytes_c2(wl, gal.n, ran.n) if args.workload == "c2" else None
    cb = committed_estimate_traffic() if args.workload == "c2" else None
    roof["whole_estimate"] = {
        "model_bytes": None if mb is None else round(mb),
        "model_frac": None if mb is None else round(mb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "counter_bytes": None if cb is None else round(cb),
        "counter_frac": None if cb is None else round(cb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"whole estimate: model {roof['whole_estimate']['model_frac']}, counters {roof['whole_estimate']['counter_frac']} "
        "of the HBM peak")

    extra = {}
    if args.fp64_steps > 0:
        del plan
        torch.cuda.empty_cache()
        plan64 = plan_for(lpp, wl, "f64")
        dt64, res64, _ = time_steps(plan64, gdev, rdev, args.fp64_steps, 1, torch)
        extra["fp64"] = {"value": round(args.fp64_steps / dt64, 4), "ms_per_step": round(1e3 * dt64 / args.fp64_steps, 2),
                         "fp32_rel_err_per_series": fp32_errors(res, res64)}
        log(f"fp64: {1e3 * dt64 / args.fp64_steps:.1f} ms/estimate")
        del plan64

    if args.lmax8:
        wl8 = dict(wl, lmax=8)
        plan8 = plan_for(lpp, wl8, "f32")
        dt8, res8, _ = time_steps(plan8, gdev, rdev, max(1, min(args.steps, 3)), 1, torch)
        extra["lmax8"] = {"ms_per_step": round(1e3 * dt8 / max(1, min(args.steps, 3)), 2),
                          "series": len(res8["series"]), "fft_fields": 1 + 5 + 9 + 13 + 17 + 5 + 9 + 13 + 17 +
                          1 + 5 + 9 + 13 + 17 + 9 + 13 + 17}
        log(f"lmax 8: {extra['lmax8']['ms_per_step']} ms/estimate")
        del plan8
        torch.cuda.empty_cache()
    if args.batch_mocks > 0:
        extra["batch_c3"] = batch_c3(lpp, torch, args.batch_mocks, args.batch_reps,
                                     os.path.join(ROOT, "gpurun_out", "lpp_autotune_c3.jsonl"))
    if args.validation_mocks > 0:
        extra["validation_f2"] = validation_f2(lpp, torch, args.validation_mocks)
    if args.emulator:
        extra["emulator_c5"] = emulator_c5(lpp, torch, wl, ran, gal, rdev, args.emu_epochs)

    cpu = None
    if args.cpu_baseline:
        cpu = cpu_baseline(wl, gal, ran)

    out = {
        "metric": "catalog multipole estimates/sec at 512^3 (FP32 vs FP64), %HBM peak; emulator speedup",
        "value": round(value, 4), "unit": "estimates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("single mock, 512^3 mesh, wedge RA 0-90 Dec 0-40 r 1000-1600 Mpc/h, "
                                "1.5M galaxies + 15M randoms, TSC + interlacing, l<=4, 50 shells")
                   if args.workload == "c2" else
                   ("single mock, 1024^3 mesh, wedge RA 0-90 Dec 0-40 r 1000-1800 Mpc/h, 10M galaxies + 50M "
                    "randoms, TSC + interlacing, l<=4, 80 shells") if args.workload == "c4" else args.workload,
                   "mesh": n, "n_gal": gal.n, "n_ran": ran.n, "n_kbins": wl["n_kbins"],
                   "series": len(res["series"]), "fft_fields": 53, "sums": "fp64"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
