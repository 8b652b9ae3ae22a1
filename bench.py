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
    one y pass and one z pass of the strided kernel."""
    assert len(res["series"]) == 15, res["series"]
    return 15, 76


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


def batch_c3(lpp, torch, k, reps):
    """The 256^3 batch workload: k mocks spread over the 64-mock size ladder
    N_i = round(0.2e6 10^(i/63)) galaxies (10x randoms), each with its own
    GRF, device-resident in float32, through lpp_estimate_batch (one captured
    graph, replayed) and, for comparison, through lpp_estimate one by one."""
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
    torch.cuda.synchronize()
    ngal = sum(ladder[i] for i in pick)
    log(f"batch: {len(pick)} mocks generated in {time.perf_counter() - t0:.1f} s ({ngal} galaxies)")
    plan = plan_for(lpp, wl, "f32")
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
    log(f"batch: {len(pick)} mocks in {1e3 * dt:.1f} ms per batch (graph), {1e3 * de:.1f} ms one by one")
    return {"workload": f"{len(pick)} mocks of the 256^3 wedge batch (mock indices {pick[0]}..{pick[-1]} of the "
                        f"0.2M-2M galaxy ladder, 10x randoms)", "mocks": len(pick), "galaxies": ngal,
            "mocks_per_s": round(len(pick) / dt, 3), "ms_per_batch": round(1e3 * dt, 2),
            "eager_mocks_per_s": round(len(pick) / de, 3), "graph_captures": caps, "graph_launches": launches}


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
    log(f"emulator: plain {1e3 * t_plain2k:.2f} ms / 2000 pts, emulator {1e3 * t_emu:.3f} ms, "
        f"max held-out err {rel.max():.4f}, separable {1e3 * t_sep:.3f} ms (err {sep_rel.max():.1e})")
    return out


def cpu_baseline(wl, gal, ran):
    """The FP64 oracle timed on a bounded sample of the same workload.

    Sample: one interlaced copy of the oracle's unit of work at the full mesh,
    i.e. (a) the FP64 deposit of the density set (galaxies and randoms), (b)
    one numpy 3D FFT of the mesh and (c) the complex deposit of the shape
    set.  The oracle's FFT route does 2 copies x (23 density-set + 59
    shape-set) such transforms per estimate (its Cartesian-tensor count at
    l <= 4: 1 + 22 density, 1 + 22 + 21 + 15 shape), so
    t_estimate = 2 (23 (a + b) + 59 (c + b)); shell sums are not included,
    which makes the baseline an upper bound on the oracle's rate."""
    import numpy as np
    from oracle import mesh as M
    n, box, origin, p = wl["mesh"], wl["box"], wl["origin"], wl["assignment"]
    gpos, rpos = gal.pos(), ran.pos()
    allpos = np.concatenate([gpos, rpos])
    alpha = gal.w.sum() / ran.w.sum()
    w = np.concatenate([gal.w, -alpha * ran.w])
    t0 = time.perf_counter()
    D = M.deposit(allpos, w, n, box, origin, p)
    ta = time.perf_counter() - t0
    log(f"cpu baseline: density deposit {ta:.1f} s")
    t0 = time.perf_counter()
    F = np.fft.fftn(D)
    tb = time.perf_counter() - t0
    del D, F
    log(f"cpu baseline: fft {tb:.1f} s")
    t0 = time.perf_counter()
    G = M.deposit(gpos, gal.w * (gal.g1 + 1j * gal.g2), n, box, origin, p)
    tc = time.perf_counter() - t0
    del G
    log(f"cpu baseline: shape deposit {tc:.1f} s")
    t_est = 2 * (23 * (ta + tb) + 59 * (tc + tb))
    return {"value": 1.0 / t_est, "unit": "estimates/s", "cores": 1, "kind": "oracle",
            "sample": (f"one interlaced copy at {n}^3: FP64 deposit of {gal.n + ran.n} density objects "
                       f"({ta:.1f} s), one numpy FFT ({tb:.1f} s), complex deposit of {gal.n} shape objects "
                       f"({tc:.1f} s); scaled to 2 x (23 density + 59 shape) transforms per estimate; "
                       "numpy FFT and bincount are single-threaded"),
            "seconds_sampled": ta + tb + tc}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--batch-mocks", type=int, default=8,
                    help="mocks of the 256^3 batch workload (spread over its 64-mock size ladder) "
                         "timed through the graph-captured batch path; 0 skips it")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--emulator", type=int, default=1,
                    help="1: window multipoles of the 512^3 randoms, the plain template path over the 22,000-point "
                         "design and the emulator trained on 20,000 of them (accuracy on the other 2,000, speedup)")
    ap.add_argument("--emu-epochs", type=int, default=1500)
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
    nd_mesh, ns_mesh = launches_per_set(res)
    yd, zd = strided_pass_bytes(np.concatenate([gal.pos(), ran.pos()]), wl)
    ys, zs = strided_pass_bytes(gal.pos(), wl)
    n_strided = 2 * (nd_mesh + ns_mesh)
    assert launches == n_strided * psteps, (launches, n_strided)
    alg_bytes = (nd_mesh * (yd + zd) + ns_mesh * (ys + zs)) / n_strided  # per launch
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = committed_traffic(strided_kernel_name(n, plan.tuning(), names_only=True))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "kernel": strided_kernel_name(n, plan.tuning()),
            "alg_bytes_per_launch": round(alg_bytes), "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "stage_ms_per_step": {k: round(v[0] / psteps, 3) for k, v in prof.items()},
            "stages_serial_ms_per_step": round(sum(v[0] for v in prof.values()) / psteps, 2)}

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

    if args.batch_mocks > 0:
        extra["batch_c3"] = batch_c3(lpp, torch, args.batch_mocks, args.batch_reps)
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
