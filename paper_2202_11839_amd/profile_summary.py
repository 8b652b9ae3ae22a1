"""Short text summaries of rocprofv3 output for the profiles/ folder.

``kernels DB [--title T] [--command C]``
    Per-kernel launch count, average and total duration from a
    ``--kernel-trace`` SQLite database (rocprofv3's ``*_results.db``).

``traffic FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB [--kernel REGEX | --estimates K]``
    HBM bytes per launch of the kernels whose name matches REGEX, from a
    ``--pmc FETCH_SIZE`` and a ``--pmc WRITE_SIZE`` run of the same program.
    Both counters are scaled by what they read for a plain device copy of
    known size (``bench.py --copy-calibration``: 1 GiB read and 1 GiB written
    per ``__amd_rocclr_copyBuffer`` launch), and the SHA-256 of the kernel
    source and of the host code that sequences its launches is recorded, so
    that a stale figure can be recognised.  With --estimates K: the bytes of
    every library kernel launched by a run of K estimates, per estimate (the
    record keeps the SHA-256 of every library source).  Without either: a
    table of read and written bytes per launch of every kernel.

``sq DB [DB ...] --kernel REGEX``
    Per launch of the kernels whose name matches REGEX, every counter of the
    ``--pmc`` runs given: the SQ counters summed over the shader engines that
    report them, the GRBM counters averaged over the XCDs (each reports the
    whole GPU's clock), then the mean over launches; and, where the counters
    are there, the VALU issue fraction (wave64 VALU instructions x 4 cycles
    over the SIMDs' cycles), the active lanes per VALU instruction and the
    mean resident waves per CU (SQ_WAVE_CYCLES counts in units of 4 cycles).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
import statistics

CUS, SIMDS = 256, 1024
COPY_BYTES = 1 << 30  # bytes read and bytes written by one calibration copy
HERE = os.path.dirname(os.path.abspath(__file__))
# a traffic record holds for these sources only: the strided-pass kernel and
# the host code that decides which passes run
TRAFFIC_SOURCES = ["csrc/kernels_fft.hip", "csrc/api.hip"]


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    name = name.replace("lpp::dev::V2<float>::type", "float2").replace("lpp::dev::V2<double>::type", "double2")
    return re.sub(r"\(.*", "", name).strip()


def kernel_table(db: str) -> list[tuple[str, int, float, float]]:
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(end - start), sum(end - start) from kernels group by name").fetchall()
    out = [(_short(n), c, a / 1e6, s / 1e6) for n, c, a, s in rows]
    return sorted(out, key=lambda r: -r[3])


def fft_pass_split(db: str) -> list[tuple[str, int, float, float]]:
    """Durations of the z-blocked FFT kernel by pass.  A transform launches
    the x pass (the along-x instantiation) and then the y and z passes, so in
    launch order the two launches after an x pass are its y and z passes."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    by = {"x": [], "y": [], "z": []}
    last = None
    for name, t0, t1 in rows:
        name = _short(name)
        if "fft_zb_kernel<" not in name:
            continue
        args = name[name.index("<") + 1:name.rindex(">")].split(", ")
        d = (t1 - t0) / 1e6
        if args[3] == "true":
            last = "x"
        elif last in ("x", "y"):
            last = "y" if last == "x" else "z"
        else:
            continue
        by[last].append(d)
    return [(p, len(v), statistics.mean(v), statistics.median(v)) for p, v in by.items() if v]


def counter(db: str, name: str) -> dict[str, list[float]]:
    con = sqlite3.connect(db)
    per: dict[str, list[float]] = {}
    for kname, value in con.execute("select name, counter_value from pmc_events where counter_name = ?", (name,)):
        per.setdefault(kname, []).append(float(value))
    return per


def scale(db: str, name: str) -> float:
    """Bytes per counter unit, from the calibration copies (first copy skipped)."""
    vals = [v for k, vs in counter(db, name).items() if "copyBuffer" in k for v in vs]
    if not vals:
        raise SystemExit(f"no copy kernel in {db}")
    vals = vals[1:] if len(vals) > 1 else vals
    return COPY_BYTES / statistics.mean(vals)


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--title", default="")
    k.add_argument("--command", default="")
    k.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("copy_fetch_db")
    t.add_argument("copy_write_db")
    t.add_argument("--kernel", default="")
    t.add_argument("--source", action="append", default=None,
                   help="source files whose SHA-256 the record keeps (default: the FFT kernels and the "
                        "host code that sets their launch sequence)")
    t.add_argument("--command", default="")
    t.add_argument("--estimates", type=int, default=0)
    q = sub.add_parser("sq")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--kernel", required=True)
    q.add_argument("--command", default="")
    args = ap.parse_args()

    if args.mode == "sq":
        pat = re.compile(args.kernel)
        if args.command:
            print(f"# command: {args.command}")
        per: dict[str, dict[str, list[float]]] = {}
        for db in args.dbs:
            con = sqlite3.connect(db)
            inst: dict[tuple, list[float]] = {}
            for kname, disp, cname, value in con.execute(
                    "select name, dispatch_id, counter_name, counter_value from pmc_events"):
                k = _short(kname)
                if pat.search(k):
                    inst.setdefault((k, disp, cname), []).append(float(value))
            for (k, _, cname), vs in inst.items():
                v = statistics.mean(vs) if cname.startswith("GRBM_") else sum(vs)
                per.setdefault(k, {}).setdefault(cname, []).append(v)
        print(f"# MI355X: {SIMDS} SIMDs in {CUS} CUs; a wave64 VALU instruction occupies its SIMD for 4 cycles")
        for k in sorted(per):
            m = {c: statistics.mean(vs) for c, vs in per[k].items()}
            print(f"## {k}")
            for c in sorted(m):
                print(f"{c:32s} {m[c]:18.1f}   ({len(per[k][c])} launches)")
            clk = m.get("GRBM_GUI_ACTIVE")
            if clk and "SQ_INSTS_VALU" in m:
                print(f"{'= VALU issue fraction':32s} {4 * m['SQ_INSTS_VALU'] / (SIMDS * clk):18.3f}")
            if m.get("SQ_INSTS_VALU") and "SQ_THREAD_CYCLES_VALU" in m:
                print(f"{'= active lanes per VALU instr.':32s} {m['SQ_THREAD_CYCLES_VALU'] / m['SQ_INSTS_VALU']:18.1f}")
            if clk and "SQ_WAVE_CYCLES" in m:
                print(f"{'= resident waves per CU':32s} {4 * m['SQ_WAVE_CYCLES'] / (CUS * clk):18.2f}")
            if clk:
                print(f"{'= duration at 2.4 GHz (ms)':32s} {clk / 2.4e6:18.4f}")
        return

    if args.mode == "kernels":
        rows = kernel_table(args.db)
        if args.title:
            print(f"# {args.title}")
        if args.command:
            print(f"# command: {args.command}")
        total = sum(r[3] for r in rows)
        print(f"{'kernel':70s} {'calls':>6s} {'avg ms':>9s} {'total ms':>10s} {'share':>6s}")
        for name, calls, avg, tot in rows[: args.top]:
            print(f"{name[:70]:70s} {calls:6d} {avg:9.4f} {tot:10.2f} {100 * tot / total:5.1f}%")
        print(f"{'all kernels':70s} {sum(r[1] for r in rows):6d} {'':9s} {total:10.2f}")
        split = fft_pass_split(args.db)
        if split:
            print("# fft_zb_kernel launches split by pass (launch order x, y, z per transform): "
                  "pass, launches, mean ms, median ms")
            for p, n, mean, med in split:
                print(f"#   {p} {n} {mean:.4f} {med:.4f}")
        return

    fs, ws = scale(args.copy_fetch_db, "FETCH_SIZE"), scale(args.copy_write_db, "WRITE_SIZE")
    if args.estimates > 0:
        rd = sum(v for n, vs in counter(args.fetch_db, "FETCH_SIZE").items() if n.startswith("lpp::") or
                 "lpp::" in n for v in vs) * fs / args.estimates
        wr = sum(v for n, vs in counter(args.write_db, "WRITE_SIZE").items() if n.startswith("lpp::") or
                 "lpp::" in n for v in vs) * ws / args.estimates
        digests = {}
        for name in sorted(os.listdir(os.path.join(HERE, "csrc"))):
            with open(os.path.join(HERE, "csrc", name), "rb") as f:
                digests[name] = hashlib.sha256(f.read()).hexdigest()
        rec = {"estimates": args.estimates, "read_bytes_per_estimate": round(rd), "write_bytes_per_estimate": round(wr),
               "bytes_per_estimate": round(rd) + round(wr), "fetch_scale_bytes_per_unit": fs,
               "write_scale_bytes_per_unit": ws, "sources_sha256": digests, "command": args.command}
        print(json.dumps(rec, indent=1))
        return
    if not args.kernel:
        fetch_all, write_all = counter(args.fetch_db, "FETCH_SIZE"), counter(args.write_db, "WRITE_SIZE")
        dur = {}
        con = sqlite3.connect(args.fetch_db)
        for kname, d in con.execute("select name, duration from pmc_events where counter_name = 'FETCH_SIZE'"):
            dur.setdefault(kname, []).append(d / 1e6)
        if args.command:
            print(f"# command: {args.command}")
        print(f"# counters scaled by the calibration copy: FETCH_SIZE x {fs:.1f} B, WRITE_SIZE x {ws:.1f} B")
        print(f"{'kernel':60s} {'calls':>6s} {'read GB':>9s} {'write GB':>9s} {'ms (pmc run)':>13s}")
        rows = []
        for kname, vals in fetch_all.items():
            wv = write_all.get(kname, [0.0])
            rows.append((_short(kname), len(vals), statistics.mean(vals) * fs / 1e9, statistics.mean(wv) * ws / 1e9,
                         statistics.mean(dur.get(kname, [0.0]))))
        for r in sorted(rows, key=lambda r: -r[1] * r[4])[:25]:
            print(f"{r[0][:60]:60s} {r[1]:6d} {r[2]:9.3f} {r[3]:9.3f} {r[4]:13.4f}")
        return
    pat = re.compile(args.kernel)
    fetch = [v for n, vs in counter(args.fetch_db, "FETCH_SIZE").items() if pat.search(_short(n)) for v in vs]
    write = [v for n, vs in counter(args.write_db, "WRITE_SIZE").items() if pat.search(_short(n)) for v in vs]
    if not fetch or not write:
        raise SystemExit(f"no launches of {args.kernel!r}")
    sources = args.source or TRAFFIC_SOURCES
    digests = {}
    for src in sources:
        with open(os.path.join(HERE, src) if not os.path.isabs(src) else src, "rb") as f:
            digests[os.path.basename(src)] = hashlib.sha256(f.read()).hexdigest()
    rd, wr = statistics.mean(fetch) * fs, statistics.mean(write) * ws
    rec = {"kernel": args.kernel, "launches": len(fetch), "read_bytes_per_launch": round(rd),
           "write_bytes_per_launch": round(wr), "bytes_per_launch": round(rd) + round(wr),
           "fetch_scale_bytes_per_unit": fs, "write_scale_bytes_per_unit": ws,
           "sources_sha256": digests, "command": args.command}
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
