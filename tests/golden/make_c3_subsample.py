"""Write tests/golden/c3_subsample_256.json: the FP64 oracle (oracle.estimator.mesh64,
the FFT route with the paper's Cartesian tensors) on a subsample of one mock
of the 256^3 batch workload, for the batch path's parity test.

The catalog is made by synth.make_catalogs from the 256^3 batch recipe (box
1700 Mpc/h at origin -50, observer at 0, wedge RA 0-90, Dec 0-40, r
1000-1600) with 30,000 galaxies and 300,000 randoms (mock 5, its own GRF on
the 256^3 mesh); the estimate uses the workload's own settings (256^3 mesh,
TSC with interlacing, compensation, l <= 4, 50 shells).  The file also stores
checksums of the catalog, so that the test can tell a changed generator from
a changed estimator.  Only oracle/ and synth/ are called.

Usage:  python tests/golden/make_c3_subsample.py      (a few minutes, 5 GB)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import estimator as E  # noqa: E402
from synth import WORKLOADS, make_catalogs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_subsample_256.json")
RECIPE = dict(workload="c3", mock=5, n_gal=30_000, n_ran=300_000, grf_mesh=256)


def catalogs():
    wl = WORKLOADS[RECIPE["workload"]]
    return make_catalogs(wl, mock=RECIPE["mock"], n_gal=RECIPE["n_gal"], n_ran=RECIPE["n_ran"],
                         grf_mesh=RECIPE["grf_mesh"])


def checksums(g, r):
    return {"n_gal": g.n, "n_ran": r.n, "sum_gx": float(np.sum(g.x)), "sum_gz": float(np.sum(g.z)),
            "sum_g1": float(np.sum(g.g1)), "sum_g2": float(np.sum(g.g2)), "sum_rx": float(np.sum(r.x)),
            "sum_ry": float(np.sum(r.y))}


def config(families):
    wl = WORKLOADS[RECIPE["workload"]]
    return E.Config(mesh=wl["mesh"], box=wl["box"], origin=wl["origin"], observer=wl["observer"],
                    assignment=wl["assignment"], interlacing=wl["interlacing"], compensate=1, lmax=wl["lmax"],
                    n_kbins=wl["n_kbins"], families=families)


def main():
    t0 = time.time()
    g, r = catalogs()
    print(f"catalogs: {g.n} galaxies, {r.n} randoms ({time.time() - t0:.0f} s)", flush=True)
    rows = {}
    res = None
    for fams in (("DD",), ("GD",), ("PLUS", "MINUS")):
        t1 = time.time()
        res = E.mesh64(g, r, config(fams))
        for i, s in enumerate(res["series"]):
            rows[s] = (res["re"][i].tolist(), res["im"][i].tolist())
        print(f"{'+'.join(fams)}: {time.time() - t1:.0f} s", flush=True)
    names = E.series_names(WORKLOADS["c3"]["lmax"])
    out = dict(
        source="oracle.estimator.mesh64 (FP64, numpy/scipy), written by tests/golden/make_c3_subsample.py",
        recipe=RECIPE, checksums=checksums(g, r), series=names,
        n_modes=[int(v) for v in res["n_modes"]], k_eff=res["k_eff"].tolist(), k_lo=res["k_lo"].tolist(),
        re=[rows[s][0] for s in names], im=[rows[s][1] for s in names],
        **{k: float(res[k]) for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran")})
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
