"""Mass assignment, interlacing, compensation and k-shell bins (oracle side).

The paper works with fields on a grid (Sec. IV.A) and does not fix the mass
assignment; the reading used here (and stated in the design notes) is:

* mesh node c = (cx, cy, cz) sits at origin + c*H, H = box/N, indices wrap
  periodically; u = (x - origin)/H is the position in cell units;
* NGP (p=1): node round-half-up(u); CIC (p=2): floor(u) and floor(u)+1 with
  weights 1-f, f; TSC (p=3): c = floor(u + 1/2), d = u - c, weights
  (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2 at c-1, c, c+1;
* interlacing: a second deposit on the grid shifted by +H/2 on every axis
  (nodes at origin + (c + 1/2)H, i.e. u -> u - 1/2); its transform carries
  the phase exp(-i k.s), s = (H/2)(1,1,1), and the two are averaged;
* compensation: divide by W_p(k) = prod_i sinc(pi n_i / N)^p.

k-shell bins (a definition written out in integers): bin b collects the
modes n != 0 with T_b <= |n|^2 < T_{b+1}, T_b = ceil((b * dn)^2) with the
bin width dn = num/den in units of the fundamental frequency kf = 2 pi / box.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as _sfft


def stencil_1d(u: np.ndarray, p: int):
    """Per-axis node indices (unwrapped) and weights, shapes (n, p)."""
    if p == 1:
        c = np.floor(u + 0.5).astype(np.int64)
        return c[:, None], np.ones((u.shape[0], 1))
    if p == 2:
        c = np.floor(u).astype(np.int64)
        f = u - c
        return np.stack([c, c + 1], axis=1), np.stack([1.0 - f, f], axis=1)
    if p == 3:
        c = np.floor(u + 0.5).astype(np.int64)
        d = u - c
        return (np.stack([c - 1, c, c + 1], axis=1),
                np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=1))
    raise ValueError("assignment order must be 1, 2 or 3")


def deposit(pos: np.ndarray, values: np.ndarray, n: int, box: float, origin, p: int,
            shift: float = 0.0) -> np.ndarray:
    """FP64 deposit of per-object ``values`` (real or complex) onto an n^3 mesh
    indexed [ix, iy, iz]; ``shift`` = 0.5 gives the interlaced grid."""
    h = box / n
    u = (pos - np.asarray(origin, dtype=np.float64)[None, :]) / h - shift
    ci, wi = [], []
    for a in range(3):
        c, w = stencil_1d(u[:, a], p)
        ci.append(np.mod(c, n))
        wi.append(w)
    cplx = np.iscomplexobj(values)
    # every (object, stencil node) pair, then one sum per node
    flats, vals = [], []
    for a in range(p):
        for b in range(p):
            for c in range(p):
                flats.append((ci[0][:, a] * n + ci[1][:, b]) * n + ci[2][:, c])
                vals.append(wi[0][:, a] * wi[1][:, b] * wi[2][:, c] * values)
    flat = np.concatenate(flats)
    v = np.concatenate(vals)
    del flats, vals
    out = np.bincount(flat, weights=v.real if cplx else v, minlength=n ** 3)
    if cplx:
        out = out + 1j * np.bincount(flat, weights=v.imag, minlength=n ** 3)
    return out.reshape(n, n, n)


def workers() -> int:
    """Host threads for the FFTs: OMP_NUM_THREADS if set (the share of the
    host this process may use), else every core."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, int(v)) if v.isdigit() else (os.cpu_count() or 1)


def fftn(a: np.ndarray) -> np.ndarray:
    """Forward 3D DFT, exp(-2 pi i n.c/N) (scipy's FFT on workers() threads)."""
    return _sfft.fftn(a, workers=workers())


def ifftn(a: np.ndarray) -> np.ndarray:
    """Inverse 3D DFT with the 1/N^3 factor (scipy's FFT on workers() threads)."""
    return _sfft.ifftn(a, workers=workers())


def signed_modes(n: int) -> np.ndarray:
    return np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)


def compensation(n: int, p: int) -> np.ndarray:
    """W_p(k) on the full mesh, shape (n, n, n)."""
    s = np.sinc(signed_modes(n) / n)  # numpy sinc(x) = sin(pi x)/(pi x)
    w1 = s ** p
    return w1[:, None, None] * w1[None, :, None] * w1[None, None, :]


def interlace_phase(n: int) -> np.ndarray:
    """exp(-i k.s) with s = (H/2)(1,1,1): exp(-i pi (nx+ny+nz)/n)."""
    m = signed_modes(n)
    t = m[:, None, None] + m[None, :, None] + m[None, None, :]
    return np.exp(-1j * np.pi * t / n)


def default_dn(n: int, n_kbins: int):
    """Bin width N/(2 n_kbins) in units of kf, as a reduced fraction (num, den)."""
    num, den = n, 2 * n_kbins
    g = math.gcd(num, den)
    return num // g, den // g


def thresholds(n_kbins: int, num: int, den: int):
    """Integer thresholds T_b = ceil((b num/den)^2), b = 0..n_kbins (Python ints)."""
    return [-((-(b * b * num * num)) // (den * den)) for b in range(n_kbins + 1)]


def bin_index(n: int, n_kbins: int, num: int, den: int) -> np.ndarray:
    """Bin of every mode of the full mesh (-1 = not binned: DC or beyond the last edge)."""
    m = signed_modes(n)
    q = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    T = np.asarray(thresholds(n_kbins, num, den), dtype=np.int64)
    b = np.searchsorted(T, q, side="right") - 1
    b[(q >= T[-1]) | (q == 0)] = -1
    return b


def mode_counts(n: int, n_kbins: int, num: int, den: int) -> np.ndarray:
    b = bin_index(n, n_kbins, num, den)
    return np.bincount(b[b >= 0].ravel(), minlength=n_kbins).astype(np.int64)
