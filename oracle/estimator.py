"""FP64 LPP estimators of the projected-tensor power-spectrum multipoles.

Three independent routes to the same quantities:

``brute``   the defining sums written out (tiny inputs only): for every mesh
            mode k and every object, the line-of-sight kernel of the paper's
            estimators evaluated with the phase factor of eq.
            def_of_phase_factor and the associated Legendre polynomial of eq.
            def_of_asso (Sec. III.A, eqs. lpp_dens_app, lpp_estimator_cross,
            app_lpp_est_auto_plus, app_lpp_est_auto_minus), times the
            mesh-consistent plane wave of the object (the transform of its
            mass-assignment stencil, averaged over the interlaced grids and
            divided by the assignment window).

``mesh64``  the FFT route of Sec. III.A: FP64 deposit + numpy FFT of the
            Cartesian-tensor fields.  Each kernel (k.m)^s R^s_L(k.xhat), with
            2 e*_ij k_i k_j = (k.m)^2, m = e_theta - i e_phi, is expanded into
            monomials of the components of khat; every monomial coefficient
            (a product of Cartesian components of xhat and m) is deposited and
            transformed, and the transforms are contracted with the same
            monomials of khat on the mesh (eqs. def_of_Xiij, def_of_Xiijkl,
            delta_ell).

``gpp``     the global-plane-parallel estimators of Sec. II.C with a single
            line of sight n (E/B rotation Gamma = gamma exp(-2 i phi_{k,n}),
            eq. def_of_phase_factor), used for the distant-observer limit.

Output convention (all routes): ``re``/``im`` arrays [series, bin] with

  DD_l     (2l+1)/(I N_b) sum_k delta^(l)(k) delta(-k)          - N_dd [l=0]
  GD_L     c2_L /(I N_b) sum_k Xi^(L)_ij khat_i khat_j delta(-k)
  PLUS_l   (2l+1)/(I N_b) sum_k gamma^(l)(k) gamma*(-k)          - N_+  [l=0]
  MINUS_L  c4_L /(I N_b) sum_k Xi^(L)_ijkl khat^4 gamma(-k)
  EE_l, BB_l = (PLUS_l +- sum_L C_{lL} Re MINUS_L)/2

with c_L^m = (2L+1)(L-m)!/(L+m)!, alpha = sum w_g / sum w_r,
I = alpha sum_r w_r^2 nbar_r, N_dd = (sum w_g^2 + alpha^2 sum w_r^2)/I,
N_+ = sum w_g^2 |gamma|^2 / I.  Real parts are the spectra; imaginary parts
are the parity-odd diagnostics (which vanish by parity, Sec. II.C).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import geometry, mesh, special

FAMILIES = ("DD", "GD", "PLUS", "MINUS")


@dataclass
class Config:
    mesh: int
    box: float
    origin: tuple
    observer: tuple = (0.0, 0.0, 0.0)
    assignment: int = 3
    interlacing: int = 1
    compensate: int = 1
    lmax: int = 4
    n_kbins: int = 16
    dn: Optional[tuple] = None          # (num, den) bin width in units of kf
    families: tuple = FAMILIES

    def bin_width(self):
        return self.dn if self.dn is not None else mesh.default_dn(self.mesh, self.n_kbins)


def series_names(lmax: int, families=FAMILIES) -> List[str]:
    out = []
    if "DD" in families:
        out += [f"DD_l{l}" for l in range(0, lmax + 1, 2)]
    if "GD" in families:
        out += [f"GD_L{L}" for L in range(2, lmax + 1, 2)]
    if "PLUS" in families:
        out += [f"PLUS_l{l}" for l in range(0, lmax + 1, 2)]
    if "MINUS" in families:
        out += [f"MINUS_L{L}" for L in range(4, lmax + 1, 2)]
    if "PLUS" in families and "MINUS" in families and lmax >= 4:
        out += [f"EE_l{l}" for l in range(0, lmax + 1, 2)]
        out += [f"BB_l{l}" for l in range(0, lmax + 1, 2)]
    return out


def scalars(gal, ran) -> Dict[str, float]:
    """alpha, I, N_dd, N_+ in FP64 (normalisation and shot noise)."""
    swg = float(np.sum(gal.w))
    swr = float(np.sum(ran.w))
    if swr == 0.0:
        raise ValueError("random catalog has zero total weight")
    alpha = swg / swr
    norm = alpha * float(np.sum(ran.w ** 2 * ran.nbar))
    gam2 = gal.g1 ** 2 + gal.g2 ** 2
    return dict(alpha=alpha, norm_I=norm,
                shot_dd=(float(np.sum(gal.w ** 2)) + alpha ** 2 * float(np.sum(ran.w ** 2))) / norm,
                shot_plus=float(np.sum(gal.w ** 2 * gam2)) / norm,
                sum_w_gal=swg, sum_w_ran=swr)


def _khat(n: int):
    m = mesh.signed_modes(n).astype(np.float64)
    kx, ky, kz = np.meshgrid(m, m, m, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    inv = np.where(kk > 0, 1.0 / np.where(kk > 0, kk, 1.0), 0.0)
    return kx * inv, ky * inv, kz * inv, kk


def _flip(F: np.ndarray) -> np.ndarray:
    """F(-k): index -n mod N on every axis."""
    return np.roll(np.flip(F, axis=(0, 1, 2)), 1, axis=(0, 1, 2))


def _finish(cfg: Config, acc: Dict[str, np.ndarray], sc: Dict[str, float], counts, ksum):
    """Bin sums -> multipoles (prefactors, normalisation, shot noise, E/B)."""
    names = series_names(cfg.lmax, cfg.families)
    nb = cfg.n_kbins
    safe = np.where(counts > 0, counts, 1).astype(np.float64)
    re = np.zeros((len(names), nb))
    im = np.zeros((len(names), nb))
    for i, s in enumerate(names):
        if s.startswith("EE") or s.startswith("BB"):
            continue
        fam, lab = s.split("_")
        L = int(lab[1:])
        m = {"DD": 0, "PLUS": 0, "GD": 2, "MINUS": 4}[fam]
        pref = float(special.prefactor(m, L))
        z = acc[s] * pref / (sc["norm_I"] * safe)
        re[i] = z.real
        im[i] = z.imag
        if s == "DD_l0":
            re[i] -= sc["shot_dd"]
        if s == "PLUS_l0":
            re[i] -= sc["shot_plus"]
    if "EE_l0" in names:
        for l in range(0, cfg.lmax + 1, 2):
            ip = names.index(f"PLUS_l{l}")
            mix = np.zeros(nb)
            for L in range(4, cfg.lmax + 1, 2):
                mix += float(special.cmap_minus_to_legendre(l, L)) * re[names.index(f"MINUS_L{L}")]
            re[names.index(f"EE_l{l}")] = 0.5 * (re[ip] + mix)
            re[names.index(f"BB_l{l}")] = 0.5 * (re[ip] - mix)
    num, den = cfg.bin_width()
    kf = 2.0 * math.pi / cfg.box
    edges = np.arange(nb + 1) * (num / den) * kf
    res = dict(series=names, re=re, im=im, n_modes=counts.astype(np.int64),
               k_eff=np.where(counts > 0, ksum * kf / safe, 0.0), k_lo=edges[:-1], k_hi=edges[1:])
    res.update(sc)
    return res


def _bin_sums(cfg: Config, bidx: np.ndarray, z: np.ndarray) -> np.ndarray:
    sel = bidx >= 0
    b = bidx[sel]
    v = z[sel]
    return (np.bincount(b, weights=v.real, minlength=cfg.n_kbins)
            + 1j * np.bincount(b, weights=v.imag, minlength=cfg.n_kbins))


# ---------------------------------------------------------------------------
# mesh64: the FFT route with Cartesian tensors

def _transform(cfg: Config, pos: np.ndarray, values: np.ndarray, comp: np.ndarray,
               phase: Optional[np.ndarray]) -> np.ndarray:
    n, p = cfg.mesh, cfg.assignment
    F = mesh.fftn(mesh.deposit(pos, values, n, cfg.box, cfg.origin, p))
    if cfg.interlacing:
        F2 = mesh.fftn(mesh.deposit(pos, values, n, cfg.box, cfg.origin, p, shift=0.5))
        F = 0.5 * (F + phase * F2)
    return F / comp


def _mul_linear(poly: dict, v: np.ndarray) -> dict:
    """Multiply a polynomial in khat (dict multi-index -> per-object coefficient)
    by the linear form khat . v (v has shape (n_obj, 3))."""
    out = {}
    for a, c in poly.items():
        for i in range(3):
            b = list(a)
            b[i] += 1
            b = tuple(b)
            out[b] = out.get(b, 0) + c * v[:, i]
    return out


def _kernel_transform(cfg, pos, weight, xh, mvec, s, j, kh, comp, phase):
    """sum_alpha khat^alpha FT[weight * coef_alpha((khat.m)^s (khat.xhat)^j)](k)."""
    poly = {(0, 0, 0): np.ones(pos.shape[0])}
    for _ in range(s):
        poly = _mul_linear(poly, mvec)
    for _ in range(j):
        poly = _mul_linear(poly, xh)
    out = np.zeros((cfg.mesh,) * 3, dtype=np.complex128)
    for a, c in poly.items():
        mono = kh[0] ** a[0] * kh[1] ** a[1] * kh[2] ** a[2]
        out += mono * _transform(cfg, pos, weight * c, comp, phase)
    return out


def _assemble_family(cfg, pos, weight, xh, mvec, s, Ls, kh, comp, phase):
    """{L: sum_j r^s_{Lj} T_j(k)} with R^s_L(mu) = sum_j r^s_{Lj} mu^j."""
    need = {}
    for L in Ls:
        for j, c in enumerate(special.reduced_assoc(s, L)):
            if c != 0:
                need.setdefault(j, []).append((L, float(c)))
    out = {L: np.zeros((cfg.mesh,) * 3, dtype=np.complex128) for L in Ls}
    for j in sorted(need):
        T = _kernel_transform(cfg, pos, weight, xh, mvec, s, j, kh, comp, phase)
        for L, c in need[j]:
            out[L] += c * T
    return out


def mesh64(gal, ran, cfg: Config) -> dict:
    """The FFT-based LPP estimator in FP64 with the Cartesian decomposition."""
    n = cfg.mesh
    sc = scalars(gal, ran)
    kx, ky, kz, kk = _khat(n)
    kh = (kx, ky, kz)
    comp = mesh.compensation(n, cfg.assignment) if cfg.compensate else np.ones((n,) * 3)
    phase = mesh.interlace_phase(n) if cfg.interlacing else None
    num, den = cfg.bin_width()
    bidx = mesh.bin_index(n, cfg.n_kbins, num, den)
    counts = np.bincount(bidx[bidx >= 0], minlength=cfg.n_kbins)
    ksum = np.bincount(bidx[bidx >= 0], weights=kk[bidx >= 0], minlength=cfg.n_kbins)

    gpos, rpos = gal.pos(), ran.pos()
    gxh, get, gep = geometry.basis(gpos, cfg.observer)
    gm = get - 1j * gep
    gam = gal.g1 + 1j * gal.g2
    allpos = np.concatenate([gpos, rpos])
    allxh = np.concatenate([gxh, geometry.los(rpos, cfg.observer)])
    dw = np.concatenate([gal.w, -sc["alpha"] * ran.w])
    gw = gal.w * gam
    acc = {}
    fam = cfg.families
    ells = list(range(0, cfg.lmax + 1, 2))
    Fd = Fg = None
    if "DD" in fam or "GD" in fam:
        Fd = _transform(cfg, allpos, dw, comp, phase)
    if "PLUS" in fam or "MINUS" in fam:
        Fg = _transform(cfg, gpos, gw, comp, phase)
    if "DD" in fam:
        dl = _assemble_family(cfg, allpos, dw, allxh, None, 0, ells, kh, comp, phase)
        Fdm = _flip(Fd)
        for l in ells:
            acc[f"DD_l{l}"] = _bin_sums(cfg, bidx, dl[l] * Fdm)
    if "GD" in fam:
        Ls = list(range(2, cfg.lmax + 1, 2))
        X = _assemble_family(cfg, gpos, gw, gxh, gm, 2, Ls, kh, comp, phase)
        Fdm = _flip(Fd)
        for L in Ls:
            acc[f"GD_L{L}"] = _bin_sums(cfg, bidx, X[L] * Fdm)
    if "PLUS" in fam:
        gl = _assemble_family(cfg, gpos, gw, gxh, None, 0, ells, kh, comp, phase)
        Fgc = np.conj(Fg)  # gamma*(-k) = conj(gamma(k))
        for l in ells:
            acc[f"PLUS_l{l}"] = _bin_sums(cfg, bidx, gl[l] * Fgc)
    if "MINUS" in fam and cfg.lmax >= 4:
        Ls = list(range(4, cfg.lmax + 1, 2))
        Y = _assemble_family(cfg, gpos, gw, gxh, gm, 4, Ls, kh, comp, phase)
        Fgm = _flip(Fg)
        for L in Ls:
            acc[f"MINUS_L{L}"] = _bin_sums(cfg, bidx, Y[L] * Fgm)
    return _finish(cfg, acc, sc, counts, ksum)


# ---------------------------------------------------------------------------
# brute: the defining sums (tiny inputs)

def _axis_phase(u: np.ndarray, n: int, p: int, shift: float) -> np.ndarray:
    """Per object and axis mode n_a: sum_c W(u - c) exp(-2 pi i n_a (c + shift)/N)
    with u already in grid units of the (possibly shifted) grid."""
    c, w = mesh.stencil_1d(u, p)
    modes = mesh.signed_modes(n).astype(np.float64)
    ph = np.exp(-2j * np.pi * (c[:, :, None] + shift) * modes[None, None, :] / n)
    return np.sum(w[:, :, None] * ph, axis=1)  # (n_obj, N)


def _object_planewaves(cfg: Config, pos: np.ndarray) -> np.ndarray:
    """Mesh-consistent exp(-i k.x_o) for all modes: shape (n_obj, N, N, N)."""
    n, p = cfg.mesh, cfg.assignment
    h = cfg.box / n
    u = (pos - np.asarray(cfg.origin, dtype=np.float64)[None, :]) / h
    a = [_axis_phase(u[:, i], n, p, 0.0) for i in range(3)]
    pw = a[0][:, :, None, None] * a[1][:, None, :, None] * a[2][:, None, None, :]
    if cfg.interlacing:
        b = [_axis_phase(u[:, i] - 0.5, n, p, 0.5) for i in range(3)]
        pw = 0.5 * (pw + b[0][:, :, None, None] * b[1][:, None, :, None] * b[2][:, None, None, :])
    if cfg.compensate:
        pw = pw / mesh.compensation(n, p)[None]
    return pw


def brute(gal, ran, cfg: Config) -> dict:
    """The estimators as defining double sums (modes x objects); tiny inputs."""
    n = cfg.mesh
    if n > 16:
        raise ValueError("brute() is for meshes of at most 16^3")
    sc = scalars(gal, ran)
    kx, ky, kz, kk = _khat(n)
    khat = np.stack([kx, ky, kz], axis=-1)  # (N,N,N,3)
    num, den = cfg.bin_width()
    bidx = mesh.bin_index(n, cfg.n_kbins, num, den)
    counts = np.bincount(bidx[bidx >= 0], minlength=cfg.n_kbins)
    ksum = np.bincount(bidx[bidx >= 0], weights=kk[bidx >= 0], minlength=cfg.n_kbins)

    gpos, rpos = gal.pos(), ran.pos()
    gxh, get, gep = geometry.basis(gpos, cfg.observer)
    rxh = geometry.los(rpos, cfg.observer)
    eij = geometry.e_tensor(get, gep)
    gam = gal.g1 + 1j * gal.g2
    pw_g = _object_planewaves(cfg, gpos)
    pw_r = _object_planewaves(cfg, rpos)
    alpha = sc["alpha"]

    mu_g = np.einsum("xyzi,oi->oxyz", khat, gxh)
    mu_r = np.einsum("xyzi,oi->oxyz", khat, rxh)
    # e^{2 i phi_{k,x}} (1 - mu^2) = 2 e_ij(xhat) khat_i khat_j   (eq. def_of_phase_factor)
    e2k = 2.0 * np.einsum("xyzi,oij,xyzj->oxyz", khat, eij, khat)
    one_m = 1.0 - mu_g ** 2
    ok = one_m > 1e-13
    emi2 = np.where(ok, np.conj(e2k) / np.where(ok, one_m, 1.0), 0.0)  # e^{-2 i phi}

    Fd = np.einsum("o,oxyz->xyz", gal.w, pw_g) - alpha * np.einsum("o,oxyz->xyz", ran.w, pw_r)
    Fg = np.einsum("o,oxyz->xyz", gal.w * gam, pw_g)
    ells = list(range(0, cfg.lmax + 1, 2))
    acc = {}
    fam = cfg.families
    if "DD" in fam:
        for l in ells:
            dl = (np.einsum("o,oxyz,oxyz->xyz", gal.w, special.peval(special.legendre(l), mu_g), pw_g)
                  - alpha * np.einsum("o,oxyz,oxyz->xyz", ran.w, special.peval(special.legendre(l), mu_r), pw_r))
            acc[f"DD_l{l}"] = _bin_sums(cfg, bidx, dl * _flip(Fd))
    if "GD" in fam:
        for L in range(2, cfg.lmax + 1, 2):
            ker = emi2 * special.assoc_legendre(2, L, mu_g)
            X = np.einsum("o,oxyz,oxyz->xyz", gal.w * gam, ker, pw_g)
            acc[f"GD_L{L}"] = _bin_sums(cfg, bidx, X * _flip(Fd))
    if "PLUS" in fam:
        for l in ells:
            gl = np.einsum("o,oxyz,oxyz->xyz", gal.w * gam, special.peval(special.legendre(l), mu_g), pw_g)
            acc[f"PLUS_l{l}"] = _bin_sums(cfg, bidx, gl * np.conj(Fg))
    if "MINUS" in fam:
        for L in range(4, cfg.lmax + 1, 2):
            ker = emi2 ** 2 * special.assoc_legendre(4, L, mu_g)
            Y = np.einsum("o,oxyz,oxyz->xyz", gal.w * gam, ker, pw_g)
            acc[f"MINUS_L{L}"] = _bin_sums(cfg, bidx, Y * _flip(Fg))
    return _finish(cfg, acc, sc, counts, ksum)


# ---------------------------------------------------------------------------
# gpp: one global line of sight

def gpp(gal, ran, cfg: Config, nhat) -> dict:
    """Global-plane-parallel multipoles with line of sight ``nhat`` (Sec. II.C).

    gamma(k) is the transform of the catalog's gamma (its components taken as
    given), Gamma = gamma exp(-2 i phi_{k,n}) with exp(2 i phi) =
    2 e_ij(n) k_i k_j / (1 - mu^2), mu = khat.n; the multipoles are the
    associated-Legendre (m=2, 4) and Legendre moments of Gamma delta*,
    Gamma Gamma* and Gamma(k) Gamma(-k)."""
    n = cfg.mesh
    sc = scalars(gal, ran)
    nhat = np.asarray(nhat, dtype=np.float64)
    nhat = nhat / np.linalg.norm(nhat)
    kx, ky, kz, kk = _khat(n)
    khat = np.stack([kx, ky, kz], axis=-1)
    comp = mesh.compensation(n, cfg.assignment) if cfg.compensate else np.ones((n,) * 3)
    phase = mesh.interlace_phase(n) if cfg.interlacing else None
    num, den = cfg.bin_width()
    bidx = mesh.bin_index(n, cfg.n_kbins, num, den)
    counts = np.bincount(bidx[bidx >= 0], minlength=cfg.n_kbins)
    ksum = np.bincount(bidx[bidx >= 0], weights=kk[bidx >= 0], minlength=cfg.n_kbins)
    gpos, rpos = gal.pos(), ran.pos()
    Fd = _transform(cfg, np.concatenate([gpos, rpos]),
                    np.concatenate([gal.w, -sc["alpha"] * ran.w]), comp, phase)
    Fg = _transform(cfg, gpos, gal.w * (gal.g1 + 1j * gal.g2), comp, phase)
    _, et, ep = geometry.basis(nhat[None, :] * 1.0, (0.0, 0.0, 0.0))
    e = geometry.e_tensor(et, ep)[0]
    mu = khat @ nhat
    e2 = 2.0 * np.einsum("xyzi,ij,xyzj->xyz", khat, e, khat)
    one_m = 1.0 - mu * mu
    ok = one_m > 1e-13
    emi2 = np.where(ok, np.conj(e2) / np.where(ok, one_m, 1.0), 0.0)
    G = Fg * emi2                       # Gamma(k)
    Gm = _flip(Fg) * _flip(emi2)        # Gamma(-k)
    ells = list(range(0, cfg.lmax + 1, 2))
    acc = {}
    for l in ells:
        acc[f"DD_l{l}"] = _bin_sums(cfg, bidx, special.peval(special.legendre(l), mu) * Fd * np.conj(Fd))
        # Gamma Gamma* = gamma gamma*: the rotation phase cancels (eq. relation_auto_gpp_+),
        # also on modes along n where phi_{k,n} is undefined
        acc[f"PLUS_l{l}"] = _bin_sums(cfg, bidx, special.peval(special.legendre(l), mu) * Fg * np.conj(Fg))
    for L in range(2, cfg.lmax + 1, 2):
        acc[f"GD_L{L}"] = _bin_sums(cfg, bidx, special.assoc_legendre(2, L, mu) * G * np.conj(Fd))
    for L in range(4, cfg.lmax + 1, 2):
        acc[f"MINUS_L{L}"] = _bin_sums(cfg, bidx, special.assoc_legendre(4, L, mu) * G * Gm)
    return _finish(cfg, acc, sc, counts, ksum)
