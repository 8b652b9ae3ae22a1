"""Field-level validation mocks of Sec. IV.A, generated on the GPU with torch.

Input generation only (no estimator arithmetic): a Gaussian density field
delta on an N^3 mesh of a periodic box with the analytic spectrum of
``synth.power_spectrum``, its tidal tensor T_ij = (khat_i khat_j -
delta_ij/3) delta (eq. validation_projection's input), and at every mesh
node inside a survey window (RA, Dec, distance ranges seen from an
observer) the projected field gamma = e_ij(dhat) T_ij, with dhat either the
node's own line of sight (cases (a) and (b) of Sec. IV.B) or one global
direction n (case (c)).

The mocks are handed to the estimator as field-level catalogs (as
``synth.lattice_catalogs`` does on the host): one galaxy and one random at
every window node, galaxy weight 1 + delta, galaxy shapes gamma / (1 + delta)
and randoms of weight 1, so that with nearest-grid-point assignment on the
same mesh the deposited density is delta - <delta> and the deposited shape
field is gamma exactly; nbar = 1 / H^3.  There is no Poisson noise: the
shot-noise terms the estimator subtracts are to be added back.

Seeds: torch's CUDA generator seeded with (2202 * 1000003 + 11839) * 1009 + mock.
"""
from __future__ import annotations

import math

import numpy as np

from . import power_spectrum

PAPER_WINDOW = dict(ra=(120.0, 260.0), dec=(-5.0, 70.0), r=(1000.0, 1500.0))


def _basis(dx, dy, dz, torch):
    """(e_theta, e_phi) of unit directions (columns of the standard rotation;
    phi = 0 at the poles)."""
    ct = dz.clamp(-1.0, 1.0)
    st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
    rho = torch.hypot(dx, dy)
    ok = rho > 0
    cp = torch.where(ok, dx / torch.where(ok, rho, torch.ones_like(rho)), torch.ones_like(rho))
    sp = torch.where(ok, dy / torch.where(ok, rho, torch.ones_like(rho)), torch.zeros_like(rho))
    et = (ct * cp, ct * sp, -st)
    ep = (-sp, cp, torch.zeros_like(cp))
    return et, ep


class FieldMocks:
    """Window nodes and their line-of-sight bases are set up once; each call
    of ``realise(mock)`` draws one density field and returns its catalogs."""

    def __init__(self, n=512, box=3000.0, origin=(0.0, 0.0, 0.0), observer=(2950.0, 1590.0, 150.0),
                 window=PAPER_WINDOW, global_los=None, device="cuda"):
        import torch
        self.torch = torch
        self.n, self.box = n, float(box)
        self.h = self.box / n
        self.origin = np.asarray(origin, dtype=np.float64)
        self.observer = np.asarray(observer, dtype=np.float64)
        self.device = device
        ra, dec, rr = window["ra"], window["dec"], window["r"]
        if global_los is None:  # direction of the window's angular midpoint
            a, d = math.radians(0.5 * (ra[0] + ra[1])), math.radians(0.5 * (dec[0] + dec[1]))
            global_los = (math.cos(d) * math.cos(a), math.cos(d) * math.sin(a), math.sin(d))
        g = np.asarray(global_los, dtype=np.float64)
        self.nhat = g / np.linalg.norm(g)
        # window nodes, one z-plane at a time (FP64 positions)
        idx = []
        ii = torch.arange(n, device=device, dtype=torch.float64)
        X, Y = torch.meshgrid(ii, ii, indexing="ij")
        for iz in range(n):
            px = self.origin[0] + X * self.h - self.observer[0]
            py = self.origin[1] + Y * self.h - self.observer[1]
            pz = torch.full_like(px, self.origin[2] + iz * self.h - self.observer[2])
            r = torch.sqrt(px * px + py * py + pz * pz)
            decd = torch.rad2deg(torch.asin(torch.clamp(pz / r, -1.0, 1.0)))
            rad = torch.remainder(torch.rad2deg(torch.atan2(py, px)), 360.0)
            inside = ((r >= rr[0]) & (r < rr[1]) & (decd >= dec[0]) & (decd < dec[1]) &
                      (rad >= ra[0]) & (rad < ra[1]))
            k = torch.nonzero(inside.reshape(-1)).reshape(-1)
            idx.append(k + iz * n * n)   # flat index (ix n + iy) + iz n^2 of the [iz][ix][iy] order below
        flat = torch.cat(idx)
        self.count = int(flat.numel())
        iz = flat // (n * n)
        ixy = flat % (n * n)
        ix, iy = ixy // n, ixy % n
        # the density and tidal fields are computed in [ix][iy][iz] order
        self.lin = (ix * n + iy) * n + iz
        self.x = (self.origin[0] + ix.to(torch.float64) * self.h).contiguous()
        self.y = (self.origin[1] + iy.to(torch.float64) * self.h).contiguous()
        self.z = (self.origin[2] + iz.to(torch.float64) * self.h).contiguous()
        dx, dy, dz = self.x - self.observer[0], self.y - self.observer[1], self.z - self.observer[2]
        rn = torch.sqrt(dx * dx + dy * dy + dz * dz)
        self.e_local = _basis(dx / rn, dy / rn, dz / rn, torch)
        nt = torch.tensor(self.nhat, device=device, dtype=torch.float64)
        et, ep = _basis(nt[0:1], nt[1:2], nt[2:3], torch)
        self.e_global = (tuple(v.expand(self.count) for v in et), tuple(v.expand(self.count) for v in ep))
        self.nbar = torch.full((self.count,), 1.0 / self.h ** 3, device=device, dtype=torch.float64)
        self.ones = torch.ones(self.count, device=device, dtype=torch.float64)
        # spectrum amplitude on the half-complex mesh
        kf = 2.0 * math.pi / self.box
        k1 = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64) * kf
        kz = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64) * kf
        self.kx, self.ky, self.kz = k1[:, None, None], k1[None, :, None], kz[None, None, :]
        kk = torch.sqrt(self.kx ** 2 + self.ky ** 2 + self.kz ** 2)
        pk = torch.from_numpy(power_spectrum(kk.cpu().numpy())).to(device)
        amp = torch.where(kk > 0, torch.sqrt(pk / self.h ** 3), torch.zeros_like(kk))
        self.amp = amp
        self.k2 = torch.where(kk > 0, kk * kk, torch.ones_like(kk))

    def realise(self, mock: int):
        """(gal_local, gal_global, ran): catalogs of CUDA FP64 tensors; the two
        galaxy catalogs share positions and weights and differ in the line of
        sight of the projection (own line of sight, or the global n)."""
        from . import Catalog
        torch = self.torch
        n = self.n
        gen = torch.Generator(device=self.device)
        gen.manual_seed((2202 * 1000003 + 11839) * 1009 + int(mock))
        # FP64 throughout: 1 + delta, the weight that the shapes are divided by, is
        # then never exactly zero in practice (an FP32 delta hits -1 exactly
        # about once per 10^8 nodes)
        white = torch.randn((n, n, n), generator=gen, device=self.device, dtype=torch.float64)
        dk = torch.fft.rfftn(white) * self.amp
        del white
        delta = torch.fft.irfftn(dk, s=(n, n, n)).reshape(-1)[self.lin]
        comps = (self.kx, self.ky, self.kz)
        T = {}
        for i in range(3):
            for j in range(i, 3):
                f = comps[i] * comps[j] / self.k2
                if i == j:
                    f = f - 1.0 / 3.0
                T[(i, j)] = torch.fft.irfftn(dk * f, s=(n, n, n)).reshape(-1)[self.lin]
                T[(j, i)] = T[(i, j)]
        del dk

        def project(et, ep):
            tt = sum(et[a] * T[(a, b)] * et[b] for a in range(3) for b in range(3))
            pp = sum(ep[a] * T[(a, b)] * ep[b] for a in range(3) for b in range(3))
            tp = sum(et[a] * T[(a, b)] * ep[b] for a in range(3) for b in range(3))
            return 0.5 * (tt - pp), tp
        w = 1.0 + delta
        g1l, g2l = project(*self.e_local)
        g1g, g2g = project(*self.e_global)
        gal_l = Catalog(self.x, self.y, self.z, w, self.nbar, (g1l / w).contiguous(), (g2l / w).contiguous())
        gal_g = Catalog(self.x, self.y, self.z, w, self.nbar, (g1g / w).contiguous(), (g2g / w).contiguous())
        ran = Catalog(self.x, self.y, self.z, self.ones, self.nbar)
        return gal_l, gal_g, ran
