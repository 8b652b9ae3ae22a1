"""The learned stand-in for the plain window-convolved template path.

Training data come from ``template_plain`` (lpp_template_plain); the network,
its encoding of the templates and its inverse all run in the library
(lpp_mlp_*, lpp_emulator_encode, lpp_emulator_predict).  Torch tensors only
hold the device arrays.
"""
from __future__ import annotations

import ctypes as C

from ._lib import Mlp, _check, load

K_OUT_DEFAULT = tuple(0.01 * i for i in range(1, 31))


class Emulator:
    def __init__(self, ranges, n_k: int = 30, hidden=(256, 256, 256), max_batch: int = 4096, seed: int = 0):
        self.lib = load()
        self.ranges = [float(v) for r in ranges for v in r]
        self.n_k = n_k
        self.net = Mlp([5, *hidden, 5 * n_k], max_batch=max_batch, seed=seed)
        self.mean = self.sd = None

    def _r(self):
        return (C.c_double * 10)(*self.ranges)

    def fit(self, params, templates, nbar: float, sigma_gamma: float, epochs: int = 300, batch: int = 256,
            lr0: float = 2e-3, lr1: float = 1e-5, seed: int = 0) -> float:
        """params: float64 CUDA tensor [n, 5]; templates: float64 CUDA tensor [n, 5, n_k]."""
        import torch
        n = params.shape[0]
        X = torch.empty((n, 5), dtype=torch.float32, device="cuda")
        T = torch.empty((n, 5 * self.n_k), dtype=torch.float32, device="cuda")
        self.mean = torch.empty(5 * self.n_k, dtype=torch.float64, device="cuda")
        self.sd = torch.empty(5 * self.n_k, dtype=torch.float64, device="cuda")
        self.nbar, self.sigma_gamma = float(nbar), float(sigma_gamma)
        p = lambda t: C.c_void_p(t.data_ptr())
        _check(self.lib.lpp_emulator_encode(p(params), p(templates.contiguous()), C.c_int64(n), C.c_int32(self.n_k),
                                            self._r(), C.c_double(nbar), C.c_double(sigma_gamma), p(X), p(T),
                                            p(self.mean), p(self.sd),
                                            C.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "lpp_emulator_encode")
        return self.net.fit(X, T, batch=batch, epochs=epochs, lr0=lr0, lr1=lr1, seed=seed)

    def predict(self, params, out) -> None:
        """out: float64 CUDA tensor [n, 5, n_k] for params [n, 5]."""
        p = lambda t: C.c_void_p(t.data_ptr())
        self.net._stream()
        _check(self.lib.lpp_emulator_predict(self.net.handle, p(params), C.c_int64(params.shape[0]),
                                             C.c_int32(self.n_k), self._r(), C.c_double(self.nbar),
                                             C.c_double(self.sigma_gamma), p(self.mean), p(self.sd), p(out)),
               "lpp_emulator_predict")


def accuracy(emu, plain):
    """Per point and multipole: max_k |emu - plain| / max_k |plain| (the 1 %
    criterion), and the largest per-k relative error where |plain| exceeds
    10 % of its peak over k.  Arrays [n, 5, n_k] (numpy)."""
    import numpy as np
    peak = np.max(np.abs(plain), axis=2)
    rel = np.max(np.abs(emu - plain), axis=2) / peak
    mask = np.abs(plain) > 0.1 * peak[:, :, None]
    perk = np.where(mask, np.abs(emu - plain) / np.where(mask, np.abs(plain), 1.0), 0.0).max(axis=2)
    return rel, perk
