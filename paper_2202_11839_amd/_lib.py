"""ctypes binding of liblpp.so (include/lpp.h): argument marshalling only.

Every step of the estimator runs in the library's HIP kernels; this module
passes pointers and sizes and never computes any part of the result.  PyTorch
provides the device memory (the plan's workspace is a torch uint8 tensor) and
the stream (torch's current stream).  If the shared library is missing the
import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpp.so")

LPP_F32, LPP_F64 = 0, 1
LPP_DD, LPP_GD, LPP_PLUS, LPP_MINUS, LPP_ALL = 1, 2, 4, 8, 15
STATUS = ["LPP_OK", "LPP_E_INVALID", "LPP_E_NONFINITE", "LPP_E_OUT_OF_BOX", "LPP_E_AT_OBSERVER",
          "LPP_E_NO_RANDOMS", "LPP_E_WORKSPACE", "LPP_E_NOMEM", "LPP_E_DEVICE", "LPP_E_UNSUPPORTED"]

EXPORTS = ["lpp_plan_create", "lpp_plan_destroy", "lpp_workspace_size", "lpp_set_workspace", "lpp_set_stream",
           "lpp_result_layout", "lpp_series_name", "lpp_estimate", "lpp_estimate_batch", "lpp_deposit_weights",
           "lpp_fft3d", "lpp_fft3d_zblocked", "lpp_status_string", "lpp_version", "lpp_set_profiling", "lpp_get_profile",
           "lpp_reset_profile", "lpp_batch_stats", "lpp_get_tuning", "lpp_set_tuning", "lpp_autotune",
           "lpp_window_multipoles", "lpp_window_pairs", "lpp_window_coefficient", "lpp_template_plain", "lpp_template_multipoles",
           "lpp_template_plain_noalloc", "lpp_mlp_create",
           "lpp_mlp_destroy", "lpp_mlp_set_stream", "lpp_mlp_num_params", "lpp_mlp_get_params", "lpp_mlp_set_params",
           "lpp_mlp_forward", "lpp_mlp_train_step", "lpp_mlp_fit", "lpp_emulator_encode", "lpp_emulator_predict"]
TUNING_FIELDS = ["fft_rows_x", "fft_cols_y", "fft_cols_z", "bin_blocks", "gather_density", "gather_shape", "serial",
                 "fft_streaming", "unfused"]
STAGES = ["sort", "deposit", "fft_x", "fft_yz", "bin", "other"]


class LppError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{what}: {name}")


class Tuning(C.Structure):
    _fields_ = [(name, C.c_int32) for name in TUNING_FIELDS]


class Config(C.Structure):
    _fields_ = [("mesh_n", C.c_int32), ("box_size", C.c_double), ("box_origin", C.c_double * 3),
                ("observer", C.c_double * 3), ("assignment", C.c_int32), ("interlacing", C.c_int32),
                ("compensate", C.c_int32), ("precision", C.c_int32), ("lmax", C.c_int32),
                ("spectra", C.c_uint32), ("n_kbins", C.c_int32), ("dn_num", C.c_int32), ("dn_den", C.c_int32),
                ("global_los", C.c_int32), ("los", C.c_double * 3)]


class CatalogStruct(C.Structure):
    _fields_ = [("n", C.c_int64), ("on_device", C.c_int32), ("dtype", C.c_int32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("w", C.c_void_p),
                ("nbar", C.c_void_p), ("g1", C.c_void_p), ("g2", C.c_void_p)]


class ResultStruct(C.Structure):
    _fields_ = [("n_modes", C.c_void_p), ("k_eff", C.c_void_p), ("k_lo", C.c_void_p), ("k_hi", C.c_void_p),
                ("re", C.c_void_p), ("im", C.c_void_p), ("alpha", C.c_double), ("norm_I", C.c_double),
                ("shot_dd", C.c_double), ("shot_plus", C.c_double), ("sum_w_gal", C.c_double),
                ("sum_w_ran", C.c_double)]


_LIB = None


def load() -> C.CDLL:
    """Load the in-tree liblpp.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_11839_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.lpp_plan_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
    lib.lpp_plan_destroy.argtypes = [P]
    lib.lpp_workspace_size.argtypes = [P, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
    lib.lpp_set_workspace.argtypes = [P, P, C.c_size_t]
    lib.lpp_set_stream.argtypes = [P, P]
    lib.lpp_result_layout.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lpp_series_name.argtypes = [P, C.c_int32]
    lib.lpp_series_name.restype = C.c_char_p
    lib.lpp_estimate.argtypes = [P, C.POINTER(CatalogStruct), C.POINTER(CatalogStruct), C.POINTER(ResultStruct)]
    lib.lpp_estimate_batch.argtypes = [P, C.c_int32, C.POINTER(CatalogStruct), C.POINTER(CatalogStruct),
                                       C.POINTER(ResultStruct), C.POINTER(C.c_int32)]
    lib.lpp_deposit_weights.argtypes = [P, C.POINTER(CatalogStruct), C.c_double, P]
    lib.lpp_fft3d.argtypes = [P, P]
    lib.lpp_status_string.argtypes = [C.c_int]
    lib.lpp_status_string.restype = C.c_char_p
    lib.lpp_version.restype = C.c_char_p
    lib.lpp_set_profiling.argtypes = [P, C.c_int32]
    lib.lpp_get_profile.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    lib.lpp_reset_profile.argtypes = [P]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or C.c_int
    for name in ("lpp_plan_create", "lpp_plan_destroy", "lpp_workspace_size", "lpp_set_workspace",
                 "lpp_set_stream", "lpp_result_layout", "lpp_estimate", "lpp_estimate_batch",
                 "lpp_deposit_weights", "lpp_fft3d", "lpp_set_profiling", "lpp_get_profile",
                 "lpp_reset_profile"):
        getattr(lib, name).restype = C.c_int
    _LIB = lib
    return lib


def _check(st: int, what: str):
    if st != 0:
        raise LppError(st, what)


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Cols:
    """Keeps the arrays behind a CatalogStruct alive."""

    def __init__(self, cat, dtype: int, keep: list):
        self.keep = keep
        cols = {}
        first = cat.x
        on_dev = _is_torch(first) and first.is_cuda
        np_dtype = np.float64 if dtype == LPP_F64 else np.float32
        n = int(first.shape[0])
        for name in ("x", "y", "z", "w", "nbar", "g1", "g2"):
            a = getattr(cat, name, None)
            if a is None:
                cols[name] = None
                continue
            if on_dev:
                import torch
                tdt = torch.float64 if dtype == LPP_F64 else torch.float32
                if a.dtype != tdt or not a.is_contiguous() or not a.is_cuda:
                    raise TypeError(f"device column {name} must be a contiguous CUDA tensor of {tdt}")
                cols[name] = a.data_ptr()
                keep.append(a)
            else:
                arr = np.ascontiguousarray(a, dtype=np_dtype)
                keep.append(arr)
                cols[name] = arr.ctypes.data
            if int(a.shape[0]) != n:
                raise ValueError(f"column {name} has {a.shape[0]} rows, expected {n}")
        self.struct = CatalogStruct(n, 1 if on_dev else 0, dtype, cols["x"], cols["y"], cols["z"], cols["w"],
                                    cols["nbar"], cols["g1"], cols["g2"])


class Plan:
    """One estimator configuration (mesh, box, observer, assignment, multipoles, bins).

    ``los``: None for each object's own line of sight (the LPP estimator), or
    a vector: one line of sight for every object (global plane-parallel)."""

    def __init__(self, mesh_n: int, box_size: float, box_origin, observer=(0.0, 0.0, 0.0), assignment: int = 3,
                 interlacing: int = 1, compensate: int = 1, precision: str = "f32", lmax: int = 4,
                 spectra: int = LPP_ALL, n_kbins: int = 16, dn=None, los=None):
        self.lib = load()
        cfg = Config()
        cfg.mesh_n = mesh_n
        cfg.box_size = box_size
        cfg.box_origin = (C.c_double * 3)(*box_origin)
        cfg.observer = (C.c_double * 3)(*observer)
        cfg.assignment = assignment
        cfg.interlacing = interlacing
        cfg.compensate = compensate
        cfg.precision = LPP_F64 if precision in ("f64", LPP_F64) else LPP_F32
        cfg.lmax = lmax
        cfg.spectra = spectra
        cfg.n_kbins = n_kbins
        cfg.dn_num, cfg.dn_den = (0, 0) if dn is None else dn
        cfg.global_los = 0 if los is None else 1
        cfg.los = (C.c_double * 3)(*((0.0, 0.0, 0.0) if los is None else los))
        self.cfg = cfg
        self.precision = cfg.precision
        h = C.c_void_p()
        _check(self.lib.lpp_plan_create(C.byref(cfg), C.byref(h)), "lpp_plan_create")
        self.handle = h
        ns, nb = C.c_int32(), C.c_int32()
        _check(self.lib.lpp_result_layout(h, C.byref(ns), C.byref(nb)), "lpp_result_layout")
        self.n_series, self.n_kbins = ns.value, nb.value
        self.series = [self.lib.lpp_series_name(h, i).decode() for i in range(self.n_series)]
        self._ws = None
        self._ws_cap = (0, 0)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.lpp_plan_destroy(h)
            self.handle = None

    # ---- device plumbing (torch owns memory and stream) ----
    def _prepare_device(self, n_gal: int, n_ran: int):
        import torch
        if not torch.cuda.is_available():
            raise LppError(8, "no HIP device")
        self.lib.lpp_set_stream(self.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        if n_gal > self._ws_cap[0] or n_ran > self._ws_cap[1]:
            ng, nr = max(n_gal, self._ws_cap[0]), max(n_ran, self._ws_cap[1])
            sz = C.c_size_t()
            _check(self.lib.lpp_workspace_size(self.handle, ng, nr, C.byref(sz)), "lpp_workspace_size")
            self._ws = None
            self._ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device="cuda")
            ptr = (self._ws.data_ptr() + 255) // 256 * 256
            _check(self.lib.lpp_set_workspace(self.handle, C.c_void_p(ptr), int(sz.value)), "lpp_set_workspace")
            self._ws_cap = (ng, nr)

    def _result(self):
        nb, ns = self.n_kbins, self.n_series
        arrs = dict(n_modes=np.zeros(nb, np.int64), k_eff=np.zeros(nb), k_lo=np.zeros(nb), k_hi=np.zeros(nb),
                    re=np.zeros((ns, nb)), im=np.zeros((ns, nb)))
        rs = ResultStruct(*(arrs[k].ctypes.data for k in ("n_modes", "k_eff", "k_lo", "k_hi", "re", "im")))
        return arrs, rs

    @staticmethod
    def _pack(arrs, rs, series) -> Dict:
        out = dict(arrs)
        out["series"] = list(series)
        for k in ("alpha", "norm_I", "shot_dd", "shot_plus", "sum_w_gal", "sum_w_ran"):
            out[k] = float(getattr(rs, k))
        return out

    def estimate(self, gal, ran, dtype: Optional[int] = None) -> Dict:
        """Multipoles of one catalog pair; returns numpy arrays (re/im [series, bin], n_modes, k_eff, ...)."""
        dt = self._dtype(gal) if dtype is None else dtype
        keep: list = []
        cg = _Cols(gal, dt, keep)
        cr = _Cols(ran, dt, keep)
        self._prepare_device(cg.struct.n, cr.struct.n)
        arrs, rs = self._result()
        _check(self.lib.lpp_estimate(self.handle, C.byref(cg.struct), C.byref(cr.struct), C.byref(rs)),
               "lpp_estimate")
        return self._pack(arrs, rs, self.series)

    def estimate_batch(self, gals: List, rans: List, dtype: Optional[int] = None):
        n = len(gals)
        dt = self._dtype(gals[0]) if dtype is None else dtype
        keep: list = []
        cg = [_Cols(g, dt, keep) for g in gals]
        cr = [_Cols(r, dt, keep) for r in rans]
        self._prepare_device(max(c.struct.n for c in cg), max(c.struct.n for c in cr))
        G = (CatalogStruct * n)(*[c.struct for c in cg])
        R = (CatalogStruct * n)(*[c.struct for c in cr])
        res = [self._result() for _ in range(n)]
        RS = (ResultStruct * n)(*[r[1] for r in res])
        st = (C.c_int32 * n)()
        self.lib.lpp_estimate_batch(self.handle, n, G, R, RS, st)
        outs = []
        for i in range(n):
            if st[i] != 0:
                outs.append(LppError(st[i], f"catalog {i}"))
            else:
                outs.append(self._pack(res[i][0], RS[i], self.series))
        return outs

    def tuning(self) -> Dict[str, int]:
        """Launch shapes in use (defaults resolved)."""
        t = Tuning()
        _check(self.lib.lpp_get_tuning(self.handle, C.byref(t)), "lpp_get_tuning")
        return {name: getattr(t, name) for name in TUNING_FIELDS}

    def set_tuning(self, **kw) -> None:
        """Set launch shapes (fields of lpp_tuning; 0 = default, unnamed fields keep their value)."""
        t = Tuning()
        _check(self.lib.lpp_get_tuning(self.handle, C.byref(t)), "lpp_get_tuning")
        for name, value in kw.items():
            if name not in TUNING_FIELDS:
                raise KeyError(name)
            setattr(t, name, int(value))
        _check(self.lib.lpp_set_tuning(self.handle, C.byref(t)), "lpp_set_tuning")

    def autotune(self, gal, ran, cache_path: Optional[str] = None) -> Dict[str, int]:
        """Time the candidate launch shapes on this catalog pair and keep the fastest."""
        keep: list = []
        dt = self._dtype(gal)
        cg, cr = _Cols(gal, dt, keep), _Cols(ran, dt, keep)
        self._prepare_device(cg.struct.n, cr.struct.n)
        path = None if cache_path is None else cache_path.encode()
        _check(self.lib.lpp_autotune(self.handle, C.byref(cg.struct), C.byref(cr.struct), path), "lpp_autotune")
        return self.tuning()

    def window_multipoles(self, ran, alpha: float, lmax: int = 8, n_rbins: int = 100, rmax: float = 2000.0):
        """Q_l(r)/I, l = 0, 2, .., lmax, of the window traced by ``ran`` (see lpp_window_multipoles)."""
        import numpy as np
        keep: list = []
        cr = _Cols(ran, self._dtype(ran), keep)
        self._prepare_device(1, cr.struct.n)
        nell = lmax // 2 + 1
        Q = np.zeros(nell * n_rbins)
        r_eff = np.zeros(n_rbins)
        counts = np.zeros(n_rbins, dtype=np.int64)
        norm = C.c_double()
        dp = C.POINTER(C.c_double)
        _check(self.lib.lpp_window_multipoles(self.handle, C.byref(cr.struct), C.c_double(alpha), C.c_int32(lmax),
                                              C.c_int32(n_rbins), C.c_double(rmax), Q.ctypes.data_as(dp),
                                              r_eff.ctypes.data_as(dp), counts.ctypes.data_as(C.POINTER(C.c_int64)),
                                              C.byref(norm)), "lpp_window_multipoles")
        return dict(ells=list(range(0, lmax + 1, 2)), Q=Q.reshape(nell, n_rbins), r_eff=r_eff, counts=counts,
                    norm_I=norm.value)

    def batch_stats(self) -> tuple:
        """(graphs captured, graph launches) of estimate_batch over the plan's life."""
        a, b = C.c_int64(), C.c_int64()
        _check(self.lib.lpp_batch_stats(self.handle, C.byref(a), C.byref(b)), "lpp_batch_stats")
        return a.value, b.value

    def deposit_weights(self, cat, scale: float, mesh) -> None:
        """Mass-assign cat.w * scale onto ``mesh`` (torch complex tensor N^3 on the device)."""
        keep: list = []
        cc = _Cols(cat, self._dtype(cat), keep)
        self._prepare_device(1, cc.struct.n)
        _check(self.lib.lpp_deposit_weights(self.handle, C.byref(cc.struct), float(scale),
                                            C.c_void_p(mesh.data_ptr())), "lpp_deposit_weights")

    def fft3d(self, mesh) -> None:
        """In-place forward 3D DFT of a contiguous complex torch tensor of shape (N, N, N) [z, y, x]."""
        import torch
        self.lib.lpp_set_stream(self.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(self.lib.lpp_fft3d(self.handle, C.c_void_p(mesh.data_ptr())), "lpp_fft3d")

    def fft3d_zblocked(self, mesh) -> None:
        """In-place forward 3D DFT of a contiguous complex torch tensor of N^3
        values in the estimator's z-blocked order (lpp_fft3d_zblocked)."""
        import torch
        self.lib.lpp_set_stream(self.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(self.lib.lpp_fft3d_zblocked(self.handle, C.c_void_p(mesh.data_ptr())), "lpp_fft3d_zblocked")

    def set_profiling(self, on: bool) -> None:
        _check(self.lib.lpp_set_profiling(self.handle, 1 if on else 0), "lpp_set_profiling")
        _check(self.lib.lpp_reset_profile(self.handle), "lpp_reset_profile")

    def profile(self) -> Dict[str, tuple]:
        """{stage: (milliseconds, kernel launches)} accumulated since set_profiling."""
        n = len(STAGES)
        ms = (C.c_double * n)()
        ln = (C.c_int64 * n)()
        _check(self.lib.lpp_get_profile(self.handle, ms, ln, n), "lpp_get_profile")
        return {STAGES[i]: (ms[i], ln[i]) for i in range(n)}

    def _dtype(self, cat) -> int:
        x = cat.x
        if _is_torch(x):
            import torch
            return LPP_F64 if x.dtype == torch.float64 else LPP_F32
        return LPP_F64 if np.asarray(x).dtype == np.float64 else LPP_F32


class Mlp:
    """The emulator network of the library (lpp_mlp_*); arrays are float32 CUDA tensors."""

    def __init__(self, widths, max_batch: int, seed: int = 0):
        self.lib = load()
        self.widths = list(widths)
        w = (C.c_int32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(self.lib.lpp_mlp_create(w, C.c_int32(len(self.widths) - 1), C.c_int64(max_batch), C.c_uint64(seed),
                                       C.byref(h)), "lpp_mlp_create")
        self.handle = h
        n = C.c_int64()
        _check(self.lib.lpp_mlp_num_params(h, C.byref(n)), "lpp_mlp_num_params")
        self.n_params = n.value

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.lpp_mlp_destroy(self.handle)
            self.handle = None

    def _stream(self):
        import torch
        self.lib.lpp_mlp_set_stream(self.handle, C.c_void_p(torch.cuda.current_stream().cuda_stream))

    @staticmethod
    def _ptr(t):
        assert t.is_cuda and t.is_contiguous(), "float32 contiguous CUDA tensor expected"
        return C.c_void_p(t.data_ptr())

    def params(self, grads: bool = False):
        import numpy as np
        self._stream()
        p = np.zeros(self.n_params, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32) if grads else None
        fp = C.POINTER(C.c_float)
        _check(self.lib.lpp_mlp_get_params(self.handle, p.ctypes.data_as(fp),
                                           g.ctypes.data_as(fp) if grads else None), "lpp_mlp_get_params")
        return (p, g) if grads else p

    def set_params(self, p) -> None:
        import numpy as np
        self._stream()
        q = np.ascontiguousarray(p, dtype=np.float32)
        _check(self.lib.lpp_mlp_set_params(self.handle, q.ctypes.data_as(C.POINTER(C.c_float))), "lpp_mlp_set_params")

    def forward(self, X, Y) -> None:
        self._stream()
        _check(self.lib.lpp_mlp_forward(self.handle, self._ptr(X), C.c_int64(X.shape[0]), self._ptr(Y)),
               "lpp_mlp_forward")

    def train_step(self, X, T, lr: float) -> float:
        self._stream()
        loss = C.c_float()
        _check(self.lib.lpp_mlp_train_step(self.handle, self._ptr(X), self._ptr(T), C.c_int64(X.shape[0]),
                                           C.c_float(lr), C.byref(loss)), "lpp_mlp_train_step")
        return loss.value

    def fit(self, X, T, batch: int, epochs: int, lr0: float, lr1: float, seed: int = 0) -> float:
        self._stream()
        loss = C.c_float()
        _check(self.lib.lpp_mlp_fit(self.handle, self._ptr(X), self._ptr(T), C.c_int64(X.shape[0]),
                                    C.c_int32(batch), C.c_int32(epochs), C.c_float(lr0), C.c_float(lr1),
                                    C.c_uint64(seed), C.byref(loss)), "lpp_mlp_fit")
        return loss.value


def window_pairs(ran, alpha: float, norm_I: float, observer=(0.0, 0.0, 0.0), los: str = "midpoint", lmax: int = 8,
                 n_rbins: int = 100, rmax: float = 2000.0) -> Dict:
    """Q_l(r)/I by pair counting of the catalog ``ran`` (lpp_window_pairs);
    ``los`` "midpoint" (the pair's direction) or "endpoint" (its first point).
    Columns: numpy arrays (FP64) or CUDA tensors of one dtype."""
    import numpy as np
    lib = load()
    first = ran.x
    dtype = LPP_F32 if (_is_torch(first) and str(first.dtype) == "torch.float32") else LPP_F64
    keep: list = []
    cr = _Cols(ran, dtype, keep)
    nell = lmax // 2 + 1
    Q = np.zeros(nell * n_rbins)
    r_eff = np.zeros(n_rbins)
    counts = np.zeros(n_rbins, dtype=np.int64)
    dp = C.POINTER(C.c_double)
    obs = (C.c_double * 3)(*[float(v) for v in observer])
    stream = C.c_void_p(0)
    if cr.struct.on_device:
        import torch
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(lib.lpp_window_pairs(C.byref(cr.struct), C.c_double(alpha), C.c_double(norm_I), obs,
                                C.c_int32({"endpoint": 0, "midpoint": 1}[los]), C.c_int32(lmax), C.c_int32(n_rbins),
                                C.c_double(rmax), Q.ctypes.data_as(dp), r_eff.ctypes.data_as(dp),
                                counts.ctypes.data_as(C.POINTER(C.c_int64)), stream), "lpp_window_pairs")
    return dict(ells=list(range(0, lmax + 1, 2)), Q=Q.reshape(nell, n_rbins), r_eff=r_eff, counts=counts)


def window_coefficient(mX: int, l: int, lp: int, lpp: int) -> float:
    """Coefficient of Q_{l''} in Q^X_{l l'} (host computation of the library)."""
    out = C.c_double()
    _check(load().lpp_window_coefficient(C.c_int32(mX), C.c_int32(l), C.c_int32(lp), C.c_int32(lpp), C.byref(out)),
           "lpp_window_coefficient")
    return out.value


TEMPLATE_ROWS = {"lpp_template_plain": 5, "lpp_template_plain_noalloc": 5, "lpp_template_multipoles": 9}
TEMPLATE_SERIES = ["DD_l0", "DD_l2", "DD_l4", "GD_L2", "GD_L4", "PLUS_l0", "PLUS_l2", "PLUS_l4", "MINUS_L4"]


def _template(entry: str, pfid, k_min, k_max, r_q, Q, params, k_out, nbar, sigma_gamma, out):
    import numpy as np
    lib = load()
    rows = TEMPLATE_ROWS[entry]
    dp = C.POINTER(C.c_double)
    pf = np.ascontiguousarray(pfid, dtype=np.float64)
    rq = np.ascontiguousarray(r_q, dtype=np.float64)
    qq = np.ascontiguousarray(Q, dtype=np.float64)
    ko = np.ascontiguousarray(k_out, dtype=np.float64)
    on_dev = hasattr(params, "is_cuda") and params.is_cuda
    if on_dev:
        import torch
        assert params.dtype == torch.float64 and params.is_contiguous() and out is not None
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == params.shape[0] * rows * ko.size
        n_pts = params.shape[0]
        p_ptr = C.cast(C.c_void_p(params.data_ptr()), dp)
        o_ptr = C.cast(C.c_void_p(out.data_ptr()), dp)
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    else:
        pr = np.ascontiguousarray(params, dtype=np.float64)
        n_pts = pr.shape[0]
        if out is None:
            out = np.zeros((n_pts, rows, ko.size))
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == n_pts * rows * ko.size
        p_ptr, o_ptr, stream = pr.ctypes.data_as(dp), out.ctypes.data_as(dp), C.c_void_p(0)
    _check(getattr(lib, entry)(pf.ctypes.data_as(dp), C.c_double(k_min), C.c_double(k_max), C.c_int32(pf.size),
                               rq.ctypes.data_as(dp), qq.ctypes.data_as(dp), C.c_int32(rq.size), p_ptr,
                               C.c_int64(n_pts), ko.ctypes.data_as(dp), C.c_int32(ko.size), C.c_double(nbar),
                               C.c_double(sigma_gamma), o_ptr, C.c_int32(1 if on_dev else 0), stream), entry)
    return out


def template_plain(pfid, k_min: float, k_max: float, r_q, Q, params, k_out, nbar: float, sigma_gamma: float,
                   out=None):
    """The plain window-convolved template path on the GPU (lpp_template_plain).

    ``params`` (n_pts, 5) and ``out`` (n_pts, 5, n_k) may be numpy arrays
    (host) or float64 CUDA tensors (device, then ``out`` must be given); the
    tables ``pfid`` (4096), ``r_q``, ``Q`` (5, n_q) and ``k_out`` are host arrays."""
    return _template("lpp_template_plain", pfid, k_min, k_max, r_q, Q, params, k_out, nbar, sigma_gamma, out)


def template_plain_noalloc(pfid, k_min: float, k_max: float, r_q, Q, params, k_out, nbar: float,
                           sigma_gamma: float, out=None):
    """lpp_template_plain_noalloc: template_plain with the library's static
    device scratch instead of per-call device allocations."""
    return _template("lpp_template_plain_noalloc", pfid, k_min, k_max, r_q, Q, params, k_out, nbar, sigma_gamma,
                     out)


def template_multipoles(pfid, k_min: float, k_max: float, r_q, Q, params, k_out, nbar: float, sigma_gamma: float,
                        out=None):
    """All four families (lpp_template_multipoles): out (n_pts, 9, n_k) in the
    order of TEMPLATE_SERIES."""
    return _template("lpp_template_multipoles", pfid, k_min, k_max, r_q, Q, params, k_out, nbar, sigma_gamma, out)


def version() -> str:
    return load().lpp_version().decode()
