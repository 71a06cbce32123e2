"""Python binding of the gfx950 level-set ILT library (ctypes, marshalling only).

Every function here checks tensor shapes, dtypes and devices, packs the C
structs declared in ``include/ilt.h`` and calls the library; all arithmetic
happens in the HIP kernels.  Importing this module loads ``libilt.so`` built
in-tree by ``paper_2303_12529_amd/build.py`` and fails loudly if it is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libilt.so")

ILT_OK, ILT_EINVAL, ILT_ENOMEM, ILT_EDEVICE, ILT_ENUMERIC, ILT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ILT_FP32 = 0
ILT_BF16X3 = 1
ILT_FP64 = 2
ILT_FLAG_RECOMPUTE_FIELDS = 1
ILT_FLAG_GWINDOW_ADJOINT = 2
ILT_FLAG_HOPKINS_FORWARD = 4
TRACE_W = 8
TRACE_COLUMNS = ("i", "loss", "l2", "pvb", "flips", "max_g", "dt", "t_ns")
PHASES = ("spectrum", "window_rows", "image", "resist", "adjoint", "gradient", "levelset_step", "reinit")


class IltError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("ILT error %d: %s" % (code, msg))
        self.code = code


class _Optics(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("P", ctypes.c_int), ("K", ctypes.c_int), ("n_sets", ctypes.c_int),
                ("precision", ctypes.c_int), ("flags", ctypes.c_int), ("h_kernels", ctypes.c_void_p),
                ("h_weights", ctypes.c_void_p)]


class _Corner(ctypes.Structure):
    _fields_ = [("set", ctypes.c_int), ("dose", ctypes.c_float), ("omega", ctypes.c_float)]


class _Params(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reinit_every", ctypes.c_int), ("dt_mode", ctypes.c_int),
                ("init_mode", ctypes.c_int), ("eta", ctypes.c_float), ("dt_max", ctypes.c_float),
                ("lambda_", ctypes.c_float), ("sigma_z", ctypes.c_float), ("i_th", ctypes.c_float),
                ("eps_kappa", ctypes.c_float), ("d_lower", ctypes.c_float), ("d_upper", ctypes.c_float),
                ("n_corners", ctypes.c_int), ("corners", _Corner * 4), ("optimizer", ctypes.c_int),
                ("iter0", ctypes.c_int)]


class _Report(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int), ("status", ctypes.c_int), ("loss", ctypes.c_double),
                ("l2", ctypes.c_longlong), ("pvb", ctypes.c_longlong), ("flips", ctypes.c_longlong)]


class _Tuning(ctypes.Structure):
    _fields_ = [("store_fields", ctypes.c_int), ("b3_xsplit", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("st_xsplit", ctypes.c_int)]


class _Clip(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("d_target", ctypes.c_void_p), ("d_phi", ctypes.c_void_p),
                ("d_trace", ctypes.c_void_p), ("params", _Params)]


ILT_BATCH_MAX_SIZES, ILT_BATCH_MAX_LANES, ILT_BATCH_MAX_CLIPS = 8, 4, 1024

_lib = None
_VP = ctypes.c_void_p


def load_library(path: str = LIB_PATH):
    """Load libilt.so and declare the C signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libilt.so is not built (%s); run paper_2303_12529_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    sig = {
        "ilt_create": [ctypes.POINTER(_VP), ctypes.POINTER(_Optics), ctypes.c_int, _VP],
        "ilt_destroy": [_VP],
        "ilt_get_dims": [_VP, ctypes.POINTER(ctypes.c_int)] + [ctypes.POINTER(ctypes.c_int)] * 3,
        "litho_forward": [_VP, _VP, ctypes.c_int, _VP],
        "litho_forward_phi": [_VP, _VP, ctypes.c_int, _VP],
        "litho_forward_f64": [_VP, _VP, ctypes.c_int, _VP],
        "litho_adjoint_f64": [_VP, _VP, _VP, ctypes.c_int, _VP],
        "ilt_solve_f64": [_VP, _VP, _VP, ctypes.POINTER(_Params), ctypes.POINTER(_Report), _VP],
        "ilt_shifted_heaviside": [_VP, ctypes.c_float, ctypes.c_longlong, _VP, _VP],
        "ilt_epe": [_VP, _VP, ctypes.c_float, ctypes.c_int, ctypes.c_float, ctypes.POINTER(ctypes.c_float), _VP, _VP],
        "litho_adjoint": [_VP, _VP, _VP, ctypes.c_int, _VP],
        "resist_loss": [_VP, _VP, _VP, ctypes.POINTER(_Params), _VP, _VP],
        "levelset_step": [_VP, _VP, _VP, _VP, ctypes.POINTER(_Params), _VP],
        "edt_reinit": [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_Params)],
        "edt_reinit_noalloc": [ctypes.c_int, _VP, _VP, ctypes.c_float, ctypes.c_float, _VP, _VP, _VP],
        "ilt_solve": [_VP, _VP, _VP, ctypes.POINTER(_Params), ctypes.POINTER(_Report), _VP],
        "ilt_solve_modulated": [_VP, _VP, _VP, _VP, ctypes.POINTER(_Params), ctypes.POINTER(_Report), _VP],
        "ilt_profile": [_VP, ctypes.c_int],
        "ilt_set_graph": [_VP, ctypes.c_int],
        "ilt_profile_read": [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int],
        "ilt_get_tuning": [_VP, ctypes.POINTER(_Tuning)],
        "ilt_set_tuning": [_VP, ctypes.POINTER(_Tuning)],
        "ilt_autotune": [_VP, ctypes.c_char_p, ctypes.POINTER(_Tuning), ctypes.POINTER(ctypes.c_double)],
        "ilt_batch_create": [ctypes.POINTER(_VP), ctypes.POINTER(_Optics), ctypes.POINTER(ctypes.c_int),
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP],
        "ilt_batch_destroy": [_VP],
        "ilt_batch_set_graph": [_VP, ctypes.c_int],
        "ilt_solve_batch": [_VP, ctypes.c_int, ctypes.POINTER(_Clip), ctypes.POINTER(_Report)],
        "ilt_batch_autotune": [_VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_Tuning),
                               ctypes.POINTER(ctypes.c_double)],
        "ilt_layout_extract": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP],
        "ilt_layout_stitch": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP],
        "ilt_layout_grid": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_int)],
        "ilt_solve_layout": [_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(_Params), _VP, _VP, _VP, ctypes.POINTER(_Report)],
        "ilt_shot_count": [_VP, _VP, ctypes.c_int, ctypes.c_int, _VP, _VP],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ilt_last_error.argtypes = []
    lib.ilt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != ILT_OK:
        raise IltError(rc, load_library().ilt_last_error().decode(errors="replace"))


@dataclasses.dataclass
class Params:
    """Method settings (see ilt_params in include/ilt.h)."""
    iters: int = 20
    reinit_every: int = 5
    dt_mode: int = 0
    init_mode: int = 0
    eta: float = 0.85
    dt_max: float = 5.0
    lam: float = 0.05
    sigma_z: float = 50.0
    i_th: float = 0.225
    eps_kappa: float = 1e-12
    d_lower: float = -100.0
    d_upper: float = 900.0
    corners: tuple = ((0, 1.0, 1.0),)
    optimizer: int = 0              # 0: gradient, 1: conjugate gradient (Polak-Ribiere+)
    iter0: int = 0                  # index of the first iteration (resuming a solve)

    @classmethod
    def from_dict(cls, d: dict, **over):
        kw = {f.name: d[f.name] for f in dataclasses.fields(cls) if f.name in d}
        kw.update(over)
        kw["corners"] = tuple(tuple(c) for c in kw.get("corners", ((0, 1.0, 1.0),)))
        return cls(**kw)

    def to_c(self) -> _Params:
        p = _Params()
        p.iters, p.reinit_every, p.dt_mode, p.init_mode = self.iters, self.reinit_every, self.dt_mode, self.init_mode
        p.eta, p.dt_max, p.lambda_, p.sigma_z = self.eta, self.dt_max, self.lam, self.sigma_z
        p.i_th, p.eps_kappa, p.d_lower, p.d_upper = self.i_th, self.eps_kappa, self.d_lower, self.d_upper
        if not 1 <= len(self.corners) <= 4:
            raise ValueError("1..4 corners")
        p.n_corners = len(self.corners)
        p.optimizer = int(self.optimizer)
        p.iter0 = int(self.iter0)
        for i, (s, d, w) in enumerate(self.corners):
            p.corners[i].set, p.corners[i].dose, p.corners[i].omega = int(s), float(d), float(w)
        return p


def _ptr(t, dtype, shape, name, device):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device != device:
        raise ValueError("%s is on %s, context is on %s" % (name, t.device, device))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _optics(kernels, weights, N, precision, flags):
    """Pack ilt_optics; returns (struct, arrays that must outlive the call)."""
    kernels = np.asarray(kernels)
    weights = np.asarray(weights, dtype=np.float64)
    if kernels.ndim == 3:
        kernels = kernels[None]
        weights = weights[None]
    ns, K, P, P2 = kernels.shape
    if P != P2 or weights.shape != (ns, K):
        raise ValueError("kernels must be [n_sets, K, P, P] and weights [n_sets, K]")
    kr = np.ascontiguousarray(np.stack([kernels.real, kernels.imag], axis=-1), dtype=np.float64)
    wr = np.ascontiguousarray(weights)
    o = _Optics(N=int(N), P=int(P), K=int(K), n_sets=int(ns), precision=int(precision), flags=int(flags),
                h_kernels=kr.ctypes.data, h_weights=wr.ctypes.data)
    return o, (kr, wr), (int(P), int(K), int(ns))


class Context:
    """A library context on the current torch CUDA (HIP) device and stream."""

    def __init__(self, kernels: np.ndarray, weights: np.ndarray, N: int, precision: int = ILT_FP32,
                 flags: int = 0):
        import torch
        lib = load_library()
        o, _keep, (P, K, ns) = _optics(kernels, weights, N, precision, flags)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        h = _VP()
        _check(lib.ilt_create(ctypes.byref(h), ctypes.byref(o), 1, _VP(self.stream.cuda_stream)))
        self._h = h
        self.N, self.P, self.K, self.n_sets = int(N), int(P), int(K), int(ns)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ilt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, t, name, dtype=None):
        import torch
        return _ptr(t, dtype or torch.float32, (self.N, self.N), name, self.device)

    def litho_forward(self, mask, set_: int = 0, out=None):
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float32, device=self.device)
        _check(load_library().litho_forward(self._h, self._img(mask, "mask"), int(set_), self._img(out, "out")))
        return out

    def litho_forward_phi(self, phi, set_: int = 0, out=None):
        """Aerial image of the mask [phi <= 0] (the mask is formed on the device)."""
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float32, device=self.device)
        _check(load_library().litho_forward_phi(self._h, self._img(phi, "phi"), int(set_), self._img(out, "out")))
        return out

    def litho_adjoint(self, mask, dL_dI, set_: int = 0, out=None):
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float32, device=self.device)
        _check(load_library().litho_adjoint(self._h, self._img(mask, "mask"), self._img(dL_dI, "dL_dI"),
                                            int(set_), self._img(out, "out")))
        return out

    def resist_loss(self, aerial, target, params: Params, G=None, stats=None):
        import torch
        shp = (self.n_sets, self.N, self.N)
        if G is None:
            G = torch.empty(shp, dtype=torch.float32, device=self.device)
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.device)
        pc = params.to_c()
        _check(load_library().resist_loss(self._h, _ptr(aerial, torch.float32, shp, "aerial", self.device),
                                          self._img(target, "target", torch.uint8), ctypes.byref(pc),
                                          _ptr(G, torch.float32, shp, "G", self.device),
                                          _ptr(stats, torch.float64, (4,), "stats", self.device)))
        return G, stats

    def levelset_step(self, phi, vel, params: Params, mod=None, stats=None):
        import torch
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.device)
        pc = params.to_c()
        _check(load_library().levelset_step(self._h, self._img(phi, "phi"), self._img(vel, "vel"),
                                            self._img(mod, "mod"), ctypes.byref(pc),
                                            _ptr(stats, torch.float64, (4,), "stats", self.device)))
        return phi, stats

    def edt_reinit(self, params: Params, phi=None, mask=None, phi_out=None, sqdist=None):
        import torch
        if phi_out is None:
            phi_out = torch.empty((self.N, self.N), dtype=torch.float32, device=self.device)
        pc = params.to_c()
        _check(load_library().edt_reinit(self._h, self._img(phi, "phi"), self._img(mask, "mask", torch.uint8),
                                         self._img(phi_out, "phi_out"),
                                         _ptr(sqdist, torch.int32, (2, self.N, self.N), "sqdist", self.device),
                                         ctypes.byref(pc)))
        return phi_out

    def ilt_solve(self, target, phi, params: Params, trace=None, mod=None):
        """The DSO loop in place on phi; mod: optional [N, N] modulation map of
        the curvature term (ilt_solve_modulated)."""
        import torch
        pc = params.to_c()
        rep = _Report()
        tr = None
        if trace is not None:
            tr = _ptr(trace, torch.float64, (params.iters, TRACE_W), "trace", self.device)
        lib = load_library()
        if mod is None:
            rc = lib.ilt_solve(self._h, self._img(target, "target", torch.uint8), self._img(phi, "phi"),
                               ctypes.byref(pc), ctypes.byref(rep), tr)
        else:
            rc = lib.ilt_solve_modulated(self._h, self._img(target, "target", torch.uint8), self._img(phi, "phi"),
                                         self._img(mod, "mod"), ctypes.byref(pc), ctypes.byref(rep), tr)
        _check(rc)
        return dict(iters_done=rep.iters_done, status=rep.status, loss=rep.loss, l2=rep.l2, pvb=rep.pvb,
                    flips=rep.flips)


    # FP64 form (a context created with precision=ILT_FP64)
    def litho_forward_f64(self, mask, set_: int = 0, out=None):
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)
        _check(load_library().litho_forward_f64(self._h, self._img(mask, "mask", torch.float64), int(set_),
                                                self._img(out, "out", torch.float64)))
        return out

    def litho_adjoint_f64(self, mask, dL_dI, set_: int = 0, out=None):
        import torch
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)
        _check(load_library().litho_adjoint_f64(self._h, self._img(mask, "mask", torch.float64),
                                                self._img(dL_dI, "dL_dI", torch.float64), int(set_),
                                                self._img(out, "out", torch.float64)))
        return out

    def ilt_solve_f64(self, target, phi, params: Params, trace=None):
        """The DSO loop in FP64, in place on phi (float64 [N, N])."""
        import torch
        pc = params.to_c()
        rep = _Report()
        tr = None
        if trace is not None:
            tr = _ptr(trace, torch.float64, (params.iters, TRACE_W), "trace", self.device)
        _check(load_library().ilt_solve_f64(self._h, self._img(target, "target", torch.uint8),
                                            self._img(phi, "phi", torch.float64), ctypes.byref(pc),
                                            ctypes.byref(rep), tr))
        return dict(iters_done=rep.iters_done, status=rep.status, loss=rep.loss, l2=rep.l2, pvb=rep.pvb,
                    flips=rep.flips)

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(load_library().ilt_get_tuning(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in _Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _Tuning(**{k: int(v) for k, v in cur.items()})
        _check(load_library().ilt_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, cache_path: str | None = None) -> dict:
        """Time the tuning candidates (or take them from cache_path) and apply
        the fastest; returns the choice, its ms per iteration and whether it
        came from the cache."""
        t = _Tuning()
        ms = ctypes.c_double()
        rc = load_library().ilt_autotune(self._h, None if cache_path is None else cache_path.encode(),
                                         ctypes.byref(t), ctypes.byref(ms))
        if rc < 0:
            _check(rc)
        out = {f: getattr(t, f) for f, _ in _Tuning._fields_}
        out.update(ms_per_iter=ms.value, from_cache=bool(rc == 1))
        return out

    def set_graph(self, enable: bool = True):
        """Capture ilt_solve into a reusable hipGraph (default) or launch directly."""
        _check(load_library().ilt_set_graph(self._h, 1 if enable else 0))

    def profile(self, enable: bool = True):
        """Turn the per-phase HIP-event timing of ilt_solve on or off."""
        _check(load_library().ilt_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{phase: (ms summed over the last ilt_solve, launches)}."""
        buf = (ctypes.c_double * (2 * len(PHASES)))()
        _check(load_library().ilt_profile_read(self._h, buf, len(buf)))
        return {name: (buf[2 * i], int(buf[2 * i + 1])) for i, name in enumerate(PHASES)}


# module-level names matching the C ABI
class Batch:
    """Batched form: ilt_solve over a list of clips of the listed sizes.

    Clip i is (target uint8 [N,N], phi float32 [N,N], Params, trace or None);
    phi is in/out as for ilt_solve.  Results equal per-clip ilt_solve calls.
    """

    def __init__(self, kernels, weights, sizes, max_clips: int = 64, n_lanes: int = 4,
                 precision: int = ILT_FP32, flags: int = 0):
        import torch
        lib = load_library()
        sizes = [int(n) for n in sizes]
        o, _keep, (P, K, ns) = _optics(kernels, weights, sizes[0], precision, flags)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        arr = (ctypes.c_int * len(sizes))(*sizes)
        h = _VP()
        _check(lib.ilt_batch_create(ctypes.byref(h), ctypes.byref(o), arr, len(sizes), int(max_clips),
                                    int(n_lanes), _VP(self.stream.cuda_stream)))
        self._h = h
        self.sizes, self.max_clips, self.n_lanes = sizes, int(max_clips), int(n_lanes)
        self.P, self.K, self.n_sets = P, K, ns
        self._clips = None
        self._clip_key = None

    def close(self):
        if getattr(self, "_h", None):
            load_library().ilt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, enable: bool = True):
        _check(load_library().ilt_batch_set_graph(self._h, 1 if enable else 0))

    def autotune(self, cache_path=None):
        """Clips per chunk and tuning per size (ilt_batch_autotune)."""
        n = len(self.sizes)
        chunk = (ctypes.c_int * n)()
        tun = (_Tuning * n)()
        us = (ctypes.c_double * n)()
        _check(load_library().ilt_batch_autotune(self._h, cache_path.encode() if cache_path else None, chunk, tun,
                                                 us))
        return [dict(N=self.sizes[i], chunk=int(chunk[i]), store_fields=int(tun[i].store_fields),
                     st_xsplit=int(tun[i].st_xsplit), b3_xsplit=int(tun[i].b3_xsplit),
                     xcd_remap=int(tun[i].xcd_remap), us_per_clip_iter=round(float(us[i]), 3)) for i in range(n)]

    def solve(self, clips):
        import torch
        n = len(clips)
        arr = (_Clip * n)()
        for i, (target, phi, params, trace) in enumerate(clips):
            N = int(target.shape[0])
            arr[i].N = N
            arr[i].d_target = _ptr(target, torch.uint8, (N, N), "target[%d]" % i, self.device)
            arr[i].d_phi = _ptr(phi, torch.float32, (N, N), "phi[%d]" % i, self.device)
            arr[i].d_trace = None if trace is None else _ptr(trace, torch.float64, (params.iters, TRACE_W),
                                                             "trace[%d]" % i, self.device)
            arr[i].params = params.to_c()
        reps = (_Report * n)()
        _check(load_library().ilt_solve_batch(self._h, n, arr, reps))
        return [dict(iters_done=r.iters_done, status=r.status, loss=r.loss, l2=r.l2, pvb=r.pvb, flips=r.flips)
                for r in reps]

    def solve_layout(self, layout, N: int, halo: int, params: Params, tile_targets=None, tile_phi=None, out=None):
        """DSO on every N x N tile of a layout (uint8 [H, W]) and the stitched
        phi [H, W]; returns (phi, per-tile reports, tile_phi [T, N, N])."""
        import torch
        H, W = (int(v) for v in layout.shape)
        rows, cols = layout_grid(H, W, N, halo)
        T = rows * cols
        if tile_targets is None:
            tile_targets = torch.empty((T, N, N), dtype=torch.uint8, device=self.device)
        if tile_phi is None:
            tile_phi = torch.empty((T, N, N), dtype=torch.float32, device=self.device)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=self.device)
        reps = (_Report * T)()
        pc = params.to_c()
        _check(load_library().ilt_solve_layout(
            self._h, _ptr(layout, torch.uint8, (H, W), "layout", self.device), H, W, int(N), int(halo),
            ctypes.byref(pc), _ptr(tile_targets, torch.uint8, (T, N, N), "tile_targets", self.device),
            _ptr(tile_phi, torch.float32, (T, N, N), "tile_phi", self.device),
            _ptr(out, torch.float32, (H, W), "out", self.device), reps))
        return out, [dict(iters_done=r.iters_done, status=r.status, loss=r.loss, l2=r.l2, pvb=r.pvb,
                          flips=r.flips) for r in reps], tile_phi


def _stream_of(t):
    import torch
    return _VP(torch.cuda.current_stream(t.device).cuda_stream)


def shifted_heaviside(phi, dh: float, out=None):
    """H(phi + dh) as float32 0/1 of the same shape (H(z) = 1 for z >= 0)."""
    import torch
    if out is None:
        out = torch.empty_like(phi)
    shp = tuple(phi.shape)
    _check(load_library().ilt_shifted_heaviside(_ptr(phi, torch.float32, shp, "phi", phi.device), float(dh),
                                                int(phi.numel()), _ptr(out, torch.float32, shp, "out", phi.device),
                                                _stream_of(phi)))
    return out


def edt_reinit_noalloc(N: int, d_lower: float, d_upper: float, phi=None, mask=None, phi_out=None, sqdist=None):
    """TSDF of [phi <= 0] or of mask (N x N) without a context or any device
    allocation by the library (its scratch is a static device array)."""
    import torch
    src = phi if phi is not None else mask
    if src is None:
        raise ValueError("give phi or mask")
    dev = src.device
    if phi_out is None:
        phi_out = torch.empty((N, N), dtype=torch.float32, device=dev)
    _check(load_library().edt_reinit_noalloc(
        int(N), _ptr(phi, torch.float32, (N, N), "phi", dev), _ptr(mask, torch.uint8, (N, N), "mask", dev),
        float(d_lower), float(d_upper), _ptr(phi_out, torch.float32, (N, N), "phi_out", dev),
        _ptr(sqdist, torch.int32, (2, N, N), "sqdist", dev), _stream_of(phi_out)))
    return phi_out


def epe(target, aerial, i_th: float, pitch_nm: float, sampling=None):
    """Edge placement error of the print [aerial >= i_th] against target
    (both [N, N] on the device): {samples, mean_abs_nm, max_abs_nm,
    over_limit}; sampling: None or (step, end, search, limit) in nm."""
    import torch
    N = int(target.shape[0])
    dev = target.device
    out = torch.zeros(4, dtype=torch.float64, device=dev)
    smp = None if sampling is None else (ctypes.c_float * 4)(*[float(v) for v in sampling])
    _check(load_library().ilt_epe(_ptr(target, torch.uint8, (N, N), "target", dev),
                                  _ptr(aerial, torch.float32, (N, N), "aerial", dev), float(i_th), N,
                                  float(pitch_nm), smp, _ptr(out, torch.float64, (4,), "out", dev),
                                  _stream_of(target)))
    v = out.cpu().tolist()
    return {"samples": int(v[0]), "mean_abs_nm": v[1], "max_abs_nm": v[2], "over_limit": int(v[3])}


def layout_grid(H: int, W: int, N: int, halo: int):
    """(rows, cols) of the tiling of an H x W layout by N x N tiles with
    cores of N - 2 halo pixels."""
    r, c = ctypes.c_int(), ctypes.c_int()
    _check(load_library().ilt_layout_grid(int(H), int(W), int(N), int(halo), ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def layout_extract(layout, N: int, halo: int, out=None):
    """Tiles [rows * cols, N, N] uint8 of a layout uint8 [H, W]."""
    import torch
    H, W = (int(v) for v in layout.shape)
    rows, cols = layout_grid(H, W, N, halo)
    if out is None:
        out = torch.empty((rows * cols, N, N), dtype=torch.uint8, device=layout.device)
    _check(load_library().ilt_layout_extract(_ptr(layout, torch.uint8, (H, W), "layout", layout.device), H, W,
                                             int(N), int(halo),
                                             _ptr(out, torch.uint8, (rows * cols, N, N), "out", layout.device),
                                             _stream_of(layout)))
    return out


def layout_stitch(tiles, H: int, W: int, N: int, halo: int, out=None):
    """Layout [H, W] float32 from the cores of tiles [rows * cols, N, N] float32."""
    import torch
    rows, cols = layout_grid(H, W, N, halo)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=tiles.device)
    _check(load_library().ilt_layout_stitch(_ptr(tiles, torch.float32, (rows * cols, N, N), "tiles", tiles.device),
                                            int(H), int(W), int(N), int(halo),
                                            _ptr(out, torch.float32, (H, W), "out", tiles.device),
                                            _stream_of(tiles)))
    return out


def shot_count(phi=None, mask=None, out=None):
    """Device int64 [3]: rectangles of the row fracturing, of the column
    fracturing, and the smaller (the shot count) of [phi <= 0] or of a
    uint8 mask."""
    import torch
    if (phi is None) == (mask is None):
        raise ValueError("give exactly one of phi and mask")
    t = phi if phi is not None else mask
    H, W = (int(v) for v in t.shape)
    if out is None:
        out = torch.empty(3, dtype=torch.int64, device=t.device)
    _check(load_library().ilt_shot_count(
        None if phi is None else _ptr(phi, torch.float32, (H, W), "phi", t.device),
        None if mask is None else _ptr(mask, torch.uint8, (H, W), "mask", t.device), H, W,
        _ptr(out, torch.int64, (3,), "out", t.device), _stream_of(t)))
    return out


def litho_forward(ctx: Context, mask, set_=0, out=None):
    return ctx.litho_forward(mask, set_, out)


def litho_adjoint(ctx: Context, mask, dL_dI, set_=0, out=None):
    return ctx.litho_adjoint(mask, dL_dI, set_, out)


def resist_loss(ctx: Context, aerial, target, params, G=None, stats=None):
    return ctx.resist_loss(aerial, target, params, G, stats)


def levelset_step(ctx: Context, phi, vel, params, mod=None, stats=None):
    return ctx.levelset_step(phi, vel, params, mod, stats)


def edt_reinit(ctx: Context, params, phi=None, mask=None, phi_out=None, sqdist=None):
    return ctx.edt_reinit(params, phi, mask, phi_out, sqdist)


def ilt_solve(ctx: Context, target, phi, params, trace=None, mod=None):
    return ctx.ilt_solve(target, phi, params, trace, mod)
