"""Python binding of DevelSet-Net (include/dsn.h): the level-set branch and
the optional modulation branch.

Marshalling only: shapes, dtypes and devices are checked here and every
computation runs in the HIP kernels of libilt.so (no fallback).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import ilt as _ilt

DSN_OK = 0
LEVELS = 4
SCALE = 100.0
EPS_AHF = 0.03

_VP = ctypes.c_void_p
_sigs_done = False


def _lib():
    global _sigs_done
    lib = _ilt.load_library()
    if not _sigs_done:
        sig = {
            "dsn_create": [ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           _VP],
            "dsn_destroy": [_VP],
            "dsn_set_params": [_VP, _VP],
            "dsn_get_params": [_VP, _VP],
            "dsn_forward": [_VP, _VP, ctypes.c_int, _VP, _VP],
            "dsn_backward": [_VP, _VP, _VP, ctypes.c_int, _VP, _VP],
            "dsn_adam_step": [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float],
            "dsn_prepare": [_VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP, _VP],
            "dsn_predict": [_VP, _VP, ctypes.c_int, ctypes.c_float, ctypes.c_float, _VP, _VP],
            "dsn_op_conv3x3": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP,
                               ctypes.c_int, ctypes.c_int, _VP, _VP],
            "dsn_op_conv3x3_dgrad": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int,
                                     _VP, _VP, _VP],
            "dsn_op_conv3x3_wgrad": [_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _VP, _VP, _VP],
            "dsn_op_conv_first": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, ctypes.c_int, _VP, _VP],
            "dsn_op_wgrad_first": [_VP, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP],
            "dsn_op_head_bwd": [_VP, ctypes.c_longlong, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP, _VP, _VP,
                                ctypes.c_int, _VP, _VP, _VP, _VP],
            "dsn_op_maxpool2_bwd": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int,
                                    _VP, _VP],
            "dsn_op_upsample2_bwd": [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP],
            "dsn_op_relu_bwd": [_VP, _VP, ctypes.c_longlong, ctypes.c_int, _VP],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.dsn_num_params.argtypes = [_VP]
        lib.dsn_num_params.restype = ctypes.c_longlong
        lib.dsn_last_error.argtypes = []
        lib.dsn_last_error.restype = ctypes.c_char_p
        _sigs_done = True
    return lib


class DsnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("DSN error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != DSN_OK:
        raise DsnError(rc, _lib().dsn_last_error().decode(errors="replace"))


def _ptr(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _VP(t.data_ptr())


def layer_table(base: int = 32, modulation: bool = False):
    """[(name, weight shape, bias shape, weight offset, bias offset)] in the
    flat parameter order of include/dsn.h."""
    ch = [base << i for i in range(LEVELS)]
    rows = []
    prev = 1
    for l in range(LEVELS):
        rows.append(("enc%d_a" % l, (ch[l], 3, 3, prev)))
        rows.append(("enc%d_b" % l, (ch[l], 3, 3, ch[l])))
        prev = ch[l]
    for l in range(LEVELS - 2, -1, -1):
        rows.append(("dec%d_up" % l, (ch[l], 3, 3, ch[l + 1])))
        rows.append(("dec%d_a" % l, (ch[l], 3, 3, 2 * ch[l])))
        rows.append(("dec%d_b" % l, (ch[l], 3, 3, ch[l])))
    rows.append(("head", (1, 1, 1, ch[0])))
    if modulation:
        rows.append(("head_m", (1, 1, 1, ch[0])))
    out = []
    off = 0
    for name, ws in rows:
        nw = int(np.prod(ws))
        out.append((name, ws, (ws[0],), off, off + nw))
        off += nw + ws[0]
    return out


def he_init(seed: int, base: int = 32, modulation: bool = False) -> np.ndarray:
    """Flat FP32 parameters: He-normal weights (std sqrt(2 / fan_in)), zero
    biases.  The modulation head's weights are drawn after all others, so the
    shared layers are the same with and without it."""
    rng = np.random.default_rng(seed)
    tab = layer_table(base, modulation)
    n = tab[-1][4] + tab[-1][2][0]
    flat = np.zeros(n, dtype=np.float32)
    for name, ws, bs, wo, bo in tab:
        fan_in = ws[1] * ws[2] * ws[3]
        flat[wo:bo] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=int(np.prod(ws))).astype(np.float32)
    return flat


class Net:
    """DevelSet-Net on the current device and torch stream; `modulation`
    adds the modulation branch's head."""

    def __init__(self, H: int = 512, W: int = 512, base: int = 32, max_batch: int = 16, modulation: bool = False):
        import torch
        lib = _lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        h = _VP()
        _check(lib.dsn_create(ctypes.byref(h), int(H), int(W), int(base), int(max_batch), int(bool(modulation)),
                              _VP(self.stream.cuda_stream)))
        self._h = h
        self.H, self.W, self.base, self.max_batch = int(H), int(W), int(base), int(max_batch)
        self.modulation = bool(modulation)
        self.n_params = int(lib.dsn_num_params(h))
        self._keep = None
        self.loss_buf = torch.zeros(2, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            _lib().dsn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import torch
        t = torch.as_tensor(flat, dtype=torch.float32).to(self.device).contiguous()
        _check(_lib().dsn_set_params(self._h, _ptr(t, torch.float32, (self.n_params,), "params")))
        torch.cuda.current_stream(self.device).synchronize()

    def get_params(self):
        import torch
        t = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(_lib().dsn_get_params(self._h, _ptr(t, torch.float32, None, "params")))
        return t

    def forward(self, x, out=None, out_m=None):
        """Level-set output [B, H, W]; with the modulation head, the pair
        (out, out_m), out_m being phi_m before the approximated Heaviside."""
        import torch
        B = int(x.shape[0])
        shape = (B, self.H, self.W)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        if self.modulation and out_m is None:
            out_m = torch.empty(shape, dtype=torch.float32, device=self.device)
        _check(_lib().dsn_forward(self._h, _ptr(x, torch.float32, shape, "x"), B, _ptr(out, torch.float32, shape, "out"),
                                  None if out_m is None else _ptr(out_m, torch.float32, shape, "out_m")))
        self._keep = (x, out, out_m)   # read again by backward
        return (out, out_m) if self.modulation else out

    def backward(self, target, grad=None, target_m=None):
        """Returns the device double[2] (L_0, L_m) of the last forward; grad:
        optional FP32 [n_params] out; target_m: modulation targets (L_m is
        left out without them)."""
        import torch
        B = int(target.shape[0])
        shape = (B, self.H, self.W)
        gp = None if grad is None else _ptr(grad, torch.float32, (self.n_params,), "grad")
        _check(_lib().dsn_backward(self._h, _ptr(target, torch.float32, shape, "target"),
                                   None if target_m is None else _ptr(target_m, torch.float32, shape, "target_m"), B,
                                   _ptr(self.loss_buf, torch.float64, (2,), "loss"), gp))
        return self.loss_buf

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(_lib().dsn_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def prepare(self, target, phi_gt=None, m_gt=None):
        """Network-grid input x and, when given the fine-grid phi_gt / m_gt,
        the targets t and t_m; returns (x, t) or, with m_gt, (x, t, t_m)."""
        import torch
        B = int(target.shape[0])
        fine = (B, 4 * self.H, 4 * self.W)
        x = torch.empty((B, self.H, self.W), dtype=torch.float32, device=self.device)
        t = None if phi_gt is None else torch.empty_like(x)
        tm = None if m_gt is None else torch.empty_like(x)
        _check(_lib().dsn_prepare(self._h, _ptr(target, torch.uint8, fine, "target"),
                                  None if phi_gt is None else _ptr(phi_gt, torch.float32, fine, "phi_gt"),
                                  None if m_gt is None else _ptr(m_gt, torch.float32, fine, "m_gt"), B,
                                  _ptr(x, torch.float32, None, "x"),
                                  None if t is None else _ptr(t, torch.float32, None, "t"),
                                  None if tm is None else _ptr(tm, torch.float32, None, "t_m")))
        return (x, t) if m_gt is None else (x, t, tm)

    def predict(self, target, d_lower: float, d_upper: float, phi0=None, m0=None, with_m: bool = False):
        """phi_0 on the fine grid; with `with_m` (or m0 given) also the
        modulation map m_0 and returns (phi0, m0)."""
        import torch
        B = int(target.shape[0])
        fine = (B, 4 * self.H, 4 * self.W)
        if phi0 is None:
            phi0 = torch.empty(fine, dtype=torch.float32, device=self.device)
        with_m = with_m or m0 is not None
        if with_m and m0 is None:
            m0 = torch.empty(fine, dtype=torch.float32, device=self.device)
        _check(_lib().dsn_predict(self._h, _ptr(target, torch.uint8, fine, "target"), B, float(d_lower),
                                  float(d_upper), _ptr(phi0, torch.float32, fine, "phi0"),
                                  _ptr(m0, torch.float32, fine, "m0") if with_m else None))
        return (phi0, m0) if with_m else phi0


# single operations (BF16 channels-last tensors)

def conv3x3(x, w, b=None, relu=False, up=False):
    import torch
    N, Hi, Wi, Cin = x.shape
    Cout = w.shape[0]
    H, W = (2 * Hi, 2 * Wi) if up else (Hi, Wi)
    y = torch.empty((N, H, W, Cout), dtype=torch.bfloat16, device=x.device)
    _check(_lib().dsn_op_conv3x3(_ptr(x, torch.bfloat16, None, "x"), N, H, W, Cin, 1 if up else 0,
                                 _ptr(w, torch.bfloat16, (Cout, 3, 3, Cin), "w"),
                                 None if b is None else _ptr(b, torch.float32, (Cout,), "b"), Cout,
                                 1 if relu else 0, _ptr(y, torch.bfloat16, None, "y"),
                                 _VP(torch.cuda.current_stream().cuda_stream)))
    return y


def conv3x3_dgrad(dy, w, mask=None):
    """Input gradient of a 3x3 convolution; with mask (bf16 [N, H, W, Cin],
    a ReLU output) zeroed where mask <= 0."""
    import torch
    N, H, W, Cout = dy.shape
    Cin = w.shape[3]
    dx = torch.empty((N, H, W, Cin), dtype=torch.bfloat16, device=dy.device)
    _check(_lib().dsn_op_conv3x3_dgrad(_ptr(dy, torch.bfloat16, None, "dy"), N, H, W, Cout,
                                       _ptr(w, torch.bfloat16, (Cout, 3, 3, Cin), "w"), Cin,
                                       None if mask is None else _ptr(mask, torch.bfloat16, (N, H, W, Cin), "mask"),
                                       _ptr(dx, torch.bfloat16, None, "dx"),
                                       _VP(torch.cuda.current_stream().cuda_stream)))
    return dx


def conv3x3_wgrad(dz, x, up=False):
    import torch
    N, H, W, Cout = dz.shape
    Cin = x.shape[3]
    dw = torch.empty((Cout, 3, 3, Cin), dtype=torch.float32, device=dz.device)
    db = torch.empty((Cout,), dtype=torch.float32, device=dz.device)
    _check(_lib().dsn_op_conv3x3_wgrad(_ptr(dz, torch.bfloat16, None, "dz"), _ptr(x, torch.bfloat16, None, "x"),
                                       N, H, W, Cin, 1 if up else 0, Cout, _ptr(dw, torch.float32, None, "dw"),
                                       _ptr(db, torch.float32, None, "db"),
                                       _VP(torch.cuda.current_stream().cuda_stream)))
    return dw, db


def _st():
    import torch
    return _VP(torch.cuda.current_stream().cuda_stream)


def conv_first(x, w, b):
    """First layer: x float32 [N, H, W], w bf16 [Cout, 3, 3, 1], b float32
    [Cout] -> bf16 [N, H, W, Cout] (bias + ReLU)."""
    import torch
    N, H, W = x.shape
    Cout = w.shape[0]
    y = torch.empty((N, H, W, Cout), dtype=torch.bfloat16, device=x.device)
    _check(_lib().dsn_op_conv_first(_ptr(x, torch.float32, (N, H, W), "x"), N, H, W,
                                    _ptr(w, torch.bfloat16, (Cout, 3, 3, 1), "w"),
                                    _ptr(b, torch.float32, (Cout,), "b"), Cout,
                                    _ptr(y, torch.bfloat16, None, "y"), _st()))
    return y


def wgrad_first(dz, x):
    """First layer's (dw float32 [C, 3, 3, 1], db float32 [C]) for dz bf16
    [N, H, W, C] and x float32 [N, H, W]."""
    import torch
    N, H, W, C = dz.shape
    dw = torch.empty((C, 3, 3, 1), dtype=torch.float32, device=dz.device)
    db = torch.empty((C,), dtype=torch.float32, device=dz.device)
    _check(_lib().dsn_op_wgrad_first(_ptr(dz, torch.bfloat16, None, "dz"), _ptr(x, torch.float32, (N, H, W), "x"),
                                     N, H, W, C, _ptr(dw, torch.float32, None, "dw"),
                                     _ptr(db, torch.float32, None, "db"), _st()))
    return dw, db


def head_bwd(x, w, out, t, B, wm=None, out_m=None, t_m=None, relu_mask=False):
    """Head backward: x bf16 [npix, C] features, w (wm) bf16 [C], out / t
    (out_m / t_m) float32 [npix].  Returns (dx bf16 [npix, C], loss float64
    [2], gw float32 [heads, C + 1]); relu_mask zeroes dx where x <= 0."""
    import torch
    npix, C = x.shape
    heads = 2 if wm is not None else 1
    dx = torch.empty_like(x)
    loss = torch.zeros(2, dtype=torch.float64, device=x.device)
    gw = torch.empty((heads, C + 1), dtype=torch.float32, device=x.device)
    f = torch.float32
    _check(_lib().dsn_op_head_bwd(
        _ptr(x, torch.bfloat16, (npix, C), "x"), npix, C, int(B), _ptr(w, torch.bfloat16, (C,), "w"),
        None if wm is None else _ptr(wm, torch.bfloat16, (C,), "wm"), _ptr(out, f, (npix,), "out"),
        None if out_m is None else _ptr(out_m, f, (npix,), "out_m"), _ptr(t, f, (npix,), "t"),
        None if t_m is None else _ptr(t_m, f, (npix,), "t_m"), int(bool(relu_mask)),
        _ptr(dx, torch.bfloat16, None, "dx"),
        _ptr(loss, torch.float64, (2,), "loss"), _ptr(gw, f, None, "gw"), _st()))
    return dx, loss, gw


def maxpool2_bwd(x, dy, dx, relu_mask=False):
    """dx (bf16 [N, H, W, C]) += dy (bf16 [N, H/2, W/2, C]) routed to the first
    maximum of each 2x2 window of x; in place, returns dx.  relu_mask then
    zeroes the windows' elements where x <= 0."""
    import torch
    N, H, W, C = x.shape
    _check(_lib().dsn_op_maxpool2_bwd(_ptr(x, torch.bfloat16, None, "x"), N, H, W, C,
                                      _ptr(dy, torch.bfloat16, (N, H // 2, W // 2, C), "dy"), int(bool(relu_mask)),
                                      _ptr(dx, torch.bfloat16, (N, H, W, C), "dx"), _st()))
    return dx


def upsample2_bwd(dy, mask=None):
    """bf16 [N, H/2, W/2, C]: the sum of each pixel's four children in dy;
    with mask (bf16 [N, H/2, W/2, C], a ReLU output) zeroed where mask <= 0."""
    import torch
    N, H, W, C = dy.shape
    dx = torch.empty((N, H // 2, W // 2, C), dtype=torch.bfloat16, device=dy.device)
    _check(_lib().dsn_op_upsample2_bwd(_ptr(dy, torch.bfloat16, None, "dy"), N, H, W, C,
                                       None if mask is None else _ptr(mask, torch.bfloat16, (N, H // 2, W // 2, C),
                                                                      "mask"),
                                       _ptr(dx, torch.bfloat16, None, "dx"), _st()))
    return dx


def relu_bwd(d, y):
    """d (bf16 [..., C]) *= [y > 0] in place; returns d."""
    import torch
    C = d.shape[-1]
    npix = d.numel() // C
    _check(_lib().dsn_op_relu_bwd(_ptr(d, torch.bfloat16, None, "d"), _ptr(y, torch.bfloat16, tuple(d.shape), "y"),
                                  npix, C, _st()))
    return d
