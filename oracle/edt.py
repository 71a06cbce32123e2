"""Exact squared EDT and the truncated signed distance function (test oracle).

Paper: the signed distance function (Sec. II-A: negative inside the curve,
positive outside, magnitude = distance to the curve), its truncation to
[D_l, D_u] (Sec. III-A, TSDF equation; D_u = 900, D_l = -100 nm), and the
CUDA_TSDF routine of Alg. 1, whose boundary is found by shift-and-XOR.

Reading of "distance to the curve" on a pixel grid: the squared distance
between pixel centres to the nearest pixel of the opposite class, with a
half-pixel shift so that the zero crossing lies on the pixel edge:
    outside (M = 0):  phi = sqrt(D_in)  - 1/2,  D_in  = min over inside  q |p-q|^2
    inside  (M = 1):  phi = 1/2 - sqrt(D_out),  D_out = min over outside q |p-q|^2
then clipped to [d_lower, d_upper] (pixel units).  [phi <= 0] = M exactly,
so re-initialisation never moves the boundary.  A class that is absent
leaves the other class at its clip bound.

The transform itself is plain C (``edt.c``), compiled with gcc on first use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "edt.c")
_LIB = os.path.join(_HERE, "_oracle_edt.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C transform into a shared object next to this file."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_sqedt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_sqedt.restype = ctypes.c_int
        _lib = lib
    return _lib


def sqedt(cls: np.ndarray, want: int) -> np.ndarray:
    """Squared distance from every pixel to the nearest pixel with cls == want
    (int64; -1 where no such pixel exists)."""
    cls = np.ascontiguousarray(np.asarray(cls), dtype=np.uint8)
    if cls.ndim != 2 or cls.shape[0] != cls.shape[1]:
        raise ValueError("square 2-D mask expected")
    N = cls.shape[0]
    out = np.empty((N, N), dtype=np.int64)
    rc = _load().oracle_sqedt(cls.ctypes.data, N, int(want), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_sqedt failed (%d)" % rc)
    return out


def sqdist_in_out(mask: np.ndarray):
    """(D_in, D_out): squared distance to the nearest inside (M = 1) pixel and
    to the nearest outside (M = 0) pixel, for every pixel."""
    m = (np.asarray(mask) != 0).astype(np.uint8)
    return sqedt(m, 1), sqedt(m, 0)


def tsdf_from_mask(mask: np.ndarray, d_lower: float, d_upper: float):
    """Truncated signed distance (pixels) of a binary mask; float64.

    Returns (phi, D_in, D_out).
    """
    m = (np.asarray(mask) != 0)
    d_in, d_out = sqdist_in_out(m)
    phi = np.empty(m.shape, dtype=np.float64)
    out = ~m
    ins = m
    # outside pixels: distance to the nearest inside pixel
    din = d_in[out]
    phi[out] = np.where(din >= 0, np.sqrt(np.maximum(din, 0).astype(np.float64)) - 0.5, d_upper)
    dout = d_out[ins]
    phi[ins] = np.where(dout >= 0, 0.5 - np.sqrt(np.maximum(dout, 0).astype(np.float64)), d_lower)
    phi = np.clip(phi, d_lower, d_upper)
    return phi, d_in, d_out


def tsdf_from_phi(phi: np.ndarray, d_lower: float, d_upper: float):
    """Re-initialisation: TSDF of the mask [phi <= 0]."""
    return tsdf_from_mask(np.asarray(phi) <= 0, d_lower, d_upper)
