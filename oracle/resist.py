"""Resist model, DSO objective and print metrics, in float64 (test oracle).

Paper: the sigmoid resist Z = 1 / (1 + exp(-sigma_z (I - I_th))) (Sec. III-A),
L_ilt = sum (Z - Z_t)^2, L_pvb = (Z_in - Z_t)^2 + (Z_out - Z_t)^2,
L_DSO = alpha L_ilt + beta L_pvb (Sec. III-A); the binary print
Z = [I >= I_th] (Sec. II-B, constant-threshold resist); squared L2
||Z - Z_t||^2 and PVBand = XOR area of the two extreme-corner prints
(Sec. II-C).

A process corner is (kernel set s, dose d, loss weight omega).  Dose scales
the intensity linearly (exposure energy): the corner sees d * I_s.
"""
from __future__ import annotations

import numpy as np


def sigmoid_resist(I: np.ndarray, sigma_z: float, i_th: float) -> np.ndarray:
    """Z = 1 / (1 + exp(-sigma_z (I - I_th)))."""
    return 1.0 / (1.0 + np.exp(-sigma_z * (np.asarray(I, dtype=np.float64) - i_th)))


def binary_print(I: np.ndarray, i_th: float) -> np.ndarray:
    """Constant-threshold resist: 1 where I >= I_th (ties print)."""
    return (np.asarray(I, dtype=np.float64) >= i_th).astype(np.uint8)


def dso_loss_and_grad(I_sets, target, corners, sigma_z: float, i_th: float):
    """L = sum_c omega_c sum_p (Z_c - Z_t)^2 and G_s = dL/dI_s per kernel set.

    I_sets: list of aerial images indexed by kernel set; corners: list of
    (set, dose, omega).  Returns (L, [G_s]).

    dZ/dI for the corner is sigma_z d Z (1 - Z), so
    G_s = sum_{c: s_c = s} omega_c 2 sigma_z d_c (Z_c - Z_t) Z_c (1 - Z_c).
    """
    Zt = np.asarray(target, dtype=np.float64)
    G = [np.zeros_like(np.asarray(I, dtype=np.float64)) for I in I_sets]
    L = 0.0
    for (s, d, omega) in corners:
        Z = sigmoid_resist(d * np.asarray(I_sets[s], dtype=np.float64), sigma_z, i_th)
        r = Z - Zt
        L += omega * float(np.sum(r * r))
        G[s] += omega * 2.0 * sigma_z * d * r * Z * (1.0 - Z)
    return L, G


def print_metrics(I_sets, target, corners, i_th: float):
    """(L2, PVB) pixel counts.

    L2 is the squared L2 of the nominal print (corner 0) against the target.
    PVB is the XOR area of the prints at corners 1 and 2 when three corners
    are given (the paper's two extremes), else 0.
    """
    Zt = np.asarray(target).astype(np.uint8)
    s0, d0, _ = corners[0]
    Z0 = binary_print(d0 * np.asarray(I_sets[s0], dtype=np.float64), i_th)
    l2 = int(np.sum(Z0 != Zt))
    pvb = 0
    if len(corners) >= 3:
        s1, d1, _ = corners[1]
        s2, d2, _ = corners[2]
        Z1 = binary_print(d1 * np.asarray(I_sets[s1], dtype=np.float64), i_th)
        Z2 = binary_print(d2 * np.asarray(I_sets[s2], dtype=np.float64), i_th)
        pvb = int(np.sum(Z1 != Z2))
    return l2, pvb
