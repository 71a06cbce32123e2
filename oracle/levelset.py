"""Level-set geometry and the DSO evolution step, in float64 (test oracle).

Paper: the mask from the level set, M = 1 where phi <= 0 (Sec. II-A);
the motion equation dphi/dt = -v |grad phi| (Sec. II-A, III-A); the
curvature term lambda m |grad phi| div(grad phi / |grad phi|) (Sec. III-A);
the DSO evolution = motion + curvature; the explicit update
phi_{i+1} = phi_i + dt dphi/dt (Sec. II-A); central differences and the
numeric curvature (Sec. III-A, "Numerical settings"); the CFL time step
dt = eta / max|v| (Sec. III-C).

Readings (the paper leaves these open):
* Descent sign: with M = [phi <= 0] and g = dL/dM, the step that lowers L
  moves phi by +dt * g * |grad phi| (phi rises, the mask shrinks, where
  adding mask would raise L).
* Curvature enters with +dt * lambda * m * K, K = |grad phi| div(n), which is
  mean-curvature flow: convex shapes shrink and corners round.
* Differences are taken with clamp-to-edge (replicated border) samples.
* The curvature denominator is phi_x^2 + phi_y^2 + eps_kappa.
* dt = eta / max|g| (CFL), optionally capped at dt_max; with max|g| = 0 the
  motion term vanishes and dt = dt_max (or no step when uncapped).
"""
from __future__ import annotations

import numpy as np


def mask_from_phi(phi: np.ndarray) -> np.ndarray:
    """M = 1 where phi <= 0, else 0."""
    return (np.asarray(phi) <= 0).astype(np.uint8)


def central_differences(phi: np.ndarray):
    """phi_x, phi_y, phi_xx, phi_yy, phi_xy with replicated borders.

    x is the column index, y the row index (row-major [y][x]).
    """
    p = np.pad(np.asarray(phi, dtype=np.float64), 1, mode="edge")
    c = p[1:-1, 1:-1]
    xp = p[1:-1, 2:]
    xm = p[1:-1, :-2]
    yp = p[2:, 1:-1]
    ym = p[:-2, 1:-1]
    pp = p[2:, 2:]      # (y+1, x+1)
    pm = p[2:, :-2]     # (y+1, x-1)
    mp = p[:-2, 2:]     # (y-1, x+1)
    mm = p[:-2, :-2]    # (y-1, x-1)
    phi_x = 0.5 * (xp - xm)
    phi_y = 0.5 * (yp - ym)
    phi_xx = xp + xm - 2.0 * c
    phi_yy = yp + ym - 2.0 * c
    phi_xy = 0.25 * ((pp - pm) - (mp - mm))
    return phi_x, phi_y, phi_xx, phi_yy, phi_xy


def grad_norm_and_curvature(phi: np.ndarray, eps_kappa: float):
    """|grad phi| and K = (phi_xx phi_y^2 - 2 phi_x phi_y phi_xy + phi_yy phi_x^2)
    / (phi_x^2 + phi_y^2 + eps_kappa)."""
    px, py, pxx, pyy, pxy = central_differences(phi)
    g2 = px * px + py * py
    num = pxx * py * py - 2.0 * px * py * pxy + pyy * px * px
    return np.sqrt(g2), num / (g2 + eps_kappa)


def cfl_dt(g: np.ndarray, eta: float, dt_mode: int, dt_max: float):
    """Time step: fixed eta (dt_mode 1) or eta / max|g| (dt_mode 0, CFL),
    capped at dt_max when dt_max > 0.  Returns (dt, max|g|)."""
    m_v = float(np.max(np.abs(g))) if np.asarray(g).size else 0.0
    if dt_mode == 1:
        return float(eta), m_v
    if m_v > 0.0:
        dt = eta / m_v
        if dt_max > 0.0:
            dt = min(dt, dt_max)
    else:
        dt = dt_max if dt_max > 0.0 else 0.0
    return float(dt), m_v


def levelset_step(phi, g, mod, eta: float, lam: float, eps_kappa: float,
                  dt_mode: int = 0, dt_max: float = 0.0):
    """One DSO evolution step.

    phi' = phi + dt * (g |grad phi| + lam * m * K), m = mod (or 1).
    Returns (phi', dt, max|g|, flips) where flips counts pixels whose mask
    value [phi <= 0] changed.
    """
    phi = np.asarray(phi, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = 1.0 if mod is None else np.asarray(mod, dtype=np.float64)
    dt, m_v = cfl_dt(g, eta, dt_mode, dt_max)
    gn, K = grad_norm_and_curvature(phi, eps_kappa)
    new = phi + dt * (g * gn + lam * m * K)
    flips = int(np.sum((new <= 0) != (phi <= 0)))
    return new, dt, m_v, flips


def cg_direction(g, state):
    """Polak-Ribiere conjugate direction with the non-negative restart (PR+).

    The paper optimises DSO with conjugate gradient (Sec. III-C) without
    naming the variant.  With g the descent velocity of this step (the same
    field plain DSO would use) and the previous step's g and direction kept
    in `state`:
        beta = max(0, <g, g - g_prev> / <g_prev, g_prev>),   d = g + beta d_prev,
    and beta = 0 on the first step.  Inner products in FP64.  Returns (d, beta)
    and updates `state` in place.
    """
    g = np.asarray(g, dtype=np.float64)
    gp = state.get("g_prev")
    beta = 0.0
    if gp is not None:
        den = float(np.sum(gp * gp))
        if den > 0.0:
            beta = max(0.0, float(np.sum(g * (g - gp))) / den)
    d = g if gp is None else g + beta * state["d_prev"]
    state["g_prev"] = g.copy()
    state["d_prev"] = d.copy()
    return d, beta
