"""The plain DSO loop, in float64 (test oracle).

Paper: DSO (Sec. III-A/B): start from the TSDF of the target (Alg. 1,
CUDA_TSDF), then repeat forward lithography -> L_DSO -> velocity
v = alpha dL_ilt/dM + beta dL_pvb/dM -> geometry gradient and curvature ->
explicit step with the CFL time step (Sec. III-C).  Periodic
re-initialisation to the TSDF keeps phi a distance function.

``params`` is a plain dict:
  iters, reinit_every, dt_mode (0 CFL, 1 fixed), eta, dt_max, lam, sigma_z,
  i_th, eps_kappa, d_lower, d_upper, corners = [(set, dose, omega), ...].
"""
from __future__ import annotations

import numpy as np

from . import edt, levelset, litho, resist


def sets_used(corners):
    return sorted({int(c[0]) for c in corners})


def forward_all(M, kernels, weights, corners):
    """Aerial images for every kernel set a corner uses (None elsewhere)."""
    I = [None] * kernels.shape[0]
    for s in sets_used(corners):
        I[s] = litho.aerial_image(M, kernels[s], weights[s])
    return I


def iteration(phi, target, kernels, weights, params, state=None, mod=None):
    """One DSO iteration before re-initialisation.

    params["optimizer"] = 1 moves phi along the conjugate direction of
    levelset.cg_direction (Sec. III-C) instead of the gradient itself; its
    state (previous gradient and direction) lives in `state` across calls.
    mod: the modulation map m of the curvature term (Sec. III-C), None = 1.
    Returns (phi', row) with row = dict(loss, l2, pvb, flips, m_v, dt, beta).
    """
    corners = params["corners"]
    M = levelset.mask_from_phi(phi)
    I = forward_all(M, kernels, weights, corners)
    L, G = resist.dso_loss_and_grad(I, target, corners, params["sigma_z"], params["i_th"])
    l2, pvb = resist.print_metrics(I, target, corners, params["i_th"])
    g = np.zeros(phi.shape)
    for s in sets_used(corners):
        g += litho.litho_adjoint(M, G[s], kernels[s], weights[s])
    beta = 0.0
    if params.get("optimizer", 0) == 1:
        g, beta = levelset.cg_direction(g, state if state is not None else {})
    new, dt, m_v, flips = levelset.levelset_step(
        phi, g, mod, params["eta"], params["lam"], params["eps_kappa"],
        params.get("dt_mode", 0), params.get("dt_max", 0.0))
    return new, dict(loss=L, l2=l2, pvb=pvb, flips=flips, m_v=m_v, dt=dt, beta=beta)


def ilt_solve(target, kernels, weights, params, phi0=None, mod=None):
    """Run params['iters'] DSO iterations (curvature term weighted by `mod`
    when given); returns (phi_T, trace, final).

    final = dict(l2, pvb, loss) of the mask [phi_T <= 0].
    """
    target = np.asarray(target).astype(np.uint8)
    if phi0 is None:
        phi, _, _ = edt.tsdf_from_mask(target, params["d_lower"], params["d_upper"])
    else:
        phi = np.asarray(phi0, dtype=np.float64).copy()
    trace = []
    state = {}
    R = int(params.get("reinit_every", 0))
    for i in range(int(params["iters"])):
        phi, row = iteration(phi, target, kernels, weights, params, state, mod)
        if R > 0 and (i + 1) % R == 0:
            phi, _, _ = edt.tsdf_from_phi(phi, params["d_lower"], params["d_upper"])
        row["i"] = i
        trace.append(row)
    M = levelset.mask_from_phi(phi)
    I = forward_all(M, kernels, weights, params["corners"])
    L, _ = resist.dso_loss_and_grad(I, target, params["corners"], params["sigma_z"], params["i_th"])
    l2, pvb = resist.print_metrics(I, target, params["corners"], params["i_th"])
    return phi, trace, dict(l2=l2, pvb=pvb, loss=L)
