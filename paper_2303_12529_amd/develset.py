"""DevelSet: DSN training data, training and use with DSO.

Sec. III-B trains the network against level-set functions produced by DSO
(level-set branch) and against the best modulation map of a shift search
(modulation branch); Sec. III-C feeds its phi_0 and m_theta to DSO.  This
module drives the library's entry points for that pipeline; every
computation runs in libilt.so.

* `make_dataset`: clips drawn with the 2048^2 recipe, each solved by the
  plain DSO loop from TSDF(target); phi_gt = TSDF(final mask).  With the
  modulation branch, m_gt = H(phi_gt + dh) for the dh in MOD_SHIFTS whose
  map, used as DSO's modulation map from TSDF(target), reaches the lowest
  final DSO loss.  The pairs are kept on the network grid (4 x 4 means).
* `train`: Adam with a cosine learning-rate decay over shuffled batches, on
  L_0 (+ L_m).
* `evaluate`: per clip, the L2 that the plain loop reaches after its
  configured iterations from TSDF(target) is the target; DevelSet starts from
  the network's phi_0 unless the mask of phi_0 prints worse than the target's
  own mask (then it starts from TSDF(target), as the plain loop does), runs
  DSO (with the network's modulation map when the net has one) until the
  target L2 is reached.  Times are wall clock with device syncs, network
  inference included.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import dsn as _dsn
from . import ilt as _ilt
from .inputs import C1_CLIP, WORKLOADS, gen_clip, workload_inputs

# shifts dh (pixels) of the modulation search: a uniform grid over [-20, 20]
MOD_SHIFTS = tuple(range(-20, 21, 5))


def clip_of_seed(seed: int):
    """The 2048^2 training clip of one seed (a module-level function, so that
    worker processes can draw clips while the device solves)."""
    return gen_clip(C1_CLIP, seed)


def make_dataset(n_clips: int, seed0: int, net: "_dsn.Net", precision: int = _ilt.ILT_FP32, log=None,
                 shifts=MOD_SHIFTS, flags: int = _ilt.ILT_FLAG_GWINDOW_ADJOINT, clips=None):
    """(x, t) or, for a net with the modulation head, (x, t, t_m, dh): device
    float32 [n, H, W] network inputs and targets, and the chosen shift per
    clip (numpy int array).  flags: the solves' context flags (by default
    the G-window adjoint, the fastest exact form of the loop).  clips: an
    optional iterable yielding the targets of seeds seed0, seed0 + 1, ... in
    order (e.g. from a process pool); drawn here otherwise."""
    import torch
    _, H, w, prm = workload_inputs("c1", 0)
    N = 2048
    ctx = _ilt.Context(H, w, N, precision=precision, flags=flags)
    ctx.autotune()
    p = _ilt.Params.from_dict(prm, init_mode=0)
    pr = _ilt.Params.from_dict(prm)
    x = torch.empty((n_clips, net.H, net.W), dtype=torch.float32, device="cuda")
    t = torch.empty_like(x)
    tm = torch.empty_like(x) if net.modulation else None
    dhs = np.zeros(n_clips, dtype=np.int64)
    tgt = torch.empty((1, N, N), dtype=torch.uint8, device="cuda")
    phi = torch.empty((1, N, N), dtype=torch.float32, device="cuda")
    # every solve runs with a modulation map (all ones for the plain loop,
    # which leaves each step unchanged), so one captured graph serves all
    mod = torch.ones((N, N), dtype=torch.float32, device="cuda")
    work = torch.empty((N, N), dtype=torch.float32, device="cuda")
    best = torch.empty((1, N, N), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for i in range(n_clips):
        Z = next(clips) if clips is not None else gen_clip(C1_CLIP, seed0 + i)
        tgt[0].copy_(torch.as_tensor(Z))
        mod.fill_(1.0)
        ctx.ilt_solve(tgt[0], work, p, mod=mod)
        ctx.edt_reinit(pr, phi=work, phi_out=phi[0])          # phi_gt = TSDF([phi_T <= 0])
        if net.modulation:
            best_loss = None
            for dh in shifts:
                _ilt.shifted_heaviside(phi[0], float(dh), out=mod)
                loss = ctx.ilt_solve(tgt[0], work, p, mod=mod)["loss"]
                if best_loss is None or loss < best_loss:
                    best_loss, dhs[i] = loss, dh
                    best[0].copy_(mod)
            xi, ti, tmi = net.prepare(tgt, phi, best)
            tm[i].copy_(tmi[0])
        else:
            xi, ti = net.prepare(tgt, phi)
        x[i].copy_(xi[0])
        t[i].copy_(ti[0])
        if log and (i + 1) % max(1, n_clips // 8) == 0:
            log("dataset %d/%d clips, %.1f s" % (i + 1, n_clips, time.perf_counter() - t0))
    torch.cuda.synchronize()
    ctx.close()
    return (x, t, tm, dhs) if net.modulation else (x, t)


def train(net: "_dsn.Net", x, t, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0, log=None, tm=None):
    """Adam (0.9, 0.999, 1e-8), lr cosine-decayed to 0 over all steps, on
    L_0 (+ L_m when tm is given); returns the per-epoch mean losses
    [L_0, L_m]."""
    import torch
    n = x.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    xb = torch.empty((batch, net.H, net.W), dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    tmb = torch.empty_like(xb) if tm is not None else None
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(n), device="cuda")
        acc = torch.zeros(2, dtype=torch.float64, device="cuda")
        for k in range(steps_per_epoch):
            idx = order[k * batch:(k + 1) * batch]
            torch.index_select(x, 0, idx, out=xb)
            torch.index_select(t, 0, idx, out=tb)
            if tmb is not None:
                torch.index_select(tm, 0, idx, out=tmb)
            net.forward(xb)
            acc += net.backward(tb, target_m=tmb)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(total, 1)))
            net.adam_step(cur)
            step += 1
        mean = [float(v) / max(steps_per_epoch, 1) for v in acc.cpu()]
        hist.append(mean)
        if log:
            log("epoch %d/%d L0 %.4f Lm %.4f (%.1f s)" % (ep + 1, epochs, mean[0], mean[1],
                                                          time.perf_counter() - t0))
    return hist


def evaluate(net: "_dsn.Net", seeds, precision: int = _ilt.ILT_FP32, extra_iters: int = 10, log=None,
             flags: int = 0, overrides: dict | None = None):
    """Time to the plain loop's L2 from TSDF(target) vs from the network's
    phi_0, with the loop in the given precision and context flags;
    overrides: loop settings that replace the 2048^2 workload's (e.g. the
    curvature weight)."""
    import torch
    _, H, w, prm = workload_inputs("c1", 0)
    if overrides:
        prm = dict(prm, **overrides)
    N = 2048
    ctx = _ilt.Context(H, w, N, precision=precision, flags=flags)
    ctx.autotune()
    T = prm["iters"]
    rows = []
    tgt = torch.empty((1, N, N), dtype=torch.uint8, device="cuda")
    phi = torch.empty((1, N, N), dtype=torch.float32, device="cuda")
    phi0 = torch.empty_like(phi)
    m0 = torch.empty_like(phi) if net.modulation else None
    m_run = torch.empty_like(phi) if net.modulation else None
    I = torch.empty((ctx.n_sets, N, N), dtype=torch.float32, device="cuda")
    pr = _ilt.Params.from_dict(prm)

    def l2_of(phi_t):
        for s in range(ctx.n_sets):
            ctx.litho_forward_phi(phi_t, s, out=I[s])
        _, st = ctx.resist_loss(I, tgt[0], pr)
        return int(st.cpu()[1])

    def first_hit(init_mode, phi_init, target_l2, mod=None):
        tmax = T + extra_iters
        tr = torch.zeros((tmax, _ilt.TRACE_W), dtype=torch.float64, device="cuda")
        phi.copy_(phi_init)
        ctx.ilt_solve(tgt[0], phi[0], _ilt.Params.from_dict(prm, iters=tmax, init_mode=init_mode), trace=tr,
                      mod=mod)
        l2 = tr[:, 2].cpu().numpy()
        hits = np.nonzero(l2 <= target_l2)[0]
        return (int(hits[0]) if len(hits) else None), int(l2[min(T, tmax - 1)])

    for seed in seeds:
        Z = gen_clip(C1_CLIP, seed)
        tgt[0].copy_(torch.as_tensor(Z))
        target_l2 = ctx.ilt_solve(tgt[0], phi[0], _ilt.Params.from_dict(prm, init_mode=0))["l2"]
        # initial masks: the target's own (TSDF) and the network's
        net.predict(tgt, prm["d_lower"], prm["d_upper"], phi0=phi0, m0=m0)
        l2_dsn0 = l2_of(phi0[0])
        ctx.edt_reinit(pr, mask=tgt[0], phi_out=phi[0])
        l2_tsdf0 = l2_of(phi[0])
        use_dsn = l2_dsn0 <= l2_tsdf0
        it_plain, l2T_plain = first_hit(0, phi, target_l2)
        it_dsn, l2T_dsn = first_hit(1, phi0, target_l2) if use_dsn else (it_plain, l2T_plain)
        row = {"seed": seed, "target_l2": int(target_l2), "l2_init_tsdf": l2_tsdf0, "l2_init_dsn": l2_dsn0,
               "dsn_used": bool(use_dsn), "iters_plain": it_plain, "iters_develset": it_dsn,
               "l2_at_T_plain": l2T_plain, "l2_at_T_develset": l2T_dsn}
        variants = [("plain", 0, it_plain, False), ("develset", 1 if use_dsn else 0, it_dsn, False)]
        if net.modulation:
            # the network's phi_0 (same fallback rule) and its modulation map
            it_m, l2T_m = first_hit(1 if use_dsn else 0, phi0 if use_dsn else phi, target_l2, mod=m0[0])
            row.update(iters_develset_m=it_m, l2_at_T_develset_m=l2T_m,
                       m0_mean=round(float(m0.mean()), 4))
            variants.append(("develset_m", 1 if use_dsn else 0, it_m, True))
        # wall time: plain = TSDF init + iterations; DevelSet = inference + iterations
        for name, mode, n_it, with_m in variants:
            if n_it is None:
                row["ms_" + name] = None
                continue
            pp = _ilt.Params.from_dict(prm, iters=max(n_it, 1), init_mode=mode)
            for rep in range(2):            # the first call captures the solve's graph
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == 1 or with_m:
                    net.predict(tgt, prm["d_lower"], prm["d_upper"], phi0=phi, m0=m_run if with_m else None)
                ctx.ilt_solve(tgt[0], phi[0], pp, mod=m_run[0] if with_m else None)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            row["ms_" + name] = round(1e3 * dt, 3)
            # the mask at the hit: edge placement error of its nominal print
            ctx.litho_forward_phi(phi[0], 0, out=I[0])
            row["epe_" + name] = round(_ilt.epe(tgt[0], I[0], prm["i_th"], C1_CLIP.pitch_nm)["mean_abs_nm"], 3)
        rows.append(row)
        if log:
            log("eval seed %d: %s" % (seed, row))
    ctx.close()
    ok = [r for r in rows if r["ms_plain"] and r["ms_develset"]]
    out = {"per_seed": rows,
           "median_ms_plain": float(np.median([r["ms_plain"] for r in ok])) if ok else None,
           "median_ms_develset": float(np.median([r["ms_develset"] for r in ok])) if ok else None,
           "median_epe_nm_plain": float(np.median([r["epe_plain"] for r in ok])) if ok else None,
           "median_epe_nm_develset": float(np.median([r["epe_develset"] for r in ok])) if ok else None,
           "dsn_used": sum(r["dsn_used"] for r in rows)}
    if ok:
        out["speedup"] = round(out["median_ms_plain"] / out["median_ms_develset"], 3)
    if net.modulation:
        okm = [r for r in rows if r["ms_plain"] and r.get("ms_develset_m")]
        out["median_ms_develset_m"] = float(np.median([r["ms_develset_m"] for r in okm])) if okm else None
        out["median_epe_nm_develset_m"] = float(np.median([r["epe_develset_m"] for r in okm])) if okm else None
        out["reached_develset_m"] = len(okm)
        if okm:
            out["speedup_m"] = round(float(np.median([r["ms_plain"] for r in okm])) / out["median_ms_develset_m"], 3)
    return out
