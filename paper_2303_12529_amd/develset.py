"""DevelSet: DSN (level-set branch) training data, training and use with DSO.

Sec. III-B trains the network against level-set functions produced by DSO
and Sec. III-C feeds its phi_0 to DSO.  This module drives the library's
entry points for that pipeline; every computation runs in libilt.so.

* `make_dataset`: clips drawn with the 2048^2 recipe, each solved by the
  plain DSO loop from TSDF(target); phi_gt = TSDF(final mask).  The pairs
  are kept on the network grid (4 x 4 means): input and target.
* `train`: Adam with a cosine learning-rate decay over shuffled batches.
* `evaluate`: per clip, the L2 that the plain loop reaches after its
  configured iterations from TSDF(target) is the target; DevelSet starts from
  the network's phi_0 unless the mask of phi_0 prints worse than the target's
  own mask (then it starts from TSDF(target), as the plain loop does), and
  runs DSO until the target L2 is reached.  Times are wall clock with device
  syncs, network inference included.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import dsn as _dsn
from . import ilt as _ilt
from .inputs import C1_CLIP, WORKLOADS, gen_clip, workload_inputs


def make_dataset(n_clips: int, seed0: int, net: "_dsn.Net", precision: int = _ilt.ILT_FP32, log=None):
    """(x, t): device float32 [n, H, W] network inputs and targets."""
    import torch
    _, H, w, prm = workload_inputs("c1", 0)
    N = 2048
    ctx = _ilt.Context(H, w, N, precision=precision)
    ctx.autotune()
    p = _ilt.Params.from_dict(prm, init_mode=0)
    pr = _ilt.Params.from_dict(prm)
    x = torch.empty((n_clips, net.H, net.W), dtype=torch.float32, device="cuda")
    t = torch.empty_like(x)
    tgt = torch.empty((1, N, N), dtype=torch.uint8, device="cuda")
    phi = torch.empty((1, N, N), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for i in range(n_clips):
        Z = gen_clip(C1_CLIP, seed0 + i)
        tgt[0].copy_(torch.as_tensor(Z))
        ctx.ilt_solve(tgt[0], phi[0], p)
        ctx.edt_reinit(pr, phi=phi[0], phi_out=phi[0])        # phi_gt = TSDF([phi_T <= 0])
        xi, ti = net.prepare(tgt, phi)
        x[i].copy_(xi[0])
        t[i].copy_(ti[0])
        if log and (i + 1) % max(1, n_clips // 8) == 0:
            log("dataset %d/%d clips, %.1f s" % (i + 1, n_clips, time.perf_counter() - t0))
    torch.cuda.synchronize()
    ctx.close()
    return x, t


def train(net: "_dsn.Net", x, t, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0, log=None):
    """Adam (0.9, 0.999, 1e-8), lr cosine-decayed to 0 over all steps; returns
    the per-epoch mean loss."""
    import torch
    n = x.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    xb = torch.empty((batch, net.H, net.W), dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(n), device="cuda")
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        for k in range(steps_per_epoch):
            idx = order[k * batch:(k + 1) * batch]
            torch.index_select(x, 0, idx, out=xb)
            torch.index_select(t, 0, idx, out=tb)
            net.forward(xb)
            acc += net.backward(tb)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(total, 1)))
            net.adam_step(cur)
            step += 1
        mean = float(acc.cpu()[0]) / max(steps_per_epoch, 1)
        hist.append(mean)
        if log:
            log("epoch %d/%d loss %.4f (%.1f s)" % (ep + 1, epochs, mean, time.perf_counter() - t0))
    return hist


def evaluate(net: "_dsn.Net", seeds, precision: int = _ilt.ILT_FP32, extra_iters: int = 10, log=None):
    """Time to the plain loop's L2 from TSDF(target) vs from the network's phi_0."""
    import torch
    _, H, w, prm = workload_inputs("c1", 0)
    N = 2048
    ctx = _ilt.Context(H, w, N, precision=precision)
    ctx.autotune()
    T = prm["iters"]
    rows = []
    tgt = torch.empty((1, N, N), dtype=torch.uint8, device="cuda")
    phi = torch.empty((1, N, N), dtype=torch.float32, device="cuda")
    phi0 = torch.empty_like(phi)
    I = torch.empty((ctx.n_sets, N, N), dtype=torch.float32, device="cuda")
    pr = _ilt.Params.from_dict(prm)

    def l2_of(phi_t):
        m = (phi_t <= 0).to(torch.float32)
        for s in range(ctx.n_sets):
            ctx.litho_forward(m, s, out=I[s])
        _, st = ctx.resist_loss(I, tgt[0], pr)
        return int(st.cpu()[1])

    def first_hit(init_mode, phi_init, target_l2):
        tmax = T + extra_iters
        tr = torch.zeros((tmax, _ilt.TRACE_W), dtype=torch.float64, device="cuda")
        phi.copy_(phi_init)
        ctx.ilt_solve(tgt[0], phi[0], _ilt.Params.from_dict(prm, iters=tmax, init_mode=init_mode), trace=tr)
        l2 = tr[:, 2].cpu().numpy()
        hits = np.nonzero(l2 <= target_l2)[0]
        return (int(hits[0]) if len(hits) else None), int(l2[min(T, tmax - 1)])

    for seed in seeds:
        Z = gen_clip(C1_CLIP, seed)
        tgt[0].copy_(torch.as_tensor(Z))
        target_l2 = ctx.ilt_solve(tgt[0], phi[0], _ilt.Params.from_dict(prm, init_mode=0))["l2"]
        # initial masks: the target's own (TSDF) and the network's
        net.predict(tgt, prm["d_lower"], prm["d_upper"], phi0=phi0)
        l2_dsn0 = l2_of(phi0[0])
        ctx.edt_reinit(pr, mask=tgt[0], phi_out=phi[0])
        l2_tsdf0 = l2_of(phi[0])
        use_dsn = l2_dsn0 <= l2_tsdf0
        it_plain, l2T_plain = first_hit(0, phi, target_l2)
        it_dsn, l2T_dsn = first_hit(1, phi0, target_l2) if use_dsn else (it_plain, l2T_plain)
        row = {"seed": seed, "target_l2": int(target_l2), "l2_init_tsdf": l2_tsdf0, "l2_init_dsn": l2_dsn0,
               "dsn_used": bool(use_dsn), "iters_plain": it_plain, "iters_develset": it_dsn,
               "l2_at_T_plain": l2T_plain, "l2_at_T_develset": l2T_dsn}
        # wall time: plain = TSDF init + iterations; DevelSet = inference + iterations
        for name, mode, n_it in (("plain", 0, it_plain), ("develset", 1 if use_dsn else 0, it_dsn)):
            if n_it is None:
                row["ms_" + name] = None
                continue
            pp = _ilt.Params.from_dict(prm, iters=max(n_it, 1), init_mode=mode)
            for rep in range(2):            # the first call captures the solve's graph
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == 1:
                    net.predict(tgt, prm["d_lower"], prm["d_upper"], phi0=phi)
                ctx.ilt_solve(tgt[0], phi[0], pp)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            row["ms_" + name] = round(1e3 * dt, 3)
        rows.append(row)
        if log:
            log("eval seed %d: %s" % (seed, row))
    ctx.close()
    ok = [r for r in rows if r["ms_plain"] and r["ms_develset"]]
    out = {"per_seed": rows,
           "median_ms_plain": float(np.median([r["ms_plain"] for r in ok])) if ok else None,
           "median_ms_develset": float(np.median([r["ms_develset"] for r in ok])) if ok else None,
           "dsn_used": sum(r["dsn_used"] for r in rows)}
    if ok:
        out["speedup"] = round(out["median_ms_plain"] / out["median_ms_develset"], 3)
    return out
