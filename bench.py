#!/usr/bin/env python3
"""Throughput of the level-set ILT loop on one MI355X.

A step is one DSO iteration over one synthetic 2048 x 2048 clip (1 nm
pixels): mask spectrum, SOCS forward imaging with K = 24 kernels for two
focus conditions, resist and L_DSO over three process corners, the SOCS
adjoint, the gradient back-transform, the curvature-regularised level-set
step, and TSDF re-initialisation every 5 steps.  Inputs are resident in HBM
before timing starts.

Output: one JSON line (rank 0) with the metric, a roofline entry for the
dominant kernel (timed with HIP events on the library's stream inside the
timed region) and the CPU FP64 oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "level-set ILT iterations/s per 2048² clip (K=24); time-to-L2 target vs plain"
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0


def algorithmic_work(N, P, K, n_sets):
    """Per-phase algorithmic flops (dense phases) and bytes (pixel phases)
    of one iteration; complex multiply-add = 8 flops."""
    N2 = float(N) * N
    return {
        "spectrum": dict(flops=4 * P * N2 + 8 * P * P * N),
        "window_rows": dict(flops=n_sets * K * 8.0 * P * P * N),
        "image": dict(flops=n_sets * K * 8.0 * P * N2),
        "adjoint": dict(flops=n_sets * K * (8.0 * P * N2 + 8.0 * P * P * N)),
        "gradient": dict(flops=4 * P * N2 + 8 * P * P * N),
        "resist": dict(bytes=N2 * (4 * n_sets + 1 + 4 * n_sets)),
        "levelset_step": dict(bytes=N2 * 12),
        "reinit": dict(bytes=N2 * 16),
    }


# Dominant-kernel names and the sources they are built from, per (phase, dtype);
# the HBM traffic measured with hardware counters is used only while those
# sources are unchanged since the measurement.
KERNELS = {
    ("adjoint", "f32"): ("k_adjoint_st", ("k_litho.hip", "ilt_device.h", "ilt_internal.h")),
    ("adjoint", "bf16x3"): ("k_adjoint_b3", ("k_bf16.hip", "ilt_device.h", "ilt_internal.h")),
    ("image", "f32"): ("k_image", ("k_litho.hip", "ilt_internal.h")),
    ("image", "bf16x3"): ("k_image_b3", ("k_bf16.hip", "ilt_internal.h")),
}
HERE = os.path.dirname(os.path.abspath(__file__))


def sources_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "paper_2303_12529_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, dtype, files):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>_<dtype>_traffic.md, or None if absent or stale."""
    path = os.path.join(HERE, "profiles", "%s_%s_traffic.md" % (kernel, dtype))
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources sha256/16") != sources_digest(files):
        return None, "stale"
    try:
        return float(vals["hbm bytes per launch"]), os.path.relpath(path, HERE)
    except (KeyError, ValueError):
        return None, None


def issued_bf16_flops(N, P, K, n_sets, phase):
    """Matrix-core flops the split-BF16 kernels issue per launch (padding and
    the three hi/lo products included)."""
    kp = 8 if 2 * P <= 8 else 24 if 2 * P <= 24 else 40 if 2 * P <= 40 else 72
    kc = (3 * kp + 31) // 32 * 32
    fb, mix = P // 16, int(P % 16 != 0 and P % 16 <= 8)
    if P % 16 > 8:
        fb += 1
    nz = 32 * fb + 16 * mix
    npad = (N + 127) // 128 * 128
    pix = float(npad) * ((N + 31) // 32 * 32)
    if phase == "adjoint":
        return n_sets * K * pix * (2 * kc * 2 + 2 * nz * 3 * 2)
    if phase == "image":
        return n_sets * K * float(npad) * npad * 2 * kc * 2
    return None


def gwindow_work(N, P, K, n_sets):
    """Algorithmic flops of one iteration with the G-window adjoint: the
    adjoint becomes one pruned (2P-1)^2 transform of G per set plus the
    window correlation."""
    Q = 2 * P - 1
    N2 = float(N) * N
    w = algorithmic_work(N, P, K, n_sets)
    w["adjoint"] = dict(flops=n_sets * (4.0 * Q * N2 + 8.0 * Q * Q * N) + n_sets * K * 8.0 * P ** 4)
    return w


def hopkins_work(N, P, K, n_sets):
    """Algorithmic flops of one iteration with the TCC-form image and the
    G-window adjoint: the image spectrum on the difference window (sum over
    D of the window overlap is P^4 per kernel), its window rows and one
    pruned inverse transform per set, instead of K field transforms."""
    Q = 2 * P - 1
    N2 = float(N) * N
    w = gwindow_work(N, P, K, n_sets)
    w["window_rows"] = dict(flops=n_sets * K * 8.0 * P ** 4)
    w["image"] = dict(flops=n_sets * (4.0 * Q * N2 + 8.0 * Q * Q * N))
    return w


def gwindow_forms(Z, H, w, N, prm, steps, autotune):
    """The loop with the G-window adjoint, in both precisions (its own cost
    model, so its own figures)."""
    import torch
    from paper_2303_12529_amd import ilt
    n_sets, K, P, _ = H.shape
    target = torch.as_tensor(Z).to("cuda")
    out = {"note": "adjoint by the G-window identity (exact): one (2P-1)^2 pruned transform of G per set "
                   "plus a window correlation, instead of K field transforms; no field store; fp32_hopkins: "
                   "the image as well through its (2P-1)^2 spectrum (TCC form, exact), no field at all"}
    gw, hop = ilt.ILT_FLAG_GWINDOW_ADJOINT, ilt.ILT_FLAG_HOPKINS_FORWARD
    for name, prec, flags in (("fp32", ilt.ILT_FP32, gw), ("bf16x3", ilt.ILT_BF16X3, gw),
                              ("fp32_hopkins", ilt.ILT_FP32, gw | hop)):
        work = (hopkins_work if flags & hop else gwindow_work)(N, P, K, n_sets)
        total = sum(v.get("flops", 0.0) for v in work.values())
        ctx = ilt.Context(H, w, N, precision=prec, flags=flags)
        if autotune:
            ctx.autotune()
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        ctx.ilt_solve(target, phi, ilt.Params.from_dict(prm, iters=5, init_mode=0))
        p = ilt.Params.from_dict(prm, iters=steps, init_mode=1)
        start = phi.clone()
        ctx.ilt_solve(target, phi, p)
        phi.copy_(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.ilt_solve(target, phi, p)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phi.copy_(start)
        ctx.profile(True)
        ctx.ilt_solve(target, phi, p)
        prof = ctx.profile_read()
        ctx.profile(False)
        out[name] = {"value": round(steps / wall, 3), "unit": "it/s", "ms_per_step": round(1e3 * wall / steps, 4),
                     "algorithmic_tflops": round(total * steps / wall / 1e12, 2),
                     "phases_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items()},
                     "final_l2": rep["l2"]}
        ctx.close()
    return out


def cpu_model():
    """The host CPU's model name (first /proc/cpuinfo entry) and logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def _oracle_iters(workload, seed, iters):
    """Wall time of `iters` oracle iterations from TSDF(target) (the TSDF
    itself untimed)."""
    from oracle import edt as o_edt
    from oracle import solve as o_solve
    from paper_2303_12529_amd.inputs import workload_inputs
    Z, H, w, prm = workload_inputs(workload, seed)
    phi, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    t0 = time.perf_counter()
    for _ in range(iters):
        phi, _ = o_solve.iteration(phi, Z, H, w, prm)
    return time.perf_counter() - t0


def cpu_baseline(workload, seed, iters, iters_1t=1, c0_iters=20):
    """The FP64 oracle on the host cores: `iters` iterations of the timed
    workload with the BLAS threads it finds (the reported value), the same
    with one thread, and the 256^2 workload's whole loop."""
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    dt = _oracle_iters(workload, seed, iters)
    model, ncpu = cpu_model()
    out = {"value": iters / dt, "unit": "it/s", "cores": int(threads), "kind": "oracle",
           "sample": "%d DSO iterations of the same %s clip (seed %d), FP64 numpy/BLAS on %d threads, %.1f s"
                     % (iters, workload, seed, threads, dt),
           "cpu_model": model, "logical_cpus": ncpu}
    with threadpool_limits(limits=1):
        if iters_1t > 0:
            d1 = _oracle_iters(workload, seed, iters_1t)
            out["one_thread"] = {"value": iters_1t / d1, "unit": "it/s", "cores": 1,
                                 "sample": "%d iteration(s), %.1f s" % (iters_1t, d1)}
    if c0_iters > 0 and workload != "c0":
        d0 = _oracle_iters("c0", seed, c0_iters)
        out["c0_whole_loop"] = {"value": c0_iters / d0, "unit": "it/s", "cores": int(threads),
                                "s": round(d0, 3),
                                "sample": "the 256^2 workload's %d iterations (seed %d)" % (c0_iters, seed)}
    return out


def time_to_target(ctxs, workload, seeds, extra_iters=10):
    """Time for each form to reach the L2 that the plain FP32 loop reaches
    after its configured number of iterations from TSDF(target), per seed.

    A form's time is the wall time of one solve (TSDF init included) that
    stops at the first iteration whose printed mask has L2 <= the target;
    that iteration count is read from a longer traced run of the same form.
    """
    import numpy as np
    import torch
    from paper_2303_12529_amd import ilt
    from paper_2303_12529_amd.inputs import workload_inputs
    per_seed = []
    for seed in seeds:
        Z, _, _, prm = workload_inputs(workload, seed)
        N = Z.shape[0]
        T = prm["iters"]
        tgt = torch.as_tensor(Z).to("cuda")
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        target_l2 = ctxs["fp32"].ilt_solve(tgt, phi, ilt.Params.from_dict(prm, iters=T, init_mode=0))["l2"]
        row = {"seed": seed, "target_l2": int(target_l2)}
        forms = [(name, ctx, 0) for name, ctx in ctxs.items()] + [("fp32_cg", ctxs["fp32"], 1)]
        for name, ctx, opt in forms:
            tmax = T + extra_iters
            tr = torch.zeros((tmax, ilt.TRACE_W), dtype=torch.float64, device="cuda")
            ctx.ilt_solve(tgt, phi, ilt.Params.from_dict(prm, iters=tmax, init_mode=0, optimizer=opt), trace=tr)
            l2 = tr[:, 2].cpu().numpy()
            hits = np.nonzero(l2 <= target_l2)[0]
            hits = hits[hits > 0]
            if len(hits) == 0:
                row[name] = None
                continue
            n_it = int(hits[0])
            p = ilt.Params.from_dict(prm, iters=n_it, init_mode=0, optimizer=opt)
            ctx.ilt_solve(tgt, phi, p)          # captures this solve's graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.ilt_solve(tgt, phi, p)
            torch.cuda.synchronize()
            ms = round(1e3 * (time.perf_counter() - t0), 3)
            # the mask at the hit: edge placement error of its nominal print
            aerial = ctx.litho_forward_phi(phi, 0)
            e = ilt.epe(tgt, aerial, prm["i_th"], 2048.0 / N)
            row[name] = {"iters": n_it, "ms": ms, "l2_at_T": int(l2[T]) if T < tmax else None,
                         "epe_nm_at_hit": round(e["mean_abs_nm"], 3)}
        per_seed.append(row)
    out = {"target": "L2 of the plain FP32 loop after its configured iterations from TSDF(target)",
           "seeds": list(seeds), "per_seed": per_seed, "median_ms": {}}
    out["median_epe_nm_at_hit"] = {}
    for name in list(ctxs) + ["fp32_cg"]:
        ms = [r[name]["ms"] for r in per_seed if r.get(name)]
        out["median_ms"][name] = round(float(np.median(ms)), 3) if len(ms) == len(per_seed) else None
        ep = [r[name]["epe_nm_at_hit"] for r in per_seed if r.get(name)]
        out["median_epe_nm_at_hit"][name] = round(float(np.median(ep)), 3) if ep else None
    for name in ctxs:
        if name != "fp32" and out["median_ms"].get("fp32") and out["median_ms"].get(name):
            out["%s_speedup_vs_plain" % name] = round(out["median_ms"]["fp32"] / out["median_ms"][name], 3)
    return out


DSN_WEIGHTS = os.path.join(HERE, "paper_2303_12529_amd", "weights", "dsn_c1_fp16.npy")
DSN_MOD_WEIGHTS = os.path.join(HERE, "paper_2303_12529_amd", "weights", "dsn_c1_mod_fp16.npy")


def develset_ttt(seeds, wide_seeds=None):
    """Time to the plain loop's L2 with the trained network's phi_0 (DevelSet,
    Sec. III-C) vs from TSDF(target): the level-set-branch network with the
    loop in FP32 (on wide_seeds when given), FP32 with the G-window adjoint,
    BF16x3, and BF16x3 with the G-window adjoint, and the two-branch network
    (level set + modulation, whose m_theta weights every step's curvature
    term) on the FP32 loop."""
    import numpy as np
    from paper_2303_12529_amd import develset, dsn
    from paper_2303_12529_amd import ilt
    out = {}
    gw = ilt.ILT_FLAG_GWINDOW_ADJOINT
    hop = gw | ilt.ILT_FLAG_HOPKINS_FORWARD
    runs = [("weights", DSN_WEIGHTS, (("fp32", ilt.ILT_FP32, 0), ("fp32_gwindow", ilt.ILT_FP32, gw),
                                      ("bf16x3", ilt.ILT_BF16X3, 0), ("bf16x3_gwindow", ilt.ILT_BF16X3, gw),
                                      ("fp32_hopkins", ilt.ILT_FP32, hop))),
            ("modulation_net", DSN_MOD_WEIGHTS, (("fp32", ilt.ILT_FP32, 0),))]
    for label, path, forms in runs:
        if not os.path.exists(path):
            continue
        flat = np.load(path, allow_pickle=False).astype(np.float32)
        # the modulation branch adds one 1x1 head (32 weights and a bias)
        modulation = flat.size == dsn.layer_table(32, True)[-1][4] + 1
        net = dsn.Net(512, 512, 32, max_batch=1, modulation=modulation)
        net.set_params(flat)
        res = {"weights": os.path.relpath(path, HERE), "modulation": modulation}
        for name, prec, flags in forms:
            sd = wide_seeds if (wide_seeds is not None and label == "weights" and name == "fp32") else seeds
            ev = develset.evaluate(net, sd, precision=prec, flags=flags)
            r = {"seeds": "%d-%d" % (min(sd), max(sd)),
                 "median_ms_plain": ev["median_ms_plain"], "median_ms_develset": ev["median_ms_develset"],
                 "speedup": ev.get("speedup"), "dsn_used": ev["dsn_used"],
                 "median_epe_nm_at_hit": {"plain": ev["median_epe_nm_plain"], "develset": ev["median_epe_nm_develset"],
                                          "develset_m": ev.get("median_epe_nm_develset_m")},
                 "iters_develset": [x["iters_develset"] for x in ev["per_seed"]],
                 "l2_at_T_plain": [x["l2_at_T_plain"] for x in ev["per_seed"]],
                 "l2_at_T_develset": [x["l2_at_T_develset"] for x in ev["per_seed"]]}
            if modulation:
                r.update(median_ms_develset_m=ev.get("median_ms_develset_m"), speedup_m=ev.get("speedup_m"),
                         iters_develset_m=[x["iters_develset_m"] for x in ev["per_seed"]],
                         l2_at_T_develset_m=[x["l2_at_T_develset_m"] for x in ev["per_seed"]])
            res[name] = r
        if modulation:
            # the paper's own curvature weight (lambda = 0.9, eta = 0.85; the
            # CFL cap of the curvature term scaled with it): where curvature
            # drives the loop, what the modulation map gains
            ov = {"eta": 0.85, "lam": 0.9, "dt_max": 0.25 / 0.9}
            ev = develset.evaluate(net, seeds, precision=ilt.ILT_FP32, overrides=ov)
            res["fp32_lambda_0.9"] = {
                "settings": ov, "median_ms_plain": ev["median_ms_plain"],
                "median_epe_nm_at_hit": {"plain": ev["median_epe_nm_plain"], "develset": ev["median_epe_nm_develset"],
                                         "develset_m": ev.get("median_epe_nm_develset_m")},
                "median_ms_develset": ev["median_ms_develset"], "speedup": ev.get("speedup"),
                "median_ms_develset_m": ev.get("median_ms_develset_m"), "speedup_m": ev.get("speedup_m"),
                "dsn_used": ev["dsn_used"],
                "iters_plain": [x["iters_plain"] for x in ev["per_seed"]],
                "iters_develset": [x["iters_develset"] for x in ev["per_seed"]],
                "iters_develset_m": [x["iters_develset_m"] for x in ev["per_seed"]],
                "l2_at_T_plain": [x["l2_at_T_plain"] for x in ev["per_seed"]],
                "l2_at_T_develset": [x["l2_at_T_develset"] for x in ev["per_seed"]],
                "l2_at_T_develset_m": [x["l2_at_T_develset_m"] for x in ev["per_seed"]]}
        net.close()
        if label == "weights":
            out.update(res)
        else:
            out[label] = res
    return out or None


def batched(n_clips, lanes, precision):
    """Batched form on n_clips synthetic clips (N uniform over 512/1024/2048,
    one 2048 nm field): one ilt_solve_batch of the full 50-iteration loop per
    clip (TSDF init included) on `lanes` streams, against the same clips on
    one lane (clips strictly one after another)."""
    import torch
    from paper_2303_12529_amd import ilt
    from paper_2303_12529_amd.inputs import BATCH_SIZES, batch_inputs
    clips, H, w = batch_inputs(n_clips)
    data = []
    flops = 0.0
    for Z, prm in clips:
        N = Z.shape[0]
        data.append((torch.as_tensor(Z).to("cuda"), torch.empty((N, N), dtype=torch.float32, device="cuda"),
                     ilt.Params.from_dict(prm, init_mode=0), None))
        flops += sum(v.get("flops", 0.0) for v in algorithmic_work(N, H.shape[2], H.shape[1], H.shape[0]).values()) \
            * prm["iters"]
    out = {"clips": n_clips, "sizes": {str(n): sum(1 for z, _ in clips if z.shape[0] == n) for n in BATCH_SIZES},
           "iters_per_clip": clips[0][1]["iters"], "dtype": "f32" if precision == ilt.ILT_FP32 else "bf16x3"}
    for nl in sorted({lanes, 1}, reverse=True):
        b = ilt.Batch(H, w, BATCH_SIZES, max_clips=n_clips, n_lanes=nl, precision=precision)
        tuned = b.autotune()               # clips per chunk and tuning per size
        b.solve(data)                      # captures the lanes' graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = b.solve(data)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        out["lanes_%d" % nl] = {"s_per_batch": round(dt, 4),
                                "clip_iters_per_s": round(n_clips * clips[0][1]["iters"] / dt, 1),
                                "algorithmic_tflops": round(flops / dt / 1e12, 2),
                                "l2_sum": int(sum(r["l2"] for r in reps)),
                                "autotune": tuned}
    if lanes > 1:
        out["speedup_vs_one_lane"] = round(out["lanes_1"]["s_per_batch"] / out["lanes_%d" % lanes]["s_per_batch"], 3)
    # the plain form: every clip alone through ilt_solve (a context per size,
    # each clip's graph captured by a first call and its replay timed), the
    # clips strictly one after another; same results bit for bit
    ctxs = {N: ilt.Context(H, w, N, precision=precision) for N in BATCH_SIZES}
    total, l2_plain = 0.0, 0
    for (tgt, phi, prm, _), (Z, _p) in zip(data, clips):
        ctx = ctxs[Z.shape[0]]
        ctx.ilt_solve(tgt, phi, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.ilt_solve(tgt, phi, prm)
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        l2_plain += int(rep["l2"])
    for c in ctxs.values():
        c.close()
    best = out["lanes_%d" % lanes]["s_per_batch"]
    out["plain_one_clip_at_a_time"] = {"s_total": round(total, 4), "algorithmic_tflops": round(flops / total / 1e12, 2),
                                       "l2_sum": l2_plain}
    out["time_to_result_vs_plain"] = {"batched_s": best, "plain_s": round(total, 4),
                                      "speedup": round(total / best, 3),
                                      "same_final_l2": l2_plain == out["lanes_%d" % lanes]["l2_sum"]}
    return out


def layout_leg(side, lanes, precision):
    """A side x side layout at 1 nm (the 2048^2 recipe scaled to its area),
    2048^2 tiles with a 256-pixel halo, every tile through the full loop on
    `lanes` streams (ilt_solve_layout: extraction, batched DSO, stitching),
    then the shot count of the stitched mask."""
    import torch
    from paper_2303_12529_amd import ilt
    from paper_2303_12529_amd.inputs import LAYOUT_HALO, LAYOUT_TILE, layout_inputs
    Z, H, w, prm = layout_inputs(side)
    N, halo = LAYOUT_TILE, LAYOUT_HALO
    rows, cols = ilt.layout_grid(side, side, N, halo)
    T = rows * cols
    b = ilt.Batch(H, w, [N], max_clips=T, n_lanes=lanes, precision=precision)
    target = torch.as_tensor(Z).to("cuda")
    tt = torch.empty((T, N, N), dtype=torch.uint8, device="cuda")
    tp = torch.empty((T, N, N), dtype=torch.float32, device="cuda")
    out = torch.empty((side, side), dtype=torch.float32, device="cuda")
    p = ilt.Params.from_dict(prm, init_mode=0)
    b.solve_layout(target, N, halo, p, tt, tp, out)          # captures the lanes' graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, reps, _ = b.solve_layout(target, N, halo, p, tt, tp, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    ilt.shot_count(phi=out, out=counts)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ilt.shot_count(phi=out, out=counts)
    e1.record()
    torch.cuda.synchronize()
    shots = counts.cpu().tolist()
    tshots = ilt.shot_count(mask=target).cpu().tolist()
    iters = prm["iters"]
    return {"layout": "%dx%d at 1 nm, the 2048^2 clip recipe scaled to the area, %.1f %% metal"
                      % (side, side, 100.0 * float(Z.mean())),
            "tile": N, "halo": halo, "tiles": T, "lanes": lanes, "iters_per_tile": iters,
            "s_per_layout": round(dt, 4), "tile_iters_per_s": round(T * iters / dt, 1),
            "um2_per_s": round(side * side * 1e-6 / dt, 3),
            "core_fraction": round(side * side / (T * N * N), 4),
            "shots_mask": shots[2], "shots_rows_cols": shots[:2], "shots_target": tshots[2],
            "shot_count_ms": round(e0.elapsed_time(e1) / 5, 4),
            "tile_l2_sum_with_halos": int(sum(r["l2"] for r in reps))}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-iters", type=int, default=4)
    ap.add_argument("--cpu-iters-1t", type=int, default=1, help="oracle iterations on one thread (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp32", "bf16x3"), default="fp32",
                    help="arithmetic of the dense contractions (default: the plain FP32 loop)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch settings instead of timing the tuning candidates first")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="first copy 256 MiB device to device (the reference kernel for scaling HBM counters)")
    ap.add_argument("--no-gwindow", action="store_true", help="skip the G-window adjoint line")
    ap.add_argument("--adjoint", choices=("fields", "gwindow"), default="fields",
                    help="adjoint of the timed loop: through the K fields (the paper's form, default) or the "
                         "G-window identity")
    ap.add_argument("--forward", choices=("fields", "hopkins"), default="fields",
                    help="image of the timed loop: through the K fields (default) or its difference-window "
                         "spectrum (TCC form; needs --adjoint gwindow and --precision fp32)")
    ap.add_argument("--batch-clips", type=int, default=64,
                    help="clips in the batched-form measurement (0: skip)")
    ap.add_argument("--batch-lanes", type=int, default=4)
    ap.add_argument("--layout-side", type=int, default=6144,
                    help="side of the full-layout measurement in pixels (0: skip)")
    ap.add_argument("--ttt-seeds", type=int, default=10,
                    help="seeds 0..n-1 for the time-to-L2-target comparison (0: skip)")
    ap.add_argument("--develset-seeds", type=int, default=100,
                    help="seeds 0..n-1 for DevelSet (level-set network, FP32 loop) against plain (0: the "
                         "time-to-target seeds)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X "
              "(see the design notes on sharding); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2303_12529_amd import ilt
    from paper_2303_12529_amd.inputs import WORKLOADS, workload_inputs

    Z, H, w, prm = workload_inputs(args.workload, args.seed)
    N = Z.shape[0]
    n_sets, K, P, _ = H.shape
    torch.cuda.set_device(0)
    if args.traffic_probe:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    prec = ilt.ILT_BF16X3 if args.precision == "bf16x3" else ilt.ILT_FP32
    if args.forward == "hopkins" and (args.adjoint != "gwindow" or args.precision != "fp32"):
        print("--forward hopkins needs --adjoint gwindow and --precision fp32", file=sys.stderr)
        sys.exit(2)
    flags = ilt.ILT_FLAG_GWINDOW_ADJOINT if args.adjoint == "gwindow" else 0
    if args.forward == "hopkins":
        flags |= ilt.ILT_FLAG_HOPKINS_FORWARD
    ctx = ilt.Context(H, w, N, precision=prec, flags=flags)
    tuning = None if args.no_autotune else ctx.autotune()
    target = torch.as_tensor(Z).to("cuda")
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")

    # warm-up: TSDF init + W iterations (loads every kernel), then one solve with
    # exactly the timed arguments so that the solve's hipGraph is captured
    # before the timed region (the timed call replays it)
    ctx.ilt_solve(target, phi, ilt.Params.from_dict(prm, iters=max(args.warmup, 1), init_mode=0))
    p = ilt.Params.from_dict(prm, iters=args.steps, init_mode=1)
    trace = torch.zeros((args.steps, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    phi_start = phi.clone()
    ctx.ilt_solve(target, phi, p, trace=trace)
    phi.copy_(phi_start)
    torch.cuda.synchronize()
    # timed region: K iterations, one graph launch, host sync on both sides
    t0 = time.perf_counter()
    rep = ctx.ilt_solve(target, phi, p, trace=trace)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # second pass over the same K iterations with a HIP event pair around each
    # phase's launches on the library's stream (events recorded inside a graph
    # carry no timestamps, so this pass launches directly)
    phi.copy_(phi_start)
    ctx.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.ilt_solve(target, phi, p, trace=trace)
    torch.cuda.synchronize()
    wall_direct = time.perf_counter() - t1
    prof = ctx.profile_read()
    ctx.profile(False)

    ms_per_step = 1e3 * wall / args.steps
    value = args.steps / wall
    if args.forward == "hopkins":
        work = hopkins_work(N, P, K, n_sets)
    elif args.adjoint == "gwindow":
        work = gwindow_work(N, P, K, n_sets)
    else:
        work = algorithmic_work(N, P, K, n_sets)
    phase_ms = {k: v[0] for k, v in prof.items()}
    dominant = max(phase_ms, key=lambda k: phase_ms[k])
    launches = prof[dominant][1]
    avg_ms = phase_ms[dominant] / max(launches, 1)
    wd = work[dominant]
    if "flops" in wd:
        # FP32 form: algorithmic FP32 flops against the FP32 matrix peak.
        # BF16x3 form: the same algorithmic flops counted as FP32-equivalent,
        # against the BF16 dense peak (each is issued as three BF16 products).
        achieved = wd["flops"] / (avg_ms * 1e-3) / 1e12
        peak = BF16_MFMA_PEAK_TFLOPS if args.precision == "bf16x3" else FP32_MFMA_PEAK_TFLOPS
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None}
    else:
        achieved = wd["bytes"] / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    dtype = "f32" if args.precision == "fp32" else "bf16x3"
    kname, ksrc = KERNELS.get((dominant, dtype), (dominant, ()))
    if (dominant == "adjoint" and args.adjoint == "gwindow") or (dominant == "image" and args.forward == "hopkins"):
        # other kernels than the field forms': the phase is named, no counter summary applies
        kname, ksrc = dominant, ()
    roof["kernel"] = kname
    roof["phase"] = dominant
    roof["avg_launch_ms"] = round(avg_ms, 4)
    if ksrc:
        roof["traffic"], roof["traffic_source"] = measured_traffic(kname, dtype, ksrc)
    if args.precision == "bf16x3":
        iss = issued_bf16_flops(N, P, K, n_sets, dominant)
        if iss:
            roof["issued_bf16_tflops"] = round(iss / (avg_ms * 1e-3) / 1e12, 1)
            roof["issued_bf16_frac"] = round(iss / (avg_ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4)
    total_flops = sum(v.get("flops", 0.0) for v in work.values())
    tr = trace.cpu().numpy()

    ttt = None
    if args.ttt_seeds > 0:
        ctxs = {"fp32": ctx if prec == ilt.ILT_FP32 and flags == 0 else ilt.Context(H, w, N, precision=ilt.ILT_FP32),
                "bf16x3": ctx if prec == ilt.ILT_BF16X3 and flags == 0 else ilt.Context(H, w, N,
                                                                                      precision=ilt.ILT_BF16X3)}
        if not args.no_gwindow:
            ctxs["fp32_gwindow"] = ilt.Context(H, w, N, precision=ilt.ILT_FP32,
                                               flags=ilt.ILT_FLAG_GWINDOW_ADJOINT)
            ctxs["bf16x3_gwindow"] = ilt.Context(H, w, N, precision=ilt.ILT_BF16X3,
                                                 flags=ilt.ILT_FLAG_GWINDOW_ADJOINT)
            ctxs["fp32_hopkins"] = ilt.Context(H, w, N, precision=ilt.ILT_FP32,
                                               flags=ilt.ILT_FLAG_GWINDOW_ADJOINT | ilt.ILT_FLAG_HOPKINS_FORWARD)
        if not args.no_autotune:
            for c in ctxs.values():
                if c is not ctx:
                    c.autotune()
        ttt = time_to_target(ctxs, args.workload, range(args.ttt_seeds))
        if args.workload == "c1":
            ttt["develset"] = develset_ttt(range(args.ttt_seeds),
                                           range(args.develset_seeds) if args.develset_seeds > 0 else None)
            for form in ("fp32_gwindow", "bf16x3", "bf16x3_gwindow", "fp32_hopkins"):
                if ttt["develset"] and ttt["median_ms"].get("fp32") and \
                        (ttt["develset"].get(form) or {}).get("median_ms_develset"):
                    ttt["develset_%s_speedup_vs_plain" % form] = round(
                        ttt["median_ms"]["fp32"] / ttt["develset"][form]["median_ms_develset"], 3)

    gw = None
    if not args.no_gwindow:
        gw = gwindow_forms(Z, H, w, N, prm, args.steps, not args.no_autotune)

    bat = None
    if args.batch_clips > 0:
        bat = batched(args.batch_clips, args.batch_lanes, prec)

    lay = None
    if args.layout_side > 0:
        lay = layout_leg(args.layout_side, args.batch_lanes, prec)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, args.seed, args.cpu_iters, args.cpu_iters_1t)

    desc = WORKLOADS[args.workload]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "%s: %dx%d clip at %.0f nm/px, K=%d kernels on a %dx%d window, %d kernel sets, "
                        "%d corners, TSDF reinit every %d" % (
                            args.workload, N, N, desc["optics"]["pitch_nm"], K, P, P, n_sets,
                            len(prm["corners"]), prm["reinit_every"]),
            "N": N, "P": P, "K": K, "n_sets": n_sets, "corners": len(prm["corners"]), "seed": args.seed,
            "adjoint": args.adjoint, "forward": args.forward,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "whole_loop_tflops": round(total_flops * value / 1e12, 2),
        "whole_loop_frac_fp32_mfma": round(total_flops * value / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4),
        "phases_ms_per_step": {k: round(v / args.steps, 4) for k, v in phase_ms.items()},
        "roofline_pass": "same %d iterations launched directly with per-phase HIP events: %.4f ms/step"
                         % (args.steps, 1e3 * wall_direct / args.steps),
        "final": {"l2": rep["l2"], "pvb": rep["pvb"], "loss": rep["loss"],
                  "l2_first": int(tr[0, 2]), "l2_last_iter": int(tr[-1, 2])},
        "tuning": tuning if tuning is not None else ctx.get_tuning(),
        "time_to_target": ttt,
        "gwindow_adjoint": gw,
        "batched": bat,
        "full_layout": lay,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
