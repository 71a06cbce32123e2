"""Train DSN on DSO results and measure DevelSet.

    python -m paper_2303_12529_amd.train_dsn --clips 1024 --epochs 10 --out DIR [--modulation]

--modulation adds the modulation branch: its targets come from the shift
search of develset.make_dataset, it trains on L_0 + L_m, and the evaluation
adds DevelSet with the network's modulation map.

Writes DIR/dsn_weights.npy (flat FP32 parameters, the layout of
include/dsn.h) and DIR/dsn_report.json (dataset and training times, the
loss per epoch, network throughput, and the DevelSet vs plain evaluation).
Seeds of the training clips start at 100000; evaluation uses seeds 0..n-1,
so the two never overlap.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def conv_flops(H, W, base=32, levels=4):
    """Algorithmic flops of one forward pass of one sample (multiply-add = 2)."""
    ch = [base << i for i in range(levels)]
    f = 0.0
    prev = 1
    for l in range(levels):
        hw = (H >> l) * (W >> l)
        f += 2.0 * hw * 9 * prev * ch[l] + 2.0 * hw * 9 * ch[l] * ch[l]
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        hw = (H >> l) * (W >> l)
        f += 2.0 * hw * 9 * (ch[l + 1] * ch[l] + 2 * ch[l] * ch[l] + ch[l] * ch[l])
    f += 2.0 * H * W * ch[0]
    return f


def speed(net, batch, steps=10):
    """ms per training step (forward, backward, Adam) and per forward pass."""
    import torch
    x = torch.rand((batch, net.H, net.W), device="cuda")
    t = torch.rand((batch, net.H, net.W), device="cuda")
    tm = t if net.modulation else None
    for _ in range(2):
        net.forward(x)
        net.backward(t, target_m=tm)
        net.adam_step(0.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.forward(x)
        net.backward(t, target_m=tm)
        net.adam_step(0.0)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    e0.record()
    for _ in range(steps):
        net.forward(x)
    e1.record()
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / steps
    f = conv_flops(net.H, net.W, net.base)
    return {"batch": batch, "ms_per_train_step": round(ms_step, 3), "ms_per_forward": round(ms_fwd, 3),
            "forward_tflops": round(batch * f / (ms_fwd * 1e-3) / 1e12, 1),
            "train_tflops": round(3 * batch * f / (ms_step * 1e-3) / 1e12, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--clips", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--speed-only", action="store_true")
    ap.add_argument("--modulation", action="store_true")
    ap.add_argument("--init", default=None,
                    help="flat parameters (.npy) to start from, e.g. a trained level-set network for the "
                         "two-branch one; parameters beyond them (the modulation head) keep their He values")
    ap.add_argument("--workers", type=int, default=0,
                    help="processes drawing the training clips while the device solves (0: draw in line)")
    args = ap.parse_args()

    # the clip-drawing workers start before this process touches the device
    pool = None
    if args.workers > 0 and not args.speed_only:
        import multiprocessing
        from .develset import clip_of_seed
        pool = multiprocessing.get_context("spawn").Pool(args.workers)
        clip_iter = pool.imap(clip_of_seed, range(100000, 100000 + args.clips), chunksize=4)

    import torch
    from . import develset
    from . import dsn

    def log(msg):
        print(msg, flush=True)

    os.makedirs(args.out, exist_ok=True)
    torch.cuda.set_device(0)
    net = dsn.Net(512, 512, 32, max_batch=args.batch, modulation=args.modulation)
    init = dsn.he_init(args.seed, modulation=args.modulation)
    if args.init:
        import numpy as np
        start = np.load(args.init, allow_pickle=False)
        if start.ndim != 1 or start.size > init.size:
            raise SystemExit("--init: expected a flat vector of at most %d parameters" % init.size)
        init[:start.size] = start.astype(np.float32)
    net.set_params(init)
    report = {"network": {"grid": [512, 512], "base": 32, "params": net.n_params, "modulation": args.modulation,
                          "forward_gflop_per_sample": round(develset_flops(net) / 1e9, 2)}}
    if args.init:
        report["init"] = os.path.basename(args.init)
    report["speed"] = speed(net, args.batch)
    log("speed %s" % report["speed"])
    if args.speed_only:
        print(json.dumps(report), flush=True)
        return
    net.set_params(init)
    t0 = time.perf_counter()
    data = develset.make_dataset(args.clips, 100000, net, log=log, clips=clip_iter if pool else None)
    if pool:
        pool.close()
        pool.join()
    x, t = data[0], data[1]
    tm = data[2] if args.modulation else None
    report["dataset"] = {"clips": args.clips, "seconds": round(time.perf_counter() - t0, 1)}
    if args.modulation:
        import numpy as np
        vals, counts = np.unique(data[3], return_counts=True)
        report["dataset"]["shift_histogram"] = {int(v): int(c) for v, c in zip(vals, counts)}
        log("shift histogram %s" % report["dataset"]["shift_histogram"])
    t0 = time.perf_counter()
    hist = develset.train(net, x, t, args.epochs, args.batch, args.lr, seed=args.seed, log=log, tm=tm)
    report["training"] = {"epochs": args.epochs, "batch": args.batch, "lr": args.lr, "loss_per_epoch": hist,
                          "seconds": round(time.perf_counter() - t0, 1)}
    del x, t, tm, data
    import numpy as np
    np.save(os.path.join(args.out, "dsn_weights.npy"), net.get_params().cpu().numpy())
    report["evaluation"] = develset.evaluate(net, range(args.eval_seeds), log=log)
    with open(os.path.join(args.out, "dsn_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "evaluation"}), flush=True)
    ev = report["evaluation"]
    print(json.dumps({k: ev.get(k) for k in ("median_ms_plain", "median_ms_develset", "speedup", "dsn_used",
                                              "median_ms_develset_m", "speedup_m", "reached_develset_m")}),
          flush=True)


def develset_flops(net):
    return conv_flops(net.H, net.W, net.base)


if __name__ == "__main__":
    sys.exit(main())
