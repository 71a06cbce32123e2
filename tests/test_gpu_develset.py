"""DevelSet (Sec. III-C): what the committed network gains over DSO alone.

The trained level-set network (weights/dsn_c1_fp16.npy, trained on seeds
from 100000 on) predicts phi_0 for held-out clips of the 2048^2 workload;
DSO from that phi_0 must reach the L2 that the plain loop reaches after its
50 iterations from TSDF(target) in fewer iterations, and be no worse than
the plain loop at iteration 50.  A network whose phi_0 prints worse than the
target's own mask must be judged useless and replaced by TSDF(target): then
DevelSet is the plain loop, iteration for iteration.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2303_12529_amd", "weights", "dsn_c1_fp16.npy")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_12529_amd import develset, dsn, ilt
    ilt.load_library()
    return develset, dsn, ilt


def test_committed_network_beats_plain_on_held_out_seeds(mods):
    develset, dsn, ilt = mods
    flat = np.load(WEIGHTS, allow_pickle=False).astype(np.float32)
    net = dsn.Net(512, 512, 32, max_batch=1)
    net.set_params(flat)
    ev = develset.evaluate(net, [0, 3, 7], precision=ilt.ILT_FP32)
    for r in ev["per_seed"]:
        _say("seed", r["seed"], "plain", r["iters_plain"], "develset", r["iters_develset"],
             "l2@T", r["l2_at_T_plain"], r["l2_at_T_develset"], "epe", r.get("epe_plain"), r.get("epe_develset"))
        assert r["dsn_used"]
        assert r["l2_init_dsn"] < r["l2_init_tsdf"]
        assert r["iters_plain"] is not None and r["iters_develset"] is not None
        assert r["iters_develset"] < r["iters_plain"]
        assert r["l2_at_T_develset"] <= r["l2_at_T_plain"]
    assert ev["speedup"] > 1.0
    net.close()


def test_useless_network_falls_back_to_plain(mods):
    develset, dsn, ilt = mods
    net = dsn.Net(512, 512, 32, max_batch=1)
    # all-zero parameters: phi_0 = 0 everywhere, so [phi_0 <= 0] is the whole
    # frame, which prints far worse than the target's own mask
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    ev = develset.evaluate(net, [1], precision=ilt.ILT_FP32)
    r = ev["per_seed"][0]
    _say(r)
    assert not r["dsn_used"]
    assert r["l2_init_dsn"] > r["l2_init_tsdf"]
    assert r["iters_develset"] == r["iters_plain"]
    assert r["l2_at_T_develset"] == r["l2_at_T_plain"]
    net.close()
