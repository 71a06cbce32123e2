"""Tuning knobs and the autotuner.

Every candidate setting must still meet the parity bars (teacher-forced
iteration against the FP64 oracle); the autotuner must pick one of the
candidates, write it to its cache and take it back from there.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import edt as o_edt  # noqa: E402
from oracle import solve as o_solve  # noqa: E402
from paper_2303_12529_amd.inputs import workload_inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ilt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_12529_amd import ilt as mod
    mod.load_library()
    return mod


CANDIDATES = [("fp32", dict(store_fields=1, st_xsplit=1)), ("fp32", dict(store_fields=1, st_xsplit=2)),
              ("fp32", dict(store_fields=0))] + \
    [("bf16x3", dict(b3_xsplit=xs, xcd_remap=rm)) for xs in (1, 2, 4) for rm in (0, 1)]


@pytest.mark.parametrize("prec,tune", CANDIDATES)
def test_every_setting_meets_parity(ilt, prec, tune):
    Z, H, w, prm = workload_inputs("c0", 5)
    N = Z.shape[0]
    precision = ilt.ILT_BF16X3 if prec == "bf16x3" else ilt.ILT_FP32
    ctx = ilt.Context(H, w, N, precision=precision)
    ctx.set_tuning(**tune)
    assert {k: ctx.get_tuning()[k] for k in tune} == tune
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    phi0 = phi0.astype(np.float32)
    prm1 = dict(prm, iters=1, reinit_every=0)
    phi = torch.as_tensor(phi0).cuda()
    tr = torch.zeros((1, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(torch.as_tensor(Z).cuda(), phi, ilt.Params.from_dict(prm1, init_mode=1), trace=tr)
    ref, row = o_solve.iteration(phi0.astype(np.float64), Z, H, w, prm1)
    t = tr.cpu().numpy()[0]
    rel = 1e-5 if prec == "fp32" else 1e-3
    assert abs(t[1] - row["loss"]) <= rel * abs(row["loss"])
    err = np.abs(phi.cpu().numpy() - ref).max()
    _say(prec, tune, "phi err", err)
    assert err <= (1e-3 if prec == "fp32" else 2e-2) * prm["eta"] + 1e-3
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_autotune_picks_a_candidate_and_caches_it(ilt, prec):
    Z, H, w, prm = workload_inputs("c0", 0)
    N = Z.shape[0]
    precision = ilt.ILT_BF16X3 if prec == "bf16x3" else ilt.ILT_FP32
    ctx = ilt.Context(H, w, N, precision=precision)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.jsonl")
        first = ctx.autotune(path)
        _say(prec, "tuned", first)
        assert not first["from_cache"] and first["ms_per_iter"] > 0
        picked = {k: first[k] for k in ("store_fields", "b3_xsplit", "xcd_remap", "st_xsplit")}
        assert picked == ctx.get_tuning()
        if prec == "fp32":
            assert picked["store_fields"] in (0, 1) and picked["st_xsplit"] == 0
        else:
            assert picked["b3_xsplit"] in (1, 2, 4) and picked["xcd_remap"] in (0, 1)
        lines = open(path).read().strip().splitlines()
        assert len(lines) == 1 and '"N": %d' % N in lines[0]
        ctx.set_tuning(xcd_remap=1 - picked["xcd_remap"]) if prec == "bf16x3" else None
        again = ctx.autotune(path)
        assert again["from_cache"] and {k: again[k] for k in picked} == picked == ctx.get_tuning()
    # the solve still runs after tuning
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    rep = ctx.ilt_solve(torch.as_tensor(Z).cuda(), phi, ilt.Params.from_dict(prm, iters=3))
    assert rep["status"] == 0
    ctx.close()


def test_bad_tuning_rejected(ilt):
    Z, H, w, prm = workload_inputs("c0", 0)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N, flags=ilt.ILT_FLAG_RECOMPUTE_FIELDS)
    with pytest.raises(ilt.IltError):
        ctx.set_tuning(store_fields=1)          # no field buffer
    with pytest.raises(ilt.IltError):
        ctx.set_tuning(b3_xsplit=5)
    with pytest.raises(ilt.IltError):
        ctx.set_tuning(st_xsplit=3)
    ctx.close()
