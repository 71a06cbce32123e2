"""Parity of the whole DSO loop (ilt_solve) against the FP64 oracle.

* Teacher-forced: from the same phi_0 (FP32 values), one GPU iteration and one
  oracle iteration; the trace row and phi_1 must agree (c0 and c1 sizes).
* Trajectory (c0): the binary print L2 depends on hard threshold flips, so
  whole trajectories are compared in a band (trajectories diverge at near-ties).
* Determinism: two runs are bitwise identical.
"""
import sys

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


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("name,seed", [("c0", 0), ("c0", 3), ("c1", 0)])
def test_one_iteration_teacher_forced(ilt, name, seed):
    _say("teacher-forced", name, seed)
    Z, H, w, prm = workload_inputs(name, seed)
    N = Z.shape[0]
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    phi0 = phi0.astype(np.float32)
    prm1 = dict(prm, iters=1, reinit_every=0)
    ctx = ilt.Context(H, w, N)
    p = ilt.Params.from_dict(prm1, init_mode=1)
    phi = _dev(phi0)
    trace = torch.zeros((1, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(_dev(Z, torch.uint8), phi, p, trace=trace)
    out = phi.cpu().numpy().astype(np.float64)
    tr = trace.cpu().numpy()[0]
    ref, row = o_solve.iteration(phi0.astype(np.float64), Z, H, w, prm1)
    _say("  loss", tr[1], row["loss"], "l2", tr[2], row["l2"], "pvb", tr[3], row["pvb"],
         "m_v", tr[5], row["m_v"], "flips", tr[4], row["flips"])
    assert abs(tr[1] - row["loss"]) <= 1e-5 * abs(row["loss"])
    assert abs(tr[5] - row["m_v"]) <= 1e-4 * row["m_v"]
    # print decisions may differ only at near-ties of I with the threshold
    assert abs(tr[2] - row["l2"]) <= max(2, 1e-4 * row["l2"])
    assert abs(tr[3] - row["pvb"]) <= max(2, 1e-4 * max(row["pvb"], 1))
    err = np.abs(out - ref)
    _say("  phi max err", err.max())
    assert err.max() <= 1e-3 * prm["eta"] + 4 * np.spacing(np.float32(np.abs(ref).max()))
    assert abs(tr[4] - row["flips"]) <= max(2, 0.01 * row["flips"])


def test_c0_trajectory_band(ilt):
    Z, H, w, prm = workload_inputs("c0", 1)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    p = ilt.Params.from_dict(prm)
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    trace = torch.zeros((prm["iters"], ilt.TRACE_W), dtype=torch.float64, device="cuda")
    rep = ctx.ilt_solve(_dev(Z, torch.uint8), phi, p, trace=trace)
    tr = trace.cpu().numpy()
    _, otr, ofin = o_solve.ilt_solve(Z, H, w, prm)
    l2g = tr[:, 2]
    l2o = np.array([r["l2"] for r in otr])
    _say("gpu l2", l2g.astype(int).tolist())
    _say("ref l2", l2o.tolist())
    _say("final", rep, ofin)
    band = 0.02 * l2o[0] + 10
    assert np.all(np.abs(l2g - l2o) <= band)
    assert abs(rep["l2"] - ofin["l2"]) <= band
    # the loop makes progress
    assert rep["l2"] < l2o[0]


def test_recompute_and_stored_fields_agree(ilt):
    Z, H, w, prm = workload_inputs("c0", 4)
    N = Z.shape[0]
    outs = []
    for flags in (0, ilt.ILT_FLAG_RECOMPUTE_FIELDS):
        ctx = ilt.Context(H, w, N, flags=flags)
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        tr = torch.zeros((6, ilt.TRACE_W), dtype=torch.float64, device="cuda")
        ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm, iters=6), trace=tr)
        outs.append((phi.cpu().numpy(), tr.cpu().numpy()))
    np.testing.assert_array_equal(outs[0][1][:, 2], outs[1][1][:, 2])
    assert np.abs(outs[0][0] - outs[1][0]).max() <= 1e-4


def test_solve_deterministic_and_init_modes(ilt):
    Z, H, w, prm = workload_inputs("c0", 2)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    p = ilt.Params.from_dict(prm, iters=7)
    outs = []
    for _ in range(2):
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        tr = torch.zeros((7, ilt.TRACE_W), dtype=torch.float64, device="cuda")
        rep = ctx.ilt_solve(_dev(Z, torch.uint8), phi, p, trace=tr)
        outs.append((phi.cpu().numpy(), tr.cpu().numpy()[:, :7], rep))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    # init_mode 1 from the TSDF gives the same run as init_mode 0
    phi0 = ctx.edt_reinit(p, mask=_dev(Z, torch.uint8))
    tr = torch.zeros((7, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(_dev(Z, torch.uint8), phi0, ilt.Params.from_dict(prm, iters=7, init_mode=1), trace=tr)
    assert np.array_equal(phi0.cpu().numpy(), outs[0][0])


def test_solve_rejects_bad_arguments(ilt):
    Z, H, w, prm = workload_inputs("c0", 0)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    bad = ilt.Params.from_dict(prm, corners=((3, 1.0, 1.0),))
    with pytest.raises(ilt.IltError) as e:
        ctx.ilt_solve(_dev(Z, torch.uint8), phi, bad)
    assert e.value.code == ilt.ILT_EINVAL
    with pytest.raises(ilt.IltError):
        ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm, d_lower=1.0))
    with pytest.raises(ilt.IltError):
        ilt.Context(H, w, 8)          # N below the minimum


@pytest.mark.parametrize("name,seed,prec", [("c0", 0, "fp32"), ("c1", 0, "fp32"), ("c1", 2, "bf16x3"),
                                            ("c0", 1, "hopkins"), ("c1", 1, "hopkins")])
def test_gwindow_adjoint_iteration_teacher_forced(ilt, name, seed, prec):
    """One iteration with the G-window adjoint (and, for "hopkins", the image
    through its difference-window spectrum) against the oracle's step."""
    Z, H, w, prm = workload_inputs(name, seed)
    N = Z.shape[0]
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    phi0 = phi0.astype(np.float32)
    prm1 = dict(prm, iters=1, reinit_every=0)
    precision = ilt.ILT_BF16X3 if prec == "bf16x3" else ilt.ILT_FP32
    flags = ilt.ILT_FLAG_GWINDOW_ADJOINT | (ilt.ILT_FLAG_HOPKINS_FORWARD if prec == "hopkins" else 0)
    ctx = ilt.Context(H, w, N, precision=precision, flags=flags)
    phi = _dev(phi0)
    trace = torch.zeros((1, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm1, init_mode=1), trace=trace)
    tr = trace.cpu().numpy()[0]
    ref, row = o_solve.iteration(phi0.astype(np.float64), Z, H, w, prm1)
    err = np.abs(phi.cpu().numpy().astype(np.float64) - ref).max()
    _say("gwindow", name, seed, prec, "loss", tr[1], row["loss"], "m_v", tr[5], row["m_v"], "phi err", err)
    fp32 = prec != "bf16x3"
    rel = 1e-5 if fp32 else 1e-3
    assert abs(tr[1] - row["loss"]) <= rel * abs(row["loss"])
    assert abs(tr[5] - row["m_v"]) <= (1e-4 if fp32 else 2e-2) * row["m_v"]
    assert err <= (1e-3 if fp32 else 2e-2) * prm["eta"] + 1e-3


def test_gwindow_trajectory_matches_stored_fields(ilt):
    Z, H, w, prm = workload_inputs("c0", 6)
    N = Z.shape[0]
    outs = []
    for flags in (0, ilt.ILT_FLAG_GWINDOW_ADJOINT, ilt.ILT_FLAG_GWINDOW_ADJOINT | ilt.ILT_FLAG_HOPKINS_FORWARD):
        ctx = ilt.Context(H, w, N, flags=flags)
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        tr = torch.zeros((8, ilt.TRACE_W), dtype=torch.float64, device="cuda")
        ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm, iters=8), trace=tr)
        outs.append(tr.cpu().numpy())
    # same method, different rounding order: print counts within near-ties
    for o in outs[1:]:
        assert np.all(np.abs(outs[0][:, 2] - o[:, 2]) <= 2)
        assert np.allclose(outs[0][:, 5], o[:, 5], rtol=1e-3)


def test_cg_first_step_equals_plain(ilt):
    """With beta = 0 on the first step the conjugate direction is the gradient."""
    Z, H, w, prm = workload_inputs("c0", 7)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    outs = []
    for opt in (0, 1):
        phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
        ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm, iters=1, optimizer=opt))
        outs.append(phi.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_cg_iterations_teacher_forced(ilt):
    """Three CG iterations (no reinit) from the same phi_0 against the oracle."""
    Z, H, w, prm = workload_inputs("c0", 8)
    N = Z.shape[0]
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    phi0 = phi0.astype(np.float32)
    prm3 = dict(prm, iters=3, reinit_every=0, optimizer=1)
    ctx = ilt.Context(H, w, N)
    phi = _dev(phi0)
    trace = torch.zeros((3, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm3, init_mode=1), trace=trace)
    tr = trace.cpu().numpy()
    ref = phi0.astype(np.float64)
    state = {}
    for i in range(3):
        ref, row = o_solve.iteration(ref, Z, H, w, prm3, state)
        _say("cg it", i, "loss", tr[i, 1], row["loss"], "m_v", tr[i, 5], row["m_v"], "beta", row["beta"])
        assert abs(tr[i, 1] - row["loss"]) <= 1e-4 * abs(row["loss"])
        assert abs(tr[i, 5] - row["m_v"]) <= 1e-3 * row["m_v"]
    err = np.abs(phi.cpu().numpy().astype(np.float64) - ref).max()
    _say("cg phi err", err)
    assert err <= 3e-3 * prm["eta"] + 1e-3


def test_cg_trajectory_band(ilt):
    Z, H, w, prm = workload_inputs("c0", 1)
    N = Z.shape[0]
    prm = dict(prm, optimizer=1)
    ctx = ilt.Context(H, w, N)
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    trace = torch.zeros((prm["iters"], ilt.TRACE_W), dtype=torch.float64, device="cuda")
    rep = ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm), trace=trace)
    l2g = trace.cpu().numpy()[:, 2]
    _, otr, ofin = o_solve.ilt_solve(Z, H, w, prm)
    l2o = np.array([r["l2"] for r in otr])
    _say("cg gpu l2", l2g.astype(int).tolist())
    _say("cg ref l2", l2o.tolist())
    band = 0.02 * l2o[0] + 10
    assert np.all(np.abs(l2g - l2o) <= band)
    assert abs(rep["l2"] - ofin["l2"]) <= band


def _modulation_map(Z, phi0, dh):
    """A modulation map of the shape the modulation branch learns: the
    Heaviside map of the target's shifted TSDF."""
    return (phi0.astype(np.float64) + dh >= 0).astype(np.float32)


@pytest.mark.parametrize("dh", [-5.0, -15.0])
def test_modulated_iterations_teacher_forced(ilt, dh):
    """Three modulated iterations (no reinit) against the oracle's loop with the
    same map; the map must change the result."""
    _say("modulated teacher-forced dh", dh)
    Z, H, w, prm = workload_inputs("c0", 4)
    N = Z.shape[0]
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    phi0 = phi0.astype(np.float32)
    mod = _modulation_map(Z, phi0, dh)
    prm3 = dict(prm, iters=3, reinit_every=0)
    ctx = ilt.Context(H, w, N)
    phi = _dev(phi0)
    trace = torch.zeros((3, ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.ilt_solve(_dev(Z, torch.uint8), phi, ilt.Params.from_dict(prm3, init_mode=1), trace=trace, mod=_dev(mod))
    tr = trace.cpu().numpy()
    ref = phi0.astype(np.float64)
    plain = phi0.astype(np.float64)
    for i in range(3):
        ref, row = o_solve.iteration(ref, Z, H, w, prm3, mod=mod.astype(np.float64))
        plain, _ = o_solve.iteration(plain, Z, H, w, prm3)
        assert abs(tr[i, 1] - row["loss"]) <= 1e-4 * abs(row["loss"])
        assert abs(tr[i, 5] - row["m_v"]) <= 1e-3 * row["m_v"]
    out = phi.cpu().numpy().astype(np.float64)
    err = np.abs(out - ref).max()
    _say("  phi err", err, "modulation effect", np.abs(ref - plain).max())
    assert err <= 3e-3 * prm["eta"] + 1e-3
    assert np.abs(ref - plain).max() > 10 * (3e-3 * prm["eta"] + 1e-3)


def test_modulated_with_ones_equals_plain_and_replays(ilt):
    """m = 1 everywhere reproduces ilt_solve bitwise; a replayed graph reads the
    map's current contents (new values at the same address)."""
    Z, H, w, prm = workload_inputs("c0", 6)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    tgt = _dev(Z, torch.uint8)
    p = ilt.Params.from_dict(prm, iters=8)
    phi_a = torch.empty((N, N), dtype=torch.float32, device="cuda")
    ctx.ilt_solve(tgt, phi_a, p)
    mod = torch.ones((N, N), dtype=torch.float32, device="cuda")
    phi_b = torch.empty_like(phi_a)
    ctx.ilt_solve(tgt, phi_b, p, mod=mod)
    assert torch.equal(phi_a, phi_b)
    phi0, _, _ = o_edt.tsdf_from_mask(Z, prm["d_lower"], prm["d_upper"])
    mod.copy_(_dev(_modulation_map(Z, phi0, 5.0)))
    ctx.ilt_solve(tgt, phi_b, p, mod=mod)                  # graph replay, new contents
    ctx.set_graph(False)
    phi_c = torch.empty_like(phi_a)
    ctx.ilt_solve(tgt, phi_c, p, mod=mod)                  # direct launches
    assert torch.equal(phi_b, phi_c) and not torch.equal(phi_a, phi_b)


def test_modulated_rejects_null_map(ilt):
    Z, H, w, prm = workload_inputs("c0", 0)
    N = Z.shape[0]
    ctx = ilt.Context(H, w, N)
    lib = ilt.load_library()
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    pc = ilt.Params.from_dict(prm).to_c()
    import ctypes
    rc = lib.ilt_solve_modulated(ctx._h, ctypes.c_void_p(_dev(Z, torch.uint8).data_ptr()),
                                 ctypes.c_void_p(phi.data_ptr()), None, ctypes.byref(pc), None, None)
    assert rc == ilt.ILT_EINVAL
