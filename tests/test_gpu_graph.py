"""hipGraph replay of ilt_solve against direct launches (needs an MI355X).

The graph is replayed several times with unrelated direct work and host
synchronisations in between; every replay must equal the direct run bitwise.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2303_12529_amd.inputs import workload_inputs, random_mask  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ilt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_12529_amd import ilt as mod
    mod.load_library()
    return mod


def _run(ctx, ilt, Z, prm, phi, trace):
    rep = ctx.ilt_solve(Z, phi, ilt.Params.from_dict(prm), trace=trace)
    return phi.cpu().numpy().copy(), trace.cpu().numpy().copy(), rep


@pytest.mark.parametrize("flags", [0, 1])
def test_graph_replays_equal_direct(ilt, flags):
    Zn, H, w, prm = workload_inputs("c0", 5)
    prm = dict(prm, iters=8)
    N = Zn.shape[0]
    ctx = ilt.Context(H, w, N, flags=flags)
    Z = torch.as_tensor(Zn).cuda()
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    trace = torch.zeros((prm["iters"], ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ctx.set_graph(False)
    ref_phi, ref_tr, ref_rep = _run(ctx, ilt, Z, prm, phi, trace)
    ctx.set_graph(True)
    other = torch.as_tensor(random_mask(N, 0.3, 7).astype(np.float32)).cuda()
    for rep_i in range(4):
        g_phi, g_tr, g_rep = _run(ctx, ilt, Z, prm, phi, trace)
        assert np.array_equal(g_phi, ref_phi), rep_i
        assert np.array_equal(g_tr[:, :7], ref_tr[:, :7]), rep_i
        assert g_rep["l2"] == ref_rep["l2"] and g_rep["loss"] == ref_rep["loss"]
        # unrelated direct work and a host sync between replays
        ctx.litho_forward(other, 0)
        torch.cuda.synchronize()
    # new arguments: a fresh capture gives the same answer again
    trace2 = torch.zeros_like(trace)
    phi2 = torch.empty_like(phi)
    g_phi, g_tr, _ = _run(ctx, ilt, Z, prm, phi2, trace2)
    assert np.array_equal(g_phi, ref_phi) and np.array_equal(g_tr[:, :7], ref_tr[:, :7])


def test_profiled_solve_matches_graph(ilt):
    """The measurement hook forces direct launches; results are unchanged."""
    Zn, H, w, prm = workload_inputs("c0", 6)
    prm = dict(prm, iters=6)
    N = Zn.shape[0]
    ctx = ilt.Context(H, w, N)
    Z = torch.as_tensor(Zn).cuda()
    phi = torch.empty((N, N), dtype=torch.float32, device="cuda")
    trace = torch.zeros((prm["iters"], ilt.TRACE_W), dtype=torch.float64, device="cuda")
    ref_phi, _, _ = _run(ctx, ilt, Z, prm, phi, trace)        # graph replay
    ctx.profile(True)
    for _ in range(2):
        g_phi, _, _ = _run(ctx, ilt, Z, prm, phi, trace)
        assert np.array_equal(g_phi, ref_phi)
        prof = ctx.profile_read()
        assert prof["adjoint"][1] == prm["iters"] and prof["adjoint"][0] > 0
        assert prof["reinit"][1] == 1 + prm["iters"] // prm["reinit_every"]
    ctx.profile(False)
