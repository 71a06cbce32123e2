"""The allocation-free TSDF entry point (edt_reinit_noalloc) against the
context-based edt_reinit: bit-exact phi and squared distances on two calls
in a row, the second on a smaller, ragged image, so the static scratch
holds the first call's contents when the second runs."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2303_12529_amd.inputs import random_mask, random_phi  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ilt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_12529_amd import ilt as mod
    mod.load_library()
    return mod


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _context_edt(ilt, N, lo, hi, phi=None, mask=None):
    rng = np.random.default_rng(0)
    H = (rng.normal(size=(1, 1, 3, 3)) + 1j * rng.normal(size=(1, 1, 3, 3))) / 3.0
    ctx = ilt.Context(H, np.ones((1, 1)), N)
    sq = torch.empty((2, N, N), dtype=torch.int32, device="cuda")
    out = ctx.edt_reinit(ilt.Params(d_lower=lo, d_upper=hi), phi=phi, mask=mask, sqdist=sq)
    torch.cuda.synchronize()
    ctx.close()
    return out, sq


def test_noalloc_equals_edt_reinit_two_calls(ilt):
    # first call: 512^2 mask; second: 197^2 phi (smaller, not a multiple of 4
    # or of the 32-row words), each checked against the context entry point
    cases = [(512, "mask", 0.3, -100.0, 900.0), (197, "phi", None, -12.5, 112.5)]
    for N, kind, dens, lo, hi in cases:
        _say("noalloc edt", N, kind)
        if kind == "mask":
            src = dict(mask=_dev(random_mask(N, dens, seed=N), torch.uint8))
        else:
            src = dict(phi=_dev(random_phi(N, seed=N).astype(np.float32)))
        out = torch.full((N, N), float("nan"), dtype=torch.float32, device="cuda")
        sq = torch.full((2, N, N), -7, dtype=torch.int32, device="cuda")
        ilt.edt_reinit_noalloc(N, lo, hi, phi_out=out, sqdist=sq, **src)
        torch.cuda.synchronize()
        ref, ref_sq = _context_edt(ilt, N, lo, hi, **src)
        assert torch.equal(out, ref)
        assert torch.equal(sq, ref_sq)
        # without the squared-distance output, and in place on a phi input
        out2 = ilt.edt_reinit_noalloc(N, lo, hi, **src)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
    t = _dev(random_phi(64, seed=5).astype(np.float32))
    ref, _ = _context_edt(ilt, 64, -12.5, 112.5, phi=t.clone())
    ilt.edt_reinit_noalloc(64, -12.5, 112.5, phi=t, phi_out=t)
    torch.cuda.synchronize()
    assert torch.equal(t, ref)


def test_noalloc_rejects_sizes_beyond_its_scratch(ilt):
    m = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    out = torch.empty((16, 16), dtype=torch.float32, device="cuda")
    lib = ilt.load_library()
    import ctypes
    for N in (0, 4097, 1 << 20):
        rc = lib.edt_reinit_noalloc(N, None, ctypes.c_void_p(m.data_ptr()), -1.0, 1.0,
                                    ctypes.c_void_p(out.data_ptr()), None, None)
        assert rc == ilt.ILT_EINVAL
        assert b"4096" in lib.ilt_last_error()
    with pytest.raises(ilt.IltError):          # neither input given
        lib_rc = lib.edt_reinit_noalloc(16, None, None, -1.0, 1.0, ctypes.c_void_p(out.data_ptr()), None, None)
        ilt._check(lib_rc)
