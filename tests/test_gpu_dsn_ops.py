"""Single-layer parity of the DevelSet-Net kernels that the whole-network test
only holds in a band (Sec. III-B): the first convolution and its weight
gradient, the head backward with and without the modulation head (L_0,
L_m and their gradients), max-pooling, upsampling and ReLU backward, and the
ReLU backward fused into the head, pooling and upsampling backward (the
training step's form).

Each call runs the same kernel, with the same work split, as the training
step.  FP32 results are compared with the FP64 oracle (dsn.py) evaluated on
the same BF16 / FP32 inputs; the BF16 copies, sums and masks are compared
bit for bit with the same operations carried out in the kernel's precision
(an FP32 sum in the kernel's order, rounded once to BF16).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dsn as ref  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dsn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_12529_amd import dsn as mod
    mod._lib()
    return mod


def _bf16(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _bits(t):
    return t.cpu().view(torch.int16).numpy()


def _round_bf16(a32):
    """Round-to-nearest-even of float32 values to BF16 (a torch CPU tensor)."""
    return torch.as_tensor(np.ascontiguousarray(a32, dtype=np.float32)).to(torch.bfloat16)


@pytest.mark.parametrize("N,H,W,C", [(3, 40, 24, 32), (2, 130, 66, 64), (1, 9, 7, 8)])
def test_conv_first(dsn, N, H, W, C):
    rng = np.random.default_rng(N + H + C)
    x = rng.random((N, H, W)).astype(np.float32)
    w = _bf16(rng.normal(scale=0.4, size=(C, 3, 3, 1)))
    b = rng.normal(scale=0.1, size=C).astype(np.float32)
    y = dsn.conv_first(torch.as_tensor(x).cuda(), w.cuda(), torch.as_tensor(b).cuda())
    yr = ref.relu(ref.conv3x3(x.astype(np.float64)[..., None], _np(w), b.astype(np.float64)))
    err = np.abs(_np(y) - yr)
    assert np.all(err <= 2.0 ** -8 * np.abs(yr) + 1e-6 * np.abs(yr).max()), err.max()


# (B, H, W, C): one range over three images; ranges of 4667 pixels that start
# mid-row; ranges of 6000 pixels that start mid-image and cross image
# boundaries; rows narrower than a thread's pixel stride; the training shape
# (512^2, batch 16: 1024 ranges of 4096 pixels)
@pytest.mark.parametrize("N,H,W,C", [(3, 40, 24, 32), (2, 100, 70, 64), (5, 40, 60, 16), (1, 7, 5, 8),
                                     (16, 512, 512, 32)])
def test_wgrad_first(dsn, N, H, W, C):
    _say("wgrad_first", N, H, W, C)
    rng = np.random.default_rng(3 * N + W + C)
    dz = _bf16(rng.standard_normal((N, H, W, C), dtype=np.float32))
    x = rng.random((N, H, W), dtype=np.float32)
    dw, db = dsn.wgrad_first(dz.cuda(), torch.as_tensor(x).cuda())
    _, dwr, dbr = ref.conv3x3_backward(x.astype(np.float64)[..., None], np.zeros((C, 3, 3, 1)), _np(dz))
    e_w, e_b = _rel(dw.cpu().numpy().astype(np.float64), dwr), _rel(db.cpu().numpy().astype(np.float64), dbr)
    _say("  dw err", e_w, "db err", e_b)
    assert e_w <= 1e-5 and e_b <= 1e-5


@pytest.mark.parametrize("relu_mask", [False, True])
@pytest.mark.parametrize("mod", [False, True])
@pytest.mark.parametrize("B,H,W,C", [(3, 40, 24, 32), (2, 64, 70, 64), (16, 256, 256, 32)])
def test_head_backward(dsn, mod, relu_mask, B, H, W, C):
    _say("head_bwd", mod, relu_mask, B, H, W, C)
    rng = np.random.default_rng(B + H + C + mod)
    npix = B * H * W
    x = _bf16(np.maximum(rng.standard_normal((npix, C), dtype=np.float32), 0))
    w = _bf16(rng.normal(scale=0.3, size=C))
    out = rng.normal(size=npix).astype(np.float32)
    t = rng.normal(size=npix).astype(np.float32)
    kw = {}
    if mod:
        wm = _bf16(rng.normal(scale=0.3, size=C))
        out_m = rng.normal(scale=0.05, size=npix).astype(np.float32)
        t_m = (rng.random(npix) < 0.5).astype(np.float32)
        kw = dict(wm=wm.cuda(), out_m=torch.as_tensor(out_m).cuda(), t_m=torch.as_tensor(t_m).cuda())
    dx, loss, gw = dsn.head_bwd(x.cuda(), w.cuda(), torch.as_tensor(out).cuda(), torch.as_tensor(t).cuda(), B,
                                relu_mask=relu_mask, **kw)
    # oracle: the head is a 1x1 convolution; its loss gradient and L_0 / L_m
    xr = _np(x)
    d0 = out.astype(np.float64) - t
    g = (2.0 / B) * d0
    L0 = float(np.sum(d0 * d0)) / B
    dxr = g[:, None] * _np(w)[None, :]
    gwr = [np.concatenate([g @ xr, [g.sum()]])]
    Lm = 0.0
    if mod:
        z = out_m.astype(np.float64)
        hm = ref.ahf(z) - t_m
        Lm = float(np.sum(hm * hm)) / B
        gm = (2.0 / B) * hm * ref.ahf_grad(z)
        dxr = dxr + gm[:, None] * _np(wm)[None, :]
        gwr.append(np.concatenate([gm @ xr, [gm.sum()]]))
    lo = loss.cpu().numpy()
    _say("  L0", lo[0], L0, "Lm", lo[1], Lm)
    assert abs(lo[0] - L0) <= 1e-6 * L0
    assert abs(lo[1] - Lm) <= 1e-6 * max(Lm, 1e-30) if mod else lo[1] == 0.0
    gwg = gw.cpu().numpy().astype(np.float64)
    for h, r in enumerate(gwr):
        e = _rel(gwg[h], r)
        _say("  head", h, "grad err", e)
        assert e <= 1e-5
    if relu_mask:
        # the features are ReLU outputs: half of them exactly zero
        keep = xr > 0
        assert 0 < np.count_nonzero(keep) < keep.size
        dxr = np.where(keep, dxr, 0.0)
        assert np.all(_np(dx)[~keep] == 0.0)
    err = np.abs(_np(dx) - dxr)
    assert np.all(err <= 2.0 ** -8 * np.abs(dxr) + 1e-5 * np.abs(dxr).max())


@pytest.mark.parametrize("relu_mask", [False, True])
@pytest.mark.parametrize("N,H,W,C", [(2, 16, 24, 32), (3, 40, 24, 64), (1, 128, 130, 256)])
def test_maxpool_backward_bit_exact(dsn, N, H, W, C, relu_mask):
    rng = np.random.default_rng(N + C)
    # coarse values so that windows hold ties (the first maximum wins)
    x = _bf16(rng.integers(-3, 4, size=(N, H, W, C)).astype(np.float32) * 0.5)
    dy = _bf16(rng.standard_normal((N, H // 2, W // 2, C), dtype=np.float32))
    dx0 = _bf16(rng.standard_normal((N, H, W, C), dtype=np.float32))
    dx = dx0.cuda()
    dsn.maxpool2_bwd(x.cuda(), dy.cuda(), dx, relu_mask=relu_mask)
    routed = ref.maxpool2_backward(_np(x), _np(dy))
    want = _round_bf16(dx0.float().numpy() + routed.astype(np.float32))
    if relu_mask:
        want = torch.where(x.float() > 0, want, torch.zeros_like(want))
    assert np.array_equal(_bits(dx), _bits(want))


@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("N,H,W,C", [(2, 16, 24, 32), (3, 40, 24, 64), (1, 256, 130, 128)])
def test_upsample_backward_bit_exact(dsn, N, H, W, C, masked):
    rng = np.random.default_rng(2 * N + C)
    dy = _bf16(rng.standard_normal((N, H, W, C), dtype=np.float32))
    mask = _bf16(np.maximum(rng.standard_normal((N, H // 2, W // 2, C), dtype=np.float32), 0)) if masked else None
    dx = dsn.upsample2_bwd(dy.cuda(), None if mask is None else mask.cuda())
    v = dy.float().numpy().reshape(N, H // 2, 2, W // 2, 2, C)
    s = np.zeros((N, H // 2, W // 2, C), dtype=np.float32)
    for k in range(4):                                  # the kernel's order: row-major children
        s = s + v[:, :, k // 2, :, k % 2, :]
    want = _round_bf16(s)
    if masked:
        want = torch.where(mask.float() > 0, want, torch.zeros_like(want))
    assert np.array_equal(_bits(dx), _bits(want))
    if masked:
        return
    # and the sum is the oracle's (FP64) within one BF16 rounding
    r = ref.upsample2_backward(_np(dy))
    assert np.all(np.abs(_np(dx) - r) <= 2.0 ** -8 * np.abs(r))


@pytest.mark.parametrize("shape", [(2, 16, 24, 32), (3, 7, 9, 64)])
def test_relu_backward_bit_exact(dsn, shape):
    rng = np.random.default_rng(shape[-1])
    d0 = _bf16(rng.standard_normal(shape, dtype=np.float32))
    yv = rng.standard_normal(shape).astype(np.float32)
    yv[..., 0] = 0.0
    yv[..., 1] = -0.0
    y = _bf16(yv)
    d = d0.cuda()
    dsn.relu_bwd(d, y.cuda())
    want = torch.where(y.float() > 0, d0, torch.zeros_like(d0))
    assert np.array_equal(_bits(d), _bits(want))


def test_ops_reject_bad_arguments(dsn):
    x = torch.zeros((2, 8, 8, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(dsn.DsnError):
        dsn.maxpool2_bwd(torch.zeros((2, 8, 7, 32), dtype=torch.bfloat16, device="cuda"),
                         torch.zeros((2, 4, 3, 32), dtype=torch.bfloat16, device="cuda"),
                         torch.zeros((2, 8, 7, 32), dtype=torch.bfloat16, device="cuda"))   # odd W
    with pytest.raises(dsn.DsnError):
        dsn.wgrad_first(torch.zeros((1, 8, 8, 24), dtype=torch.bfloat16, device="cuda"),
                        torch.zeros((1, 8, 8), dtype=torch.float32, device="cuda"))        # C = 24
    # an operand 2 bytes past an aligned address: rejected before any launch
    flat = torch.zeros(2 * 8 * 8 * 32 + 8, dtype=torch.bfloat16, device="cuda")
    off = flat[1:1 + 2 * 8 * 8 * 32].view(2, 8, 8, 32)
    w = torch.zeros((32, 3, 3, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(dsn.DsnError):
        dsn.conv3x3_dgrad(off, w)
    with pytest.raises(dsn.DsnError):
        dsn.conv3x3_wgrad(off, x)
