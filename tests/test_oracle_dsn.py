"""Pins of the FP64 DevelSet-Net reference (oracle/dsn.py) against library
routines, closed forms and finite differences (no GPU)."""
import numpy as np
import pytest
from scipy import signal

from oracle import dsn


def test_conv3x3_equals_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 9, 7, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = dsn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[n, :, :, o], ref, rtol=0, atol=1e-12)


def test_conv1x1_is_a_channel_matmul():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 4, 5, 6))
    w = rng.normal(size=(2, 1, 1, 6))
    b = rng.normal(size=2)
    y = dsn.conv1x1(x, w, b)
    assert np.allclose(y[0, 2, 3], w[:, 0, 0, :] @ x[0, 2, 3] + b, atol=1e-14)


def test_pool_and_upsample_closed_forms():
    x = np.arange(16, dtype=float).reshape(1, 4, 4, 1)
    assert np.array_equal(dsn.maxpool2(x)[0, :, :, 0], [[5, 7], [13, 15]])
    u = dsn.upsample2(np.array([[1.0, 2.0], [3.0, 4.0]]).reshape(1, 2, 2, 1))[0, :, :, 0]
    assert np.array_equal(u, [[1, 1, 2, 2], [1, 1, 2, 2], [3, 3, 4, 4], [3, 3, 4, 4]])
    # adjoint identities: <up(x), y> = <x, up^T(y)>; pool^T routes to the argmax
    rng = np.random.default_rng(2)
    a = rng.normal(size=(2, 3, 5, 4))
    y = rng.normal(size=(2, 6, 10, 4))
    assert abs(np.sum(dsn.upsample2(a) * y) - np.sum(a * dsn.upsample2_backward(y))) < 1e-12
    x = rng.normal(size=(2, 6, 8, 3))
    dy = rng.normal(size=(2, 3, 4, 3))
    dx = dsn.maxpool2_backward(x, dy)
    assert np.count_nonzero(dx) == dy.size and abs(dx.sum() - dy.sum()) < 1e-12
    # every routed gradient sits on its window's maximum
    mx = dsn.upsample2(dsn.maxpool2(x))
    assert np.all(x[dx != 0] == mx[dx != 0])
    # directional derivative of the max equals the routed gradient
    h = 1e-7
    e = rng.normal(size=x.shape)
    fd = (np.sum(dsn.maxpool2(x + h * e) * dy) - np.sum(dsn.maxpool2(x - h * e) * dy)) / (2 * h)
    assert abs(fd - np.sum(dx * e)) < 1e-6


def test_mean_pool_and_bilinear():
    x = np.arange(64, dtype=float).reshape(8, 8)
    p = dsn.mean_pool(x, 4)
    assert p[0, 0] == np.mean(x[:4, :4]) and p[1, 1] == np.mean(x[4:, 4:])
    # bilinear: constants are preserved, ramps are reproduced away from the
    # clamped border, and the resampling commutes with flips
    c = dsn.bilinear_up(np.full((5, 6), 3.25), 4)
    assert c.shape == (20, 24) and np.all(c == 3.25)
    ramp = np.add.outer(2.0 * np.arange(6), -0.5 * np.arange(7))
    up = dsn.bilinear_up(ramp, 4)
    t_y = (np.arange(24) + 0.5) / 4 - 0.5
    t_x = (np.arange(28) + 0.5) / 4 - 0.5
    inner_y = (t_y >= 0) & (t_y <= 5)
    inner_x = (t_x >= 0) & (t_x <= 6)
    expect = np.add.outer(2.0 * t_y, -0.5 * t_x)
    assert np.allclose(up[np.ix_(inner_y, inner_x)], expect[np.ix_(inner_y, inner_x)], atol=1e-12)
    r = np.random.default_rng(3).normal(size=(5, 7))
    assert np.allclose(dsn.bilinear_up(r[::-1], 4), dsn.bilinear_up(r, 4)[::-1], atol=1e-12)
    # a 2 x 2 input: output row 1 samples t = 3/8 - 1/2 < 0 -> clamped to row 0
    two = dsn.bilinear_up(np.array([[0.0, 8.0], [16.0, 24.0]]), 4)
    assert two[0, 0] == 0.0 and two[7, 7] == 24.0
    assert abs(two[2, 0] - 16.0 * (2.5 / 4 - 0.5)) < 1e-12


def _tiny():
    rng = np.random.default_rng(4)
    p = dsn.init_params(7, base=4, levels=3)
    p = {k: (w, rng.normal(scale=0.1, size=b.shape)) for k, (w, b) in p.items()}
    x = rng.uniform(size=(2, 16, 16, 1))
    t = rng.normal(size=(2, 16, 16))
    return p, x, t


def test_param_shapes_match_the_architecture():
    shapes = dsn.param_shapes(32, 4)
    names = [s[0] for s in shapes]
    assert names[:8] == ["enc0_a", "enc0_b", "enc1_a", "enc1_b", "enc2_a", "enc2_b", "enc3_a", "enc3_b"]
    assert names[8:11] == ["dec2_up", "dec2_a", "dec2_b"] and names[-1] == "head"
    n = sum(int(np.prod(w)) + int(np.prod(b)) for _, w, b in shapes)
    assert 1.8e6 < n < 2.2e6        # about 1.9 M parameters at base 32


def test_backward_matches_finite_differences():
    p, x, t = _tiny()
    out, cache = dsn.forward(p, x, levels=3)
    g, dx = dsn.backward(p, cache, out, t, levels=3)
    rng = np.random.default_rng(5)
    h = 1e-6

    def L(pp, xx):
        return dsn.loss(dsn.forward(pp, xx, levels=3)[0], t)

    for name in ("enc0_a", "enc1_b", "enc2_a", "dec1_up", "dec0_a", "dec0_b", "head"):
        w, b = p[name]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            fd = (L({**p, name: (wp, b)}, x) - L({**p, name: (wm, b)}, x)) / (2 * h)
            assert abs(fd - g[name][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
        j = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        fd = (L({**p, name: (w, bp)}, x) - L({**p, name: (w, bm)}, x)) / (2 * h)
        assert abs(fd - g[name][1][j]) <= 1e-6 * max(1.0, abs(fd)), (name, "bias")
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (L(p, xp) - L(p, xm)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_loss_closed_form():
    out = np.zeros((2, 2, 2, 1))
    t = np.ones((2, 2, 2))
    assert dsn.loss(out, t) == 4.0


def test_adam_closed_forms():
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    # the first step moves every parameter by lr against the sign of its gradient
    p1, m, v = dsn.adam_step(p, g, m, v, 1, lr=1e-3, eps=1e-12)
    assert np.allclose(p - p1, 1e-3 * np.sign(g), atol=1e-12)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    for t in range(2, 6):
        p2, m, v = dsn.adam_step(p1, g, m, v, t, lr=1e-3, eps=1e-12)
        assert np.allclose(p1 - p2, 1e-3 * np.sign(g), atol=1e-10)
        p1 = p2


def test_interface_resampling():
    Z = np.zeros((2048, 2048), dtype=np.uint8)
    Z[100:200, 300:340] = 1
    x = dsn.net_input(Z)
    assert x.shape == (512, 512) and x[30, 80] == 1.0 and x[0, 0] == 0.0 and x.sum() == Z.sum() / 16
    phi = np.full((2048, 2048), 50.0)
    assert np.all(dsn.net_target(phi) == 0.5)
    back = dsn.phi0_from_output(np.full((512, 512), 0.5), -100.0, 900.0)
    assert back.shape == (2048, 2048) and np.all(back == 50.0)
    assert np.all(dsn.phi0_from_output(np.full((4, 4), 20.0), -100.0, 900.0) == 900.0)


def test_ahf_closed_forms():
    assert dsn.ahf(0.0) == 0.5
    assert abs(dsn.ahf(1e9) - 1.0) < 1e-9 and abs(dsn.ahf(-1e9)) < 1e-9
    z = np.linspace(-0.2, 0.2, 11)
    h = 1e-7
    assert np.allclose((dsn.ahf(z + h) - dsn.ahf(z - h)) / (2 * h), dsn.ahf_grad(z), rtol=1e-6)
    # at z = eps the map is 3/4 (arctan 1 = pi/4)
    assert abs(dsn.ahf(dsn.EPS_AHF) - 0.75) < 1e-15


def test_modulation_head_backward_matches_finite_differences():
    rng = np.random.default_rng(21)
    p = dsn.init_params(9, base=4, levels=3, modulation=True)
    p = {k: (w, rng.normal(scale=0.1, size=b.shape)) for k, (w, b) in p.items()}
    x = rng.uniform(size=(2, 16, 16, 1))
    t = rng.normal(size=(2, 16, 16))
    tm = (rng.uniform(size=(2, 16, 16)) < 0.5).astype(float)
    out, cache = dsn.forward(p, x, levels=3)
    assert out.shape[-1] == 2
    g, dx = dsn.backward(p, cache, out, t, levels=3, target_m=tm)

    def L(pp):
        o = dsn.forward(pp, x, levels=3)[0]
        return dsn.loss(o, t) + dsn.loss_m(o, tm)

    h = 1e-6
    for name in ("head_m", "head", "dec0_b", "enc1_a"):
        w, b = p[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            fd = (L({**p, name: (wp, b)}) - L({**p, name: (wm, b)})) / (2 * h)
            assert abs(fd - g[name][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
    bp, bm = p["head_m"][1].copy(), p["head_m"][1].copy()
    bp[0] += h
    bm[0] -= h
    fd = (L({**p, "head_m": (p["head_m"][0], bp)}) - L({**p, "head_m": (p["head_m"][0], bm)})) / (2 * h)
    assert abs(fd - g["head_m"][1][0]) <= 1e-6 * max(1.0, abs(fd))


def test_modulation_target_picks_the_best_shift():
    phi = np.add.outer(np.arange(10.0), np.zeros(4)) - 4.5      # rows 0..4 inside (phi <= 0)
    want = np.zeros_like(phi)
    want[3:, :] = 1.0                                            # H(phi + 2): rows with r - 2.5 >= 0
    m, dh = dsn.modulation_target(phi, [-2, 0, 2, 4], lambda mm: float(np.sum(mm != want)))
    assert dh == 2 and np.array_equal(m, want)
    # ties go to the first candidate; the loss sees the Heaviside map itself
    seen = []
    m, dh = dsn.modulation_target(phi, [4, -2], lambda mm: seen.append(mm.sum()) or 0.0)
    assert dh == 4 and seen == [4.0 * 9, 4.0 * 3]
