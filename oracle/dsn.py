"""FP64 reference of the level-set branch of DevelSet-Net (Sec. III-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper gives the branch as a UNet backbone that maps the target image to
the initial level-set function phi_0 and trains it with the squared error
L_0 = sum_(x,y) (phi_0,theta - phi_gt)^2 against level-set functions produced
by DSO (Sec. III-B, level set branch supervision).  It fixes neither the
layer sizes, the resampling nor the optimiser; the readings used here (and
by the HIP path) are:

* input: the 4 x 4 mean of the binary target (2048^2 -> 512^2), one channel;
* network: four levels with C, 2C, 4C, 8C channels (C = `base`); each level
  has two 3x3 convolutions (zero padding 1, bias, ReLU); 2x2 max-pooling
  between encoder levels; on the way up a nearest 2x upsample, a 3x3
  convolution to the level's width (bias, ReLU), concatenation
  [upsampled | skip] along channels, then the level's two convolutions; a
  1x1 convolution (bias, no ReLU) produces one channel;
* target: the 4 x 4 mean of phi_gt (pixels of the 2048 grid) divided by 100;
* output to DSO: 100 x bilinear 4x upsampling of the prediction with
  half-pixel centres and clamped borders, clipped to the TSDF bounds;
* loss: L_0 per sample (a sum over pixels), averaged over the batch;
* optimiser: Adam (Kingma and Ba) on FP32 master weights.

Modulation branch (Sec. III-B, multi-branch pre-training): a second 1x1 head
on the same backbone output gives phi_m; the branch's map is the
approximated Heaviside m = H_eps(phi_m) = 1/2 (1 + (2/pi) arctan(phi_m/eps))
with eps = 0.03, trained with L_m = sum (H_eps(phi_m) - m_gt)^2 (per sample,
averaged over the batch) next to L_0.  m_gt is the Heaviside of the shifted
ground-truth level set, H(phi_gt + dh) (H(z) = 1 for z >= 0), for the shift
dh whose map, used as DSO's modulation map, gives the lowest L_DSO: the DSO
loss that the loop reaches from TSDF(target) with that map weighting its
curvature term (see `modulation_target`).

Layouts: activations [B][H][W][C] (channels last); convolution weights
[C_out][3][3][C_in]; biases [C_out].
"""
from __future__ import annotations

import numpy as np

SCALE = 100.0


# --------------------------------------------------------------------------
# architecture
# --------------------------------------------------------------------------

EPS_AHF = 0.03


def param_shapes(base: int = 32, levels: int = 4, c_in: int = 1, modulation: bool = False):
    """Ordered (name, weight shape, bias shape) of the level-set branch (and
    the modulation head after it)."""
    ch = [base << i for i in range(levels)]
    out = []
    prev = c_in
    for l in range(levels):
        out.append(("enc%d_a" % l, (ch[l], 3, 3, prev), (ch[l],)))
        out.append(("enc%d_b" % l, (ch[l], 3, 3, ch[l]), (ch[l],)))
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        out.append(("dec%d_up" % l, (ch[l], 3, 3, ch[l + 1]), (ch[l],)))
        out.append(("dec%d_a" % l, (ch[l], 3, 3, 2 * ch[l]), (ch[l],)))
        out.append(("dec%d_b" % l, (ch[l], 3, 3, ch[l]), (ch[l],)))
    out.append(("head", (1, 1, 1, ch[0]), (1,)))
    if modulation:
        out.append(("head_m", (1, 1, 1, ch[0]), (1,)))
    return out


def init_params(seed: int, base: int = 32, levels: int = 4, modulation: bool = False):
    """He-normal weights, zero biases (dict name -> (w, b))."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ws, bs in param_shapes(base, levels, modulation=modulation):
        fan_in = ws[1] * ws[2] * ws[3]
        p[name] = (rng.normal(0.0, np.sqrt(2.0 / fan_in), size=ws), np.zeros(bs))
    return p


# --------------------------------------------------------------------------
# layers (forward)
# --------------------------------------------------------------------------

def conv3x3(x, w, b):
    """y[n,i,j,o] = b[o] + sum_{dy,dx,c} w[o,dy,dx,c] x[n,i+dy-1,j+dx-1,c],
    zero outside the image."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((n, h, wd, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + h, dx:dx + wd, :] @ w[:, dy, dx, :].T
    return y


def conv1x1(x, w, b):
    return x @ w[:, 0, 0, :].T + b


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    n, h, wd, c = x.shape
    return x.reshape(n, h // 2, 2, wd // 2, 2, c).max(axis=(2, 4))


def upsample2(x):
    """Nearest-neighbour 2x: y[2i+a, 2j+b] = x[i, j]."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def mean_pool(x, f):
    """f x f block mean of a 2-D array (or [B, H, W])."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 2:
        return x.reshape(x.shape[0] // f, f, x.shape[1] // f, f).mean(axis=(1, 3))
    return x.reshape(x.shape[0], x.shape[1] // f, f, x.shape[2] // f, f).mean(axis=(2, 4))


def bilinear_up(x, f):
    """Bilinear f x upsampling of a 2-D array: output pixel i samples input
    coordinate (i + 1/2)/f - 1/2, clamped to [0, n-1] (half-pixel centres)."""
    x = np.asarray(x, dtype=np.float64)

    def axis_weights(n):
        t = (np.arange(n * f) + 0.5) / f - 0.5
        t = np.clip(t, 0.0, n - 1.0)
        i0 = np.floor(t).astype(int)
        i1 = np.minimum(i0 + 1, n - 1)
        return i0, i1, t - i0

    y0, y1, fy = axis_weights(x.shape[0])
    x0, x1, fx = axis_weights(x.shape[1])
    top = x[y0][:, x0] * (1 - fx) + x[y0][:, x1] * fx
    bot = x[y1][:, x0] * (1 - fx) + x[y1][:, x1] * fx
    return top * (1 - fy)[:, None] + bot * fy[:, None]


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------

def forward(params, x, levels: int = 4):
    """x [B,H,W,1] -> (out [B,H,W,1], cache of every layer's input/output)."""
    cache = {}
    skips = []
    h = x
    for l in range(levels):
        for part in ("a", "b"):
            name = "enc%d_%s" % (l, part)
            cache[name] = h
            h = relu(conv3x3(h, *params[name]))
            cache[name + ":y"] = h
        if l < levels - 1:
            skips.append(h)
            cache["pool%d" % l] = h
            h = maxpool2(h)
    for l in range(levels - 2, -1, -1):
        u = upsample2(h)
        cache["dec%d_up" % l] = u
        u = relu(conv3x3(u, *params["dec%d_up" % l]))
        cache["dec%d_up:y" % l] = u
        h = np.concatenate([u, skips[l]], axis=-1)
        for part in ("a", "b"):
            name = "dec%d_%s" % (l, part)
            cache[name] = h
            h = relu(conv3x3(h, *params[name]))
            cache[name + ":y"] = h
    cache["head"] = h
    out = conv1x1(h, *params["head"])
    if "head_m" in params:
        out = np.concatenate([out, conv1x1(h, *params["head_m"])], axis=-1)
    return out, cache


def ahf(z, eps=EPS_AHF):
    """Approximated Heaviside 1/2 (1 + (2/pi) arctan(z / eps))."""
    return 0.5 * (1.0 + (2.0 / np.pi) * np.arctan(np.asarray(z, dtype=np.float64) / eps))


def ahf_grad(z, eps=EPS_AHF):
    z = np.asarray(z, dtype=np.float64)
    return (1.0 / np.pi) * eps / (eps * eps + z * z)


def loss(out, target):
    """L_0 per sample, averaged over the batch: mean_b sum_p (out - target)^2."""
    d = out[..., 0] - target
    return float(np.sum(d * d)) / out.shape[0]


def loss_m(out, target_m):
    """L_m per sample, averaged over the batch: mean_b sum_p (H_eps(out_m) - m_gt)^2."""
    d = ahf(out[..., 1]) - target_m
    return float(np.sum(d * d)) / out.shape[0]


# --------------------------------------------------------------------------
# backward
# --------------------------------------------------------------------------

def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 with respect to x, w and b."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    flat = dy.reshape(-1, dy.shape[-1])
    for ky in range(3):
        for kx in range(3):
            sl = xp[:, ky:ky + h, kx:kx + wd, :]
            dw[:, ky, kx, :] = flat.T @ sl.reshape(-1, c)
            dxp[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1, :], dw, flat.sum(axis=0)


def maxpool2_backward(x, dy):
    """Route each output gradient to the first (row-major) maximum of its 2x2 window."""
    n, h, wd, c = x.shape
    blk = x.reshape(n, h // 2, 2, wd // 2, 2, c).transpose(0, 1, 3, 5, 2, 4).reshape(n, h // 2, wd // 2, c, 4)
    arg = blk.argmax(axis=-1)
    dblk = np.zeros_like(blk)
    np.put_along_axis(dblk, arg[..., None], dy[..., None], axis=-1)
    return dblk.reshape(n, h // 2, wd // 2, c, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(n, h, wd, c)


def upsample2_backward(dy):
    n, h, wd, c = dy.shape
    return dy.reshape(n, h // 2, 2, wd // 2, 2, c).sum(axis=(2, 4))


def backward(params, cache, out, target, levels: int = 4, target_m=None):
    """Gradients of loss(out, target) (+ loss_m(out, target_m) when given and
    the network has the modulation head) for every parameter: name -> (dw, db)."""
    B = out.shape[0]
    g = {}
    dout = (2.0 / B) * (out[..., 0] - target)[..., None]
    h = cache["head"]
    wh = params["head"][0]
    g["head"] = ((dout.reshape(-1, 1).T @ h.reshape(-1, h.shape[-1]))[:, None, None, :],
                 dout.reshape(-1, 1).sum(axis=0))
    dh = dout @ wh[:, 0, 0, :]
    if "head_m" in params:
        zm = out[..., 1]
        dm = np.zeros_like(zm) if target_m is None else (2.0 / B) * (ahf(zm) - target_m) * ahf_grad(zm)
        dm = dm[..., None]
        g["head_m"] = ((dm.reshape(-1, 1).T @ h.reshape(-1, h.shape[-1]))[:, None, None, :],
                       dm.reshape(-1, 1).sum(axis=0))
        dh = dh + dm @ params["head_m"][0][:, 0, 0, :]
    dskip = {}
    for l in range(0, levels - 1):
        for part in ("b", "a"):
            name = "dec%d_%s" % (l, part)
            dz = dh * (cache[name + ":y"] > 0)
            dh, dw, db = conv3x3_backward(cache[name], params[name][0], dz)
            g[name] = (dw, db)
        cu = params["dec%d_up" % l][0].shape[0]
        dskip[l] = dh[..., cu:]
        du = dh[..., :cu]
        name = "dec%d_up" % l
        dz = du * (cache[name + ":y"] > 0)
        dx, dw, db = conv3x3_backward(cache[name], params[name][0], dz)
        g[name] = (dw, db)
        dh = upsample2_backward(dx)
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            dh = maxpool2_backward(cache["pool%d" % l], dh) + dskip[l]
        for part in ("b", "a"):
            name = "enc%d_%s" % (l, part)
            dz = dh * (cache[name + ":y"] > 0)
            dh, dw, db = conv3x3_backward(cache[name], params[name][0], dz)
            g[name] = (dw, db)
    return g, dh


# --------------------------------------------------------------------------
# optimiser and resampling of the DSO interface
# --------------------------------------------------------------------------

def adam_step(p, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (p', m', v')."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def net_input(target_2048):
    """Network input: 4 x 4 mean of the binary target."""
    return mean_pool(np.asarray(target_2048, dtype=np.float64), 4)


def net_target(phi_gt_2048):
    """Training target: 4 x 4 mean of phi_gt (2048-grid pixels) / 100."""
    return mean_pool(phi_gt_2048, 4) / SCALE


def phi0_from_output(out_512, d_lower, d_upper):
    """phi_0 for DSO: 100 x bilinear 4x upsampling, clipped to the TSDF bounds."""
    return np.clip(SCALE * bilinear_up(out_512, 4), d_lower, d_upper)


def modulation_target(phi_gt, shifts, loss_of_modulation):
    """m_gt of the modulation branch (Sec. III-B): each candidate is the
    Heaviside map m = H(phi_gt + dh) of the shifted ground truth, and m_gt is
    the candidate with the lowest loss_of_modulation(m), the DSO loss reached
    when DSO runs with m as its modulation map (ties: the first in `shifts`).
    Returns (m_gt, dh)."""
    phi_gt = np.asarray(phi_gt, dtype=np.float64)
    best, best_dh, best_m = None, None, None
    for dh in shifts:
        m = (phi_gt + dh >= 0).astype(np.float64)
        L = loss_of_modulation(m)
        if best is None or L < best:
            best, best_dh, best_m = L, dh, m
    return best_m, best_dh
