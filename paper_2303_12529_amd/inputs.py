"""Seeded synthetic inputs: Manhattan metal targets and SOCS optical kernels.

This module holds none of the level-set ILT method's arithmetic.  It only
produces the two kinds of input the method consumes:

* a binary target layout Z_t (N x N, uint8), standing in for the ICCAD-2013
  M1 clips the paper evaluates on (Sec. IV, Table I), which are not available;
* a set of K coherent optical kernels H_k (frequency samples on a P x P
  pass-band window) and their weights w_k, standing in for the contest
  litho engine's 24 kernels (Sec. II-B, truncated SOCS with N_k = 24).

The kernels come from a Hopkins transmission cross-coefficient (TCC) built
from an annular source and a circular pupil (with an optional defocus phase),
restricted to the P x P window and decomposed by SVD; the top K
eigen-pairs are kept.  Normalisation: the source weights sum to one, so the
full-rank clear-field intensity is exactly 1 and a resist threshold such as
0.225 is a fraction of the clear field.

Both the test oracle and the GPU path read what this module returns; it is
the only code they share.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "ClipSpec", "C0_CLIP", "C1_CLIP", "gen_clip", "clip_density", "batch_inputs",
    "OpticsSpec", "build_kernels", "build_optics", "optics_checksum",
    "random_phi", "random_mask",
]


# --------------------------------------------------------------------------
# Target clips
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ClipSpec:
    """Recipe for one synthetic Manhattan clip (all lengths in nm)."""
    N: int                       # grid side in pixels
    pitch_nm: float              # pixel pitch
    n_min: int                   # polygon count drawn uniformly in [n_min, n_max]
    n_max: int
    width_nm: tuple              # (lo, hi) wire width
    length_nm: tuple             # (lo, hi) wire length
    spacing_nm: float            # minimum spacing between polygons
    margin_nm: float             # guard band kept empty at the frame edge
    manhattan: bool              # False: rectangles only; True: + L/T unions
    density: tuple | None = None  # if set: add polygons until density ~ U[lo, hi]


# 256 x 256 at 8 nm: 3-6 rectangles, width 10-20 px, length 20-120 px,
# spacing >= 8 px, margin >= 16 px.
C0_CLIP = ClipSpec(N=256, pitch_nm=8.0, n_min=3, n_max=6,
                   width_nm=(80.0, 160.0), length_nm=(160.0, 960.0),
                   spacing_nm=64.0, margin_nm=128.0, manhattan=False)

# 2048 x 2048 at 1 nm: 20-60 Manhattan polygons (rectangles and L/T unions),
# width 40-80 nm, length 80-400 nm, spacing >= 60 nm, margin >= 256 nm.
C1_CLIP = ClipSpec(N=2048, pitch_nm=1.0, n_min=20, n_max=60,
                   width_nm=(40.0, 80.0), length_nm=(80.0, 400.0),
                   spacing_nm=60.0, margin_nm=256.0, manhattan=True)


def _draw_polygon(rng, spec: ClipSpec):
    """One polygon as a list of (y0, x0, y1, x1) half-open pixel boxes
    relative to an anchor at (0, 0)."""
    p = spec.pitch_nm
    w = int(round(rng.uniform(*spec.width_nm) / p))
    length = int(round(rng.uniform(*spec.length_nm) / p))
    w = max(w, 1)
    length = max(length, w)
    horizontal = bool(rng.integers(0, 2))
    if horizontal:
        boxes = [(0, 0, w, length)]
    else:
        boxes = [(0, 0, length, w)]
    if spec.manhattan and rng.uniform() < 0.5:
        # second arm, perpendicular, attached at one end or at the middle
        arm = int(round(rng.uniform(*spec.length_nm) / p / 2))
        arm = max(arm, w)
        where = int(rng.integers(0, 3))          # 0: start, 1: middle, 2: end
        side = 1 if rng.integers(0, 2) else -1    # grow up/left or down/right
        if horizontal:
            xs = [0, (length - w) // 2, length - w][where]
            if side > 0:
                boxes.append((w, xs, w + arm, xs + w))
            else:
                boxes.append((-arm, xs, 0, xs + w))
        else:
            ys = [0, (length - w) // 2, length - w][where]
            if side > 0:
                boxes.append((ys, w, ys + w, w + arm))
            else:
                boxes.append((ys, -arm, ys + w, 0))
    y0 = min(b[0] for b in boxes)
    x0 = min(b[1] for b in boxes)
    return [(b[0] - y0, b[1] - x0, b[2] - y0, b[3] - x0) for b in boxes]


def gen_clip(spec: ClipSpec, seed: int) -> np.ndarray:
    """Draw a seeded Manhattan target; returns uint8 [N, N] with 1 = metal.

    Placement is by rejection: a candidate polygon is accepted only if it
    does not touch the existing metal dilated by the spacing rule, and it
    lies inside the frame minus the margin.
    """
    rng = np.random.default_rng(seed)
    N = spec.N
    p = spec.pitch_nm
    margin = int(np.ceil(spec.margin_nm / p))
    space = int(np.ceil(spec.spacing_nm / p))
    Z = np.zeros((N, N), dtype=np.uint8)
    # "keep-out": metal dilated by the spacing (a square dilation is the
    # conservative Manhattan reading of a spacing rule)
    keep = np.zeros((N, N), dtype=bool)
    if spec.density is None:
        n_target = int(rng.integers(spec.n_min, spec.n_max + 1))
        dens_target = None
    else:
        n_target = 10 ** 9
        dens_target = float(rng.uniform(*spec.density))
    placed = 0
    metal = 0
    attempts = 0
    max_attempts = 200 * max(1, min(n_target, 400))
    misses = 0
    while placed < n_target and attempts < max_attempts:
        attempts += 1
        # density mode: the frame counts as full after 1000 rejections in a row
        if dens_target is not None and misses >= 1000:
            break
        misses += 1
        boxes = _draw_polygon(rng, spec)
        h = max(b[2] for b in boxes)
        w = max(b[3] for b in boxes)
        if h > N - 2 * margin or w > N - 2 * margin:
            continue
        oy = int(rng.integers(margin, N - margin - h + 1))
        ox = int(rng.integers(margin, N - margin - w + 1))
        ok = True
        for (a0, b0, a1, b1) in boxes:
            if keep[oy + a0:oy + a1, ox + b0:ox + b1].any():
                ok = False
                break
        if not ok:
            continue
        for (a0, b0, a1, b1) in boxes:
            metal += int((Z[oy + a0:oy + a1, ox + b0:ox + b1] == 0).sum())
            Z[oy + a0:oy + a1, ox + b0:ox + b1] = 1
            keep[max(0, oy + a0 - space):oy + a1 + space,
                 max(0, ox + b0 - space):ox + b1 + space] = True
        placed += 1
        misses = 0
        if dens_target is not None and metal >= dens_target * N * N:
            break
    return Z


def clip_density(Z: np.ndarray) -> float:
    return float(np.asarray(Z, dtype=np.float64).mean())


def random_mask(N: int, density: float, seed: int) -> np.ndarray:
    """Uniform random 0/1 mask (tests)."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=(N, N)) < density).astype(np.uint8)


def random_phi(N: int, seed: int, scale: float = 8.0) -> np.ndarray:
    """A smooth random level-set function (tests): a sum of a few random
    Gaussian bumps minus a constant, in pixel units."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    phi = np.full((N, N), scale)
    for _ in range(6):
        cy, cx = rng.uniform(0, N, size=2)
        r = rng.uniform(N / 12, N / 5)
        phi -= 2.0 * scale * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * r * r))
    return phi


# --------------------------------------------------------------------------
# Optical kernels (SOCS decomposition of a windowed TCC)
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class OpticsSpec:
    N: int                  # grid side (pixels)
    pitch_nm: float         # pixel pitch; the field is N * pitch nm wide
    P: int                  # odd pass-band window side
    K: int                  # number of kernels kept
    NA: float = 1.35
    wavelength_nm: float = 193.0
    sigma_in: float = 0.6
    sigma_out: float = 0.9
    defocus_nm: float = 0.0
    n_immersion: float = 1.44


def _pupil(fy, fx, spec: OpticsSpec):
    """Circular pupil of radius NA/lambda with a defocus phase."""
    lam = spec.wavelength_nm
    fr2 = fy * fy + fx * fx
    inside = fr2 <= (spec.NA / lam) ** 2 * (1.0 + 1e-12)
    val = inside.astype(np.complex128)
    if spec.defocus_nm != 0.0:
        n = spec.n_immersion
        kz = np.sqrt(np.maximum(n * n - lam * lam * fr2, 0.0))
        val = val * np.exp(1j * 2.0 * np.pi * spec.defocus_nm * (kz - n) / lam)
    return val


def build_kernels(spec: OpticsSpec):
    """Return (kernels [K, P, P] complex128, weights [K] float64).

    kernels[k, a, b] is the frequency sample of kernel k at
    (f_y, f_x) = ((a - c), (b - c)) / (N * pitch), c = (P - 1) // 2.
    """
    if spec.P % 2 != 1:
        raise ValueError("P must be odd")
    P, K = spec.P, spec.K
    c = (P - 1) // 2
    df = 1.0 / (spec.N * spec.pitch_nm)
    lam = spec.wavelength_nm
    # source: grid points (multiples of df) inside the annulus, equal weights
    rmax = int(np.ceil(spec.sigma_out * spec.NA / lam / df)) + 1
    sy, sx = np.mgrid[-rmax:rmax + 1, -rmax:rmax + 1]
    sr = np.hypot(sy, sx) * df
    sel = (sr >= spec.sigma_in * spec.NA / lam) & (sr <= spec.sigma_out * spec.NA / lam)
    sy = sy[sel].astype(np.float64) * df
    sx = sx[sel].astype(np.float64) * df
    ws = np.full(sy.size, 1.0 / sy.size)
    # window frequencies, flattened in (a, b) row-major order
    fa = (np.arange(P) - c) * df
    FY, FX = np.meshgrid(fa, fa, indexing="ij")
    FY = FY.reshape(-1)
    FX = FX.reshape(-1)
    # Q[f, s] = sqrt(w_s) * Pupil(f + s); TCC = Q Q^H on the window
    Q = _pupil(FY[:, None] + sy[None, :], FX[:, None] + sx[None, :], spec) * np.sqrt(ws)[None, :]
    U, sv, _ = np.linalg.svd(Q, full_matrices=False)
    if K > U.shape[1]:
        raise ValueError("K exceeds the TCC rank available on this window")
    U = U[:, :K]
    w = sv[:K] ** 2
    # phase convention: the largest-magnitude entry of each kernel is real > 0
    for k in range(K):
        j = int(np.argmax(np.abs(U[:, k])))
        U[:, k] *= np.conj(U[j, k]) / abs(U[j, k])
    kernels = U.T.reshape(K, P, P).copy()
    return kernels, w.astype(np.float64)


def build_optics(N: int, pitch_nm: float, P: int, K: int, defocus_sets=(0.0,), **kw):
    """Kernel sets for several focus conditions.

    Returns (kernels [n_sets, K, P, P] complex128, weights [n_sets, K]).
    """
    ks, ws = [], []
    for z in defocus_sets:
        k, w = build_kernels(OpticsSpec(N=N, pitch_nm=pitch_nm, P=P, K=K, defocus_nm=z, **kw))
        ks.append(k)
        ws.append(w)
    return np.stack(ks), np.stack(ws)


def optics_checksum(kernels: np.ndarray, weights: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(kernels, dtype=np.complex128).tobytes())
    h.update(np.ascontiguousarray(weights, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# Workload presets (inputs and method settings; plain data only)
# --------------------------------------------------------------------------

def _params(pitch_nm, corners, iters, eta=0.85, lam=0.05, dt_mode=0, reinit_every=5):
    return dict(
        iters=iters, reinit_every=reinit_every, dt_mode=dt_mode, eta=eta,
        dt_max=(0.25 / lam if lam > 0 else 0.0), lam=lam, sigma_z=50.0, i_th=0.225,
        eps_kappa=1e-12, d_lower=-100.0 / pitch_nm, d_upper=900.0 / pitch_nm,
        corners=corners,
    )


NOMINAL_ONLY = [(0, 1.0, 1.0)]
# nominal (alpha = 1), outer (+2 % dose, nominal focus, beta = 7.5),
# inner (-2 % dose, 25 nm defocus, beta = 7.5)
THREE_CORNERS = [(0, 1.0, 1.0), (0, 1.02, 7.5), (1, 0.98, 7.5)]

WORKLOADS = {
    # 256^2 at 8 nm, K = 8, P = 9, nominal only, 20 iterations
    "c0": dict(clip=C0_CLIP, optics=dict(N=256, pitch_nm=8.0, P=9, K=8, defocus_sets=(0.0,)),
               params=_params(8.0, NOMINAL_ONLY, 20)),
    # 2048^2 at 1 nm, K = 24, P = 35, nominal + 25 nm defocus sets, 3 corners, 50 iterations
    "c1": dict(clip=C1_CLIP, optics=dict(N=2048, pitch_nm=1.0, P=35, K=24, defocus_sets=(0.0, 25.0)),
               params=_params(1.0, THREE_CORNERS, 50)),
}


# Batched workload: clips of one 2048 nm field at 512, 1024 or 2048 pixels
# (pitch 4, 2 or 1 nm), so one 35 x 35, K = 24 kernel set pair serves all;
# polygons are added until the metal density reaches U[5 %, 25 %].
BATCH_SIZES = (512, 1024, 2048)
BATCH_FIELD_NM = 2048.0


def batch_clip(N: int, seed: int):
    """(target uint8 [N,N], params dict) of one clip of the batched workload:
    a 2048 nm field at N pixels (pitch 2048/N nm), 50 iterations, three
    corners, TSDF bounds in that pitch's pixels."""
    pitch = BATCH_FIELD_NM / N
    spec = ClipSpec(N=N, pitch_nm=pitch, n_min=1, n_max=1, width_nm=(40.0, 80.0),
                    length_nm=(80.0, 400.0), spacing_nm=60.0, margin_nm=256.0, manhattan=True,
                    density=(0.05, 0.25))
    return gen_clip(spec, seed), _params(pitch, THREE_CORNERS, 50)


def batch_optics():
    """The 35 x 35, K = 24 kernel sets (nominal, 25 nm defocus) of the
    2048 nm field shared by every clip of the batched workload."""
    return build_optics(N=2048, pitch_nm=1.0, P=35, K=24, defocus_sets=(0.0, 25.0))


def batch_inputs(n_clips: int = 64, seed: int = 1234, sizes=BATCH_SIZES):
    """[(target uint8 [N,N], params dict)] for n_clips clips with N drawn
    uniformly from `sizes`, plus (kernels, weights) shared by all."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sizes), size=n_clips)
    clips = [batch_clip(int(N), seed * 1000 + i) for i, N in enumerate(Ns)]
    k, w = batch_optics()
    return clips, k, w


def workload_inputs(name: str, seed: int = 0):
    """(target uint8 [N,N], kernels [n_sets,K,P,P], weights [n_sets,K], params dict)."""
    w = WORKLOADS[name]
    Z = gen_clip(w["clip"], seed)
    k, wt = build_optics(**w["optics"])
    return Z, k, wt, dict(w["params"])


# Full-layout workload: a square layout at 1 nm drawn with the 2048^2 clip
# recipe scaled to its area (polygon count times the area ratio), tiled by
# 2048^2 tiles with a halo of LAYOUT_HALO pixels.
LAYOUT_TILE = 2048
LAYOUT_HALO = 256


def layout_inputs(side: int = 6144, seed: int = 0):
    """(layout uint8 [side, side], kernels, weights, params dict) with the
    optics and loop parameters of the 2048^2 workload."""
    scale = (side / C1_CLIP.N) ** 2
    spec = dataclasses.replace(C1_CLIP, N=side, n_min=int(C1_CLIP.n_min * scale),
                               n_max=int(C1_CLIP.n_max * scale))
    _, k, wt, prm = workload_inputs("c1", 0)
    return gen_clip(spec, seed), k, wt, prm
