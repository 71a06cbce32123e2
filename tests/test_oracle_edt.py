"""Pins for the oracle's exact squared EDT and TSDF (CPU only).

Brute force on small masks, scipy's exact EDT (feature indices give exact
integer squared distances) on larger ones, closed forms (single pixel,
empty and full masks), and the paper's Alg. 1 boundary formulation.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import edt
from paper_2303_12529_amd.inputs import gen_clip, C0_CLIP, random_mask


def _brute(cls, want):
    N = cls.shape[0]
    ys, xs = np.nonzero(cls == want)
    out = np.full((N, N), -1, dtype=np.int64)
    if ys.size == 0:
        return out
    yy, xx = np.mgrid[0:N, 0:N]
    d = (yy[..., None] - ys) ** 2 + (xx[..., None] - xs) ** 2
    return d.min(axis=-1).astype(np.int64)


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 24])
@pytest.mark.parametrize("density", [0.01, 0.1, 0.5, 0.9])
def test_sqedt_brute_force(N, density):
    for seed in range(3):
        m = random_mask(N, density, seed=seed * 31 + N)
        for want in (0, 1):
            np.testing.assert_array_equal(edt.sqedt(m, want), _brute(m, want))


def test_sqedt_scipy_exact_indices():
    for seed, N in [(0, 256), (1, 200), (2, 96)]:
        m = random_mask(N, 0.02, seed=seed)
        for want in (0, 1):
            feat = (m == want)
            if not feat.any():
                continue
            # scipy measures distance to the nearest zero of its input
            _, idx = ndi.distance_transform_edt(~feat, return_indices=True)
            yy, xx = np.mgrid[0:N, 0:N]
            ref = (yy - idx[0]) ** 2 + (xx - idx[1]) ** 2
            np.testing.assert_array_equal(edt.sqedt(m, want), ref)


def test_sqedt_clip_against_scipy():
    m = gen_clip(C0_CLIP, 3)
    for want in (0, 1):
        _, idx = ndi.distance_transform_edt(m != want, return_indices=True)
        yy, xx = np.mgrid[0:256, 0:256]
        np.testing.assert_array_equal(edt.sqedt(m, want), (yy - idx[0]) ** 2 + (xx - idx[1]) ** 2)


def test_single_pixel_and_empty_full():
    N = 37
    m = np.zeros((N, N), dtype=np.uint8)
    m[5, 30] = 1
    yy, xx = np.mgrid[0:N, 0:N]
    np.testing.assert_array_equal(edt.sqedt(m, 1), (yy - 5) ** 2 + (xx - 30) ** 2)
    assert (edt.sqedt(np.zeros((N, N), np.uint8), 1) == -1).all()
    assert (edt.sqedt(np.ones((N, N), np.uint8), 0) == -1).all()
    phi, _, _ = edt.tsdf_from_mask(np.zeros((N, N), np.uint8), -12.5, 112.5)
    assert (phi == 112.5).all()
    phi, _, _ = edt.tsdf_from_mask(np.ones((N, N), np.uint8), -12.5, 112.5)
    assert (phi == -12.5).all()


def test_alg1_boundary_formulation():
    """Alg. 1 finds the boundary by shift-and-XOR and takes, per pixel, the
    minimum distance to boundary pieces.  Restricted to boundary pixels of the
    opposite class the minimum is the same: the nearest opposite pixel always
    has a 4-neighbour of the other class."""
    N = 48
    m = random_mask(N, 0.3, seed=4)
    pad = np.pad(m, 1, mode="edge")
    xor = ((pad[1:-1, 1:-1] ^ pad[:-2, 1:-1]) | (pad[1:-1, 1:-1] ^ pad[2:, 1:-1])
           | (pad[1:-1, 1:-1] ^ pad[1:-1, :-2]) | (pad[1:-1, 1:-1] ^ pad[1:-1, 2:]))
    for want in (0, 1):
        cls = np.where((m == want) & (xor == 1), want, 1 - want).astype(np.uint8)
        d_boundary = _brute(cls, want)
        d_all = edt.sqedt(m, want)
        opp = (m != want)
        np.testing.assert_array_equal(d_boundary[opp], d_all[opp])


@pytest.mark.parametrize("seed", range(4))
def test_tsdf_round_trip_and_values(seed):
    m = random_mask(64, 0.3 + 0.1 * seed, seed=seed)
    phi, d_in, d_out = edt.tsdf_from_mask(m, -12.5, 112.5)
    assert np.array_equal(phi <= 0, m == 1)
    assert not np.any(phi == 0)
    out = m == 0
    np.testing.assert_array_equal(phi[out], np.clip(np.sqrt(d_in[out]) - 0.5, -12.5, 112.5))
    np.testing.assert_array_equal(phi[~out], np.clip(0.5 - np.sqrt(d_out[~out]), -12.5, 112.5))
    # re-initialising a re-initialised phi changes nothing
    phi2, _, _ = edt.tsdf_from_phi(phi, -12.5, 112.5)
    np.testing.assert_array_equal(phi2, phi)


def test_tsdf_straight_edge_has_unit_slope():
    N = 32
    m = np.zeros((N, N), dtype=np.uint8)
    m[:, :10] = 1
    phi, _, _ = edt.tsdf_from_mask(m, -100, 900)
    np.testing.assert_array_equal(phi[0, :12], [-9.5, -8.5, -7.5, -6.5, -5.5, -4.5, -3.5, -2.5,
                                                 -1.5, -0.5, 0.5, 1.5])
