"""Pins for the oracle's SOCS forward model and adjoint (CPU only).

Each test checks the oracle against something other than its own formula:
numpy's FFT, a naive direct-sum DFT, closed forms (clear field, delta mask,
Parseval), an independent second route (Hopkins/TCC-domain forward, G-window
adjoint), and finite differences (the aerial image is quadratic in M, so a
central difference of a linear functional of I is exact up to rounding).
"""
import numpy as np
import pytest

from oracle import litho
from paper_2303_12529_amd.inputs import build_kernels, OpticsSpec, random_mask


def _rand_kernels(K, P, seed):
    rng = np.random.default_rng(seed)
    H = rng.normal(size=(K, P, P)) + 1j * rng.normal(size=(K, P, P))
    w = rng.uniform(0.1, 1.0, size=K)
    return H, w


def _pad_spectrum(U, N):
    """Place a P x P window array at frequencies (f mod N) of an N x N grid."""
    P = U.shape[0]
    f = litho.window_freqs(P) % N
    out = np.zeros((N, N), dtype=np.complex128)
    out[np.ix_(f, f)] = U
    return out


@pytest.mark.parametrize("N,P", [(8, 3), (8, 5), (16, 5), (16, 9), (32, 9), (13, 5)])
def test_spectrum_matches_numpy_fft(N, P):
    M = random_mask(N, 0.4, seed=N * 100 + P).astype(np.float64)
    A = litho.dft_window_matrix(N, P)
    S = litho.mask_spectrum(M, A)
    F = np.fft.fft2(M)
    f = litho.window_freqs(P) % N
    np.testing.assert_allclose(S, F[np.ix_(f, f)], rtol=0, atol=1e-12 * N * N)


def test_spectrum_matches_naive_sum():
    N, P = 8, 5
    rng = np.random.default_rng(3)
    M = rng.uniform(size=(N, N))
    S = litho.mask_spectrum(M, litho.dft_window_matrix(N, P))
    c = (P - 1) // 2
    for a in range(P):
        for b in range(P):
            fy, fx = a - c, b - c
            acc = 0j
            for y in range(N):
                for x in range(N):
                    ang = -2.0 * np.pi * (fy * y + fx * x) / N
                    acc += M[y, x] * complex(np.cos(ang), np.sin(ang))
            assert abs(S[a, b] - acc) <= 1e-12 * N * N


@pytest.mark.parametrize("N,P", [(8, 3), (16, 5), (32, 9), (24, 7)])
def test_fields_match_numpy_ifft(N, P):
    M = random_mask(N, 0.3, seed=7 + N).astype(np.float64)
    H, _ = _rand_kernels(3, P, seed=P)
    E = litho.socs_fields(M, H)
    F = np.fft.fft2(M)
    f = litho.window_freqs(P) % N
    for k in range(3):
        U = H[k] * F[np.ix_(f, f)]
        ref = np.fft.ifft2(_pad_spectrum(U, N))
        scale = np.abs(ref).max()
        np.testing.assert_allclose(E[k], ref, rtol=0, atol=1e-12 * scale)


def test_parseval():
    N, P = 32, 9
    M = random_mask(N, 0.25, seed=11).astype(np.float64)
    H, _ = _rand_kernels(4, P, seed=12)
    E = litho.socs_fields(M, H)
    S = litho.mask_spectrum(M, litho.dft_window_matrix(N, P))
    for k in range(4):
        lhs = np.sum(np.abs(E[k]) ** 2)
        rhs = np.sum(np.abs(H[k] * S) ** 2) / N ** 2
        assert abs(lhs - rhs) <= 1e-12 * rhs


@pytest.mark.parametrize("N,P,K", [(64, 9, 8), (256, 9, 8), (100, 35, 24)])
def test_clear_field(N, P, K):
    H, w = build_kernels(OpticsSpec(N=N, pitch_nm=2048.0 / N, P=P, K=K))
    I = litho.aerial_image(np.ones((N, N)), H, w)
    c = (P - 1) // 2
    expect = np.sum(w * np.abs(H[:, c, c]) ** 2)
    np.testing.assert_allclose(I, expect, rtol=0, atol=1e-13 * max(1.0, expect))
    # the builder normalises the full-rank clear field to 1; K terms get close
    assert 0.95 < expect <= 1.0 + 1e-12


def test_delta_mask():
    N, P, K = 48, 9, 6
    H, w = _rand_kernels(K, P, seed=5)
    y0, x0 = 13, 29
    M = np.zeros((N, N))
    M[y0, x0] = 1.0
    I = litho.aerial_image(M, H, w)
    ref = np.zeros((N, N))
    for k in range(K):
        h = np.fft.ifft2(_pad_spectrum(H[k], N))
        ref += w[k] * np.abs(np.roll(h, (y0, x0), axis=(0, 1))) ** 2
    np.testing.assert_allclose(I, ref, rtol=0, atol=1e-12 * ref.max())
    total = np.sum(w * np.sum(np.abs(H) ** 2, axis=(1, 2))) / N ** 2
    assert abs(I.sum() - total) <= 1e-12 * total


def test_shift_invariance():
    N, P, K = 40, 7, 4
    H, w = _rand_kernels(K, P, seed=9)
    M = random_mask(N, 0.3, seed=2).astype(np.float64)
    I = litho.aerial_image(M, H, w)
    I2 = litho.aerial_image(np.roll(M, (5, -11), axis=(0, 1)), H, w)
    np.testing.assert_allclose(I2, np.roll(I, (5, -11), axis=(0, 1)), rtol=0, atol=1e-12 * I.max())


@pytest.mark.parametrize("N,P,K", [(32, 5, 3), (40, 9, 5)])
def test_hopkins_route_equals_socs(N, P, K):
    H, w = _rand_kernels(K, P, seed=N + P)
    M = random_mask(N, 0.35, seed=N).astype(np.float64)
    I_socs = litho.aerial_image(M, H, w)
    I_hop = litho.hopkins_aerial_image(M, H, w)
    np.testing.assert_allclose(I_hop, I_socs, rtol=0, atol=1e-11 * I_socs.max())


def test_adjoint_is_gradient_of_linear_functional():
    """d/dM sum(G0 * I(M)) = litho_adjoint(M, G0).  I is quadratic in M, so a
    central difference of this functional is exact up to rounding."""
    N, P, K = 24, 7, 4
    H, w = _rand_kernels(K, P, seed=21)
    rng = np.random.default_rng(22)
    M = rng.uniform(size=(N, N))
    G0 = rng.normal(size=(N, N))
    g = litho.litho_adjoint(M, G0, H, w)

    def F(Mx):
        return float(np.sum(G0 * litho.aerial_image(Mx, H, w)))

    h = 1e-2
    pix = rng.integers(0, N, size=(32, 2))
    scale = np.abs(g).max()
    for (y, x) in pix:
        Mp = M.copy(); Mp[y, x] += h
        Mm = M.copy(); Mm[y, x] -= h
        fd = (F(Mp) - F(Mm)) / (2 * h)
        assert abs(fd - g[y, x]) <= 1e-9 * scale
    # dot-product form along a random direction
    D = rng.normal(size=(N, N))
    fd = (F(M + h * D) - F(M - h * D)) / (2 * h)
    assert abs(fd - np.sum(g * D)) <= 1e-9 * abs(fd) + 1e-9 * scale


def test_adjoint_gwindow_identity():
    N, P, K = 32, 5, 3
    H, w = _rand_kernels(K, P, seed=31)
    rng = np.random.default_rng(32)
    M = random_mask(N, 0.4, seed=33).astype(np.float64)
    G = rng.normal(size=(N, N))
    W1 = litho.socs_adjoint_W(M, G, H, w)
    W2 = litho.gwindow_adjoint_W(M, G, H, w)
    np.testing.assert_allclose(W2, W1, rtol=0, atol=1e-11 * np.abs(W1).max())


def test_adjoint_of_real_kernels_matches_spatial_correlation():
    """With one kernel, dL/dM for L = sum G |M (*) h|^2 is
    2 Re[ conj(h) correlated with (G . E) ]: the paper's H' / H* form."""
    N, P = 16, 5
    H, w = _rand_kernels(1, P, seed=41)
    rng = np.random.default_rng(42)
    M = rng.uniform(size=(N, N))
    G = rng.normal(size=(N, N))
    g = litho.litho_adjoint(M, G, H, w)
    h = np.fft.ifft2(_pad_spectrum(H[0], N))          # spatial kernel, E = M (*) h
    E = np.zeros((N, N), dtype=np.complex128)
    for y in range(N):
        for x in range(N):
            E += M[y, x] * np.roll(h, (y, x), axis=(0, 1))
    X = G * E
    # dL/dM[p] = 2 w Re sum_r X(r) conj(h(r - p))
    ref = np.zeros((N, N))
    for y in range(N):
        for x in range(N):
            ref[y, x] = 2 * w[0] * np.real(np.sum(X * np.conj(np.roll(h, (y, x), axis=(0, 1)))))
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
