"""SOCS lithography imaging and its adjoint, in float64 (test oracle).

Paper: Sec. II-B (Hopkins model approximated by the sum of coherent systems,
I = sum_k w_k |M (*) h_k|^2, truncated to N_k kernels) and Sec. III-A
(the ILT gradient: dL/dM as the sum of the two conjugate convolution terms
with the rotated kernel H' and the conjugate H*).

Conventions (the paper does not fix them; these are the oracle's readings):

* Forward DFT unnormalised, inverse with 1/N^2.  Kernels are frequency
  samples Hhat_k on a P x P window centred on DC, so the clear-field
  intensity is sum_k w_k |Hhat_k(0)|^2.
* A in C^{P x N}: A[a, x] = exp(-2 pi i ((f_a x) mod N) / N), f_a = a - c,
  c = (P - 1) / 2.  The product f_a x is reduced mod N in integers before the
  angle is formed.
* Mask spectrum on the window S = A M A^T  (rows = f_y, columns = f_x).
* Field E_k = N^-2 A^H (Hhat_k . S) conj(A); aerial I = sum_k w_k |E_k|^2.
* Adjoint of M -> E_k:  X -> A^H (conj(Hhat_k) . (N^-2 A X A^T)) conj(A).
  For real M and G = dL/dI:  dL/dM = 2 Re(A^H W conj(A)) with
  W = sum_k w_k conj(Hhat_k) . V_k and V_k = N^-2 A (G . E_k) A^T.
  This is the frequency-domain form of the paper's two conjugate terms
  (the H' (*) [.. (M (*) H*)] and (H')* (*) [.. (M (*) H)] pair sum to 2 Re).
"""
from __future__ import annotations

import numpy as np


def window_freqs(P: int) -> np.ndarray:
    """Integer frequencies f_a = a - (P-1)/2 of the P-wide pass-band window."""
    if P % 2 != 1:
        raise ValueError("window side P must be odd")
    return np.arange(P) - (P - 1) // 2


def dft_window_matrix(N: int, P: int) -> np.ndarray:
    """A[a, x] = exp(-2 pi i ((f_a x) mod N) / N), shape (P, N), complex128."""
    f = window_freqs(P)
    x = np.arange(N)
    phase = np.mod(np.outer(f, x), N)          # integer reduction first
    return np.exp(-2j * np.pi * phase / N)


def mask_spectrum(M: np.ndarray, A: np.ndarray) -> np.ndarray:
    """S = A M A^T: the mask's DFT sampled on the P x P window (Sec. II-B)."""
    M = np.asarray(M, dtype=np.float64)
    return A @ M @ A.T


def socs_fields(M: np.ndarray, kernels: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
    """Coherent fields E_k = N^-2 A^H (Hhat_k . S) conj(A); shape (K, N, N).

    Each E_k is M convolved with the spatial kernel h_k (circular
    convolution), evaluated through the pruned window (Sec. II-B).
    """
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    K, P, _ = kernels.shape
    if A is None:
        A = dft_window_matrix(N, P)
    S = mask_spectrum(M, A)
    AH = A.conj().T
    Ac = A.conj()
    out = np.empty((K, N, N), dtype=np.complex128)
    for k in range(K):
        out[k] = AH @ (kernels[k] * S) @ Ac / (N * N)
    return out


def aerial_image(M: np.ndarray, kernels: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Truncated SOCS aerial image I = sum_k w_k |E_k|^2 (Sec. II-B)."""
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    K, P, _ = kernels.shape
    A = dft_window_matrix(N, P)
    S = mask_spectrum(M, A)
    AH = A.conj().T
    Ac = A.conj()
    I = np.zeros((N, N))
    for k in range(K):
        E = AH @ (kernels[k] * S) @ Ac / (N * N)
        I += weights[k] * (E.real ** 2 + E.imag ** 2)
    return I


def socs_adjoint_W(M: np.ndarray, G: np.ndarray, kernels: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """W = sum_k w_k conj(Hhat_k) . V_k, V_k = N^-2 A (G . E_k) A^T  (P x P).

    This is the window-domain half of the adjoint; the gradient is
    2 Re(A^H W conj(A)) (see ``litho_adjoint``).
    """
    M = np.asarray(M, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    N = M.shape[0]
    K, P, _ = kernels.shape
    A = dft_window_matrix(N, P)
    S = mask_spectrum(M, A)
    AH = A.conj().T
    Ac = A.conj()
    W = np.zeros((P, P), dtype=np.complex128)
    for k in range(K):
        E = AH @ (kernels[k] * S) @ Ac / (N * N)
        V = A @ (G * E) @ A.T / (N * N)
        W += weights[k] * np.conj(kernels[k]) * V
    return W


def window_to_image_real(W: np.ndarray, N: int) -> np.ndarray:
    """2 Re(A^H W conj(A)): back-transform of a window array to a real image."""
    P = W.shape[0]
    A = dft_window_matrix(N, P)
    return 2.0 * (A.conj().T @ W @ A.conj()).real


def litho_adjoint(M: np.ndarray, G: np.ndarray, kernels: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """dL/dM for a loss whose derivative in I is G (Sec. III-A, ILT gradient).

    dL/dM = 2 sum_k w_k Re T_k^H (G . T_k M), T_k M = E_k.
    """
    N = np.asarray(M).shape[0]
    return window_to_image_real(socs_adjoint_W(M, G, kernels, weights), N)


# --------------------------------------------------------------------------
# Second routes (independent formulas used to pin the two above)
# --------------------------------------------------------------------------

def hopkins_aerial_image(M: np.ndarray, kernels: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Aerial image through the Hopkins (TCC) domain instead of K fields.

    With U_k = Hhat_k . S on the window, the image spectrum on the
    (2P-1)^2 difference window is
        Ihat[D] = N^-2 sum_k w_k sum_f U_k[f + D] conj(U_k[f]),
    and I(r) = N^-2 sum_D Ihat[D] exp(+2 pi i D.r / N).
    Requires 2P - 1 <= N so that the difference window does not alias.
    """
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    K, P, _ = kernels.shape
    if 2 * P - 1 > N:
        raise ValueError("difference window aliases: need 2P-1 <= N")
    A = dft_window_matrix(N, P)
    S = mask_spectrum(M, A)
    Q = 2 * P - 1
    Ihat = np.zeros((Q, Q), dtype=np.complex128)
    for k in range(K):
        U = kernels[k] * S
        # Ihat[D] with D = (dy, dx) in [-(P-1), P-1]^2, index D + (P-1)
        for dy in range(-(P - 1), P):
            for dx in range(-(P - 1), P):
                ay0, ay1 = max(0, -dy), min(P, P - dy)
                bx0, bx1 = max(0, -dx), min(P, P - dx)
                s = np.sum(U[ay0 + dy:ay1 + dy, bx0 + dx:bx1 + dx] * np.conj(U[ay0:ay1, bx0:bx1]))
                Ihat[dy + P - 1, dx + P - 1] += weights[k] * s
    Ihat /= N * N
    B = dft_window_matrix(N, Q)                  # rows: D = -(P-1)..(P-1)
    I = (B.conj().T @ Ihat @ B.conj()) / (N * N)
    return I.real


def gwindow_adjoint_W(M: np.ndarray, G: np.ndarray, kernels: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """W through the G-window identity instead of K adjoint fields.

    V_k[f'] = N^-4 sum_f U_k[f] Ghat[f' - f], where Ghat[D] is the DFT of G
    at the difference frequencies D in [-(P-1), P-1]^2.
    """
    M = np.asarray(M, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    N = M.shape[0]
    K, P, _ = kernels.shape
    A = dft_window_matrix(N, P)
    S = mask_spectrum(M, A)
    Q = 2 * P - 1
    B = dft_window_matrix(N, Q)
    Ghat = B @ G @ B.T                          # index D + (P-1)
    W = np.zeros((P, P), dtype=np.complex128)
    for k in range(K):
        U = kernels[k] * S
        V = np.zeros((P, P), dtype=np.complex128)
        for a2 in range(P):
            for b2 in range(P):
                # f' = (a2, b2); f = (a, b); D = f' - f  -> index (a2 - a + P - 1)
                sub = Ghat[a2:a2 + P, b2:b2 + P][::-1, ::-1]
                V[a2, b2] = np.sum(U * sub)
        V /= N ** 4
        W += weights[k] * np.conj(kernels[k]) * V
    return W
