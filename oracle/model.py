"""Forward model of Section II (Eqs. forward model, forward model2, forwardModel).

y_k[n1, n2] = sum_s (x_s * h_{k,s})[n1, n2] + w_k[n1, n2],  k = 1..K, s = 1..S.

Convolutions are circular on the N1 x N2 torus (the boundary assumption under
which the paper diagonalises each H_{k,s} with the 2D DFT, Section IV-A.1).
Kernels are stored unshifted: h[0, 0] is the tap at zero offset.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def _taps(h: np.ndarray):
    """Nonzero taps (m1, m2, value) of a kernel."""
    idx = np.argwhere(h != 0.0)
    return [(int(a), int(b), float(h[a, b])) for a, b in idx]


def conv_circ(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Circular convolution (x * h)[n] = sum_m h[m] x[n - m], in space.

    Direct sum over the kernel's nonzero taps: no FFT is involved, so this is
    independent of every frequency-domain identity the method relies on."""
    out = np.zeros_like(x, dtype=np.float64)
    for a, b, v in _taps(h):
        out += v * np.roll(x, shift=(a, b), axis=(0, 1))
    return out


def corr_circ(y: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Circular correlation sum_m h[m] y[n + m]: the adjoint of ``conv_circ``."""
    out = np.zeros_like(y, dtype=np.float64)
    for a, b, v in _taps(h):
        out += v * np.roll(y, shift=(-a, -b), axis=(0, 1))
    return out


def forward(x: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """H x for x of shape (S, N1, N2) and psf of shape (K, S, N1, N2).

    Eq. forward model without the noise term."""
    K, S = psf.shape[:2]
    y = np.zeros((K,) + x.shape[1:], dtype=np.float64)
    for k in range(K):
        for s in range(S):
            y[k] += conv_circ(x[s], psf[k, s])
    return y


def adjoint(y: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """H^T y: x_s = sum_k corr(y_k, h_{k,s}) (transpose of the block matrix H
    of Eq. forwardModel, whose (k, s) block is the convolution matrix H_{k,s})."""
    K, S = psf.shape[:2]
    x = np.zeros((S,) + y.shape[1:], dtype=np.float64)
    for k in range(K):
        for s in range(S):
            x[s] += corr_circ(y[k], psf[k, s])
    return x


def dense_H(psf: np.ndarray) -> np.ndarray:
    """Explicit H in R^{K N1 N2 x S N1 N2} (Eq. forwardModel), tiny grids only.

    Block (k, s) is the BCCB matrix with entries
    H_{k,s}[(n1, n2), (m1, m2)] = h_{k,s}[(n1 - m1) mod N1, (n2 - m2) mod N2],
    vectorised row-major (n2 fastest)."""
    K, S, N1, N2 = psf.shape
    n = N1 * N2
    i1, i2 = np.divmod(np.arange(n), N2)
    d1 = (i1[:, None] - i1[None, :]) % N1
    d2 = (i2[:, None] - i2[None, :]) % N2
    H = np.zeros((K * n, S * n), dtype=np.float64)
    for k in range(K):
        for s in range(S):
            H[k * n:(k + 1) * n, s * n:(s + 1) * n] = psf[k, s][d1, d2]
    return H


def snr_noise_scale(hx: np.ndarray, snr_db: float) -> np.ndarray:
    """Per-measurement noise standard deviation sigma_k for a target SNR.

    The paper states SNRs (Section V) but not their definition; the reading
    used here is sigma_k = RMS((Hx)_k) * 10^(-SNR/20)."""
    rms = np.sqrt(np.mean(hx.reshape(hx.shape[0], -1) ** 2, axis=1))
    return rms * 10.0 ** (-snr_db / 20.0)


def measure(x: np.ndarray, psf: np.ndarray, unit_noise: np.ndarray,
            snr_db: float) -> np.ndarray:
    """Noisy measurements y = Hx + w with w_k = sigma_k * unit_noise_k."""
    hx = forward(x, psf)
    sig = snr_noise_scale(hx, snr_db)
    return hx + sig[:, None, None] * unit_noise
