"""Power spectra of observable time series (Sec. V.B: the spectrum of <m_x>(tau)
shows the gyrotropic peak and, in larger disks, a pair of spin-wave lines).

The paper does not state its spectral estimator (window, normalisation); the
reading used here is the periodogram of the sampled sequence
  P_k = |sum_t w_t (x_t - xbar) exp(-2 pi i t k / N)|^2 / N,  k = 0 .. N/2,
with xbar the sequence mean (optional) and w either 1 or the periodic Hann
window w_t = sin^2(pi t / N).  A line at frequency f (cycles per unit tau)
sampled every dt appears at bin k = f N dt.  numpy's real FFT is the one
library primitive used.
"""
from __future__ import annotations

import numpy as np


def periodogram(x, remove_mean: bool = True, window: str = "none") -> np.ndarray:
    """P_k, k = 0 .. N/2, of the real sequence x (length N, float64)."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    y = x - x.mean(axis=-1, keepdims=True) if remove_mean else x.copy()
    if window == "hann":
        t = np.arange(N)
        y = y * np.sin(np.pi * t / N) ** 2
    elif window != "none":
        raise ValueError("window: 'none' or 'hann'")
    X = np.fft.rfft(y, axis=-1)
    return (X.real ** 2 + X.imag ** 2) / N


def frequencies(N: int, dt: float) -> np.ndarray:
    """Bin frequencies (cycles per unit tau) of a length-N sequence sampled every dt."""
    return np.arange(N // 2 + 1) / (N * dt)
