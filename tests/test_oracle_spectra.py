"""Oracle pins: the periodogram of Sec. V.B's spectra (reading in oracle/spectra.py)
against a direct DFT sum, closed forms of a pure tone and of the Hann window,
and Parseval's theorem."""
import math

import numpy as np
import pytest

from oracle.spectra import frequencies, periodogram


def direct(x, remove_mean, hann):
    N = len(x)
    y = np.array(x, dtype=np.float64)
    if remove_mean:
        y = y - sum(y) / N
    if hann:
        y = y * np.array([math.sin(math.pi * t / N) ** 2 for t in range(N)])
    out = []
    for k in range(N // 2 + 1):
        re = sum(y[t] * math.cos(2 * math.pi * t * k / N) for t in range(N))
        im = -sum(y[t] * math.sin(2 * math.pi * t * k / N) for t in range(N))
        out.append((re * re + im * im) / N)
    return np.array(out)


@pytest.mark.parametrize("N", [16, 32, 64])
@pytest.mark.parametrize("rm,win", [(False, "none"), (True, "none"), (True, "hann")])
def test_periodogram_equals_direct_dft(N, rm, win):
    x = np.random.default_rng(N).standard_normal(N) + 0.3
    assert np.allclose(periodogram(x, rm, win), direct(x, rm, win == "hann"), rtol=1e-12, atol=1e-12)


def test_pure_tone_lands_in_its_bin():
    N, k0, A = 256, 19, 0.7
    t = np.arange(N)
    P = periodogram(A * np.cos(2 * np.pi * k0 * t / N + 0.4), True, "none")
    assert abs(P[k0] - A * A * N / 4) < 1e-9
    P[k0] = 0.0
    assert P.max() < 1e-20
    # frequency of the bin for a sampling step dt
    assert abs(frequencies(N, 0.4)[k0] - k0 / (N * 0.4)) < 1e-15


def test_hann_window_of_a_constant():
    # w_t = sin^2(pi t / N) = 1/2 - cos(2 pi t / N)/2: bins 0 and 1 only
    N = 128
    P = periodogram(np.ones(N), False, "hann")
    assert abs(P[0] - (N / 2) ** 2 / N) < 1e-9
    assert abs(P[1] - (N / 4) ** 2 / N) < 1e-9
    assert P[2:].max() < 1e-20


def test_parseval():
    N = 512
    x = np.random.default_rng(3).standard_normal(N)
    P = periodogram(x, True, "none")
    y = x - x.mean()
    two_sided = P[0] + 2 * P[1:N // 2].sum() + P[N // 2]
    assert abs(two_sided - (y * y).sum()) < 1e-9 * (y * y).sum()
