"""Host-side analysis of sampled observables (numpy).

* stiffness (Sec. IV.B, eq. Ux): from relaxed energies U(r) with the core held
  at distance r (units of a) from the centre, either the two-point form
  kt = 2 (U(x) - U(0)) / x^2 the paper uses at x = 2a, or a least-squares fit
  U(r) - U(0) = kt r^2/2 + k4 r^4/4;
* gyration rate: slope of the unwrapped azimuth of the core path (signed,
  rad per unit tau); the paper counts revolutions over five to ten periods;
* Thiele prediction in simulation units: Omega = -Q kt / (2 pi) (eqs. wG, OG
  with k_F = kt 2AL/a^2 and G = 2 pi L Ms/gamma);
* Boltzmann forms (Sec. V.C): <r^2> = 2T/kt (eq. r2), p(r) = (kt/T) r
  exp(-kt r^2/(2T)) (eq. pr), and for the rotational speed V = |Omega| r the
  same form with kt -> m_G-equivalent kt/Omega^2 (f(V) = p(V/Omega)/Omega);
* spectra: Bartlett average of periodograms over non-overlapping segments.
Lengths in a, energies in J = 2AL, time in t0, temperature T = kT/J.
"""
from __future__ import annotations

import math

import numpy as np


def stiffness_two_point(U0: float, Ux: float, x: float) -> float:
    return 2.0 * (Ux - U0) / (x * x)


def stiffness_fit(r, dU):
    """(kt, k4) of dU = kt r^2/2 + k4 r^4/4 (points with r > 0)."""
    r = np.asarray(r, dtype=np.float64)
    dU = np.asarray(dU, dtype=np.float64)
    A = np.stack([0.5 * r ** 2, 0.25 * r ** 4], axis=1)
    kt, k4 = np.linalg.lstsq(A, dU, rcond=None)[0]
    return float(kt), float(k4)


def unwrapped_azimuth(x, y):
    return np.unwrap(np.arctan2(np.asarray(y), np.asarray(x)))


def gyration_rate(t, x, y):
    """(Omega, mean radius, revolutions): least-squares slope of the unwrapped azimuth."""
    th = unwrapped_azimuth(x, y)
    t = np.asarray(t, dtype=np.float64)
    A = np.stack([t, np.ones_like(t)], axis=1)
    om, _ = np.linalg.lstsq(A, th, rcond=None)[0]
    return float(om), float(np.mean(np.hypot(x, y))), float(abs(th[-1] - th[0]) / (2 * math.pi))


def thiele_rate(kt: float, Q: int = 1) -> float:
    return -Q * kt / (2.0 * math.pi)


def rayleigh_cdf(r, kt, T):
    return 1.0 - np.exp(-kt * np.asarray(r) ** 2 / (2.0 * T))


def rayleigh_pdf(r, kt, T):
    r = np.asarray(r)
    return kt / T * r * np.exp(-kt * r ** 2 / (2.0 * T))


def ks_distance(samples, cdf):
    s = np.sort(np.asarray(samples).ravel())
    F = cdf(s)
    n = s.size
    return float(max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n)))


def radial_statistics(r, kt, T, bins=12):
    """<r^2> against 2T/kt, the Kolmogorov distance to the Rayleigh law and a histogram."""
    r = np.asarray(r).ravel()
    r2p = 2.0 * T / kt
    hist, edges = np.histogram(r, bins=bins, range=(0.0, 3.0 * math.sqrt(r2p)), density=True)
    mid = 0.5 * (edges[1:] + edges[:-1])
    return {"r2_measured": float(np.mean(r * r)), "r2_predicted": r2p, "ratio": float(np.mean(r * r) / r2p),
            "r_max_predicted": math.sqrt(T / kt), "p_max_predicted": math.exp(-0.5) / math.sqrt(T / kt),
            "ks_distance": ks_distance(r, lambda v: rayleigh_cdf(v, kt, T)),
            "hist_r": mid.tolist(), "hist_p": hist.tolist(), "p_boltzmann": rayleigh_pdf(mid, kt, T).tolist()}


def rotational_speeds(t, x, y, lag):
    """V = r |d theta/dt| with the azimuth rate taken over `lag` samples (centred on
    the midpoint radius) for every replica: x, y are [samples, replicas]."""
    th = np.unwrap(np.arctan2(y, x), axis=0)
    dt = t[lag:] - t[:-lag]
    w = (th[lag:] - th[:-lag]) / dt[:, None]
    xm, ym = 0.5 * (x[lag:] + x[:-lag]), 0.5 * (y[lag:] + y[:-lag])
    return np.abs(w) * np.hypot(xm, ym), w


def angular_momentum_rate(t, x, y, lag):
    """Omega = <x v_y - y v_x> / <r^2> over all samples and replicas, with the
    velocities from centred differences over `lag` samples: the rotation rate
    weighted by r^2, insensitive to the ill-defined azimuth of cores that pass
    near the centre."""
    dt = (t[2 * lag:] - t[:-2 * lag])[:, None]
    vx = (x[2 * lag:] - x[:-2 * lag]) / dt
    vy = (y[2 * lag:] - y[:-2 * lag]) / dt
    xm, ym = x[lag:-lag], y[lag:-lag]
    return float(np.mean(xm * vy - ym * vx) / np.mean(xm * xm + ym * ym))


def bartlett(x, seg: int):
    """Average periodogram of the non-overlapping length-seg segments of the rows of x
    (mean removed per segment, no window); returns (P[k], number of segments)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n = x.shape[1] // seg
    y = x[:, :n * seg].reshape(x.shape[0] * n, seg)
    y = y - y.mean(axis=1, keepdims=True)
    X = np.fft.rfft(y, axis=1)
    return (np.abs(X) ** 2 / seg).mean(axis=0), y.shape[0]
