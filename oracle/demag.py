"""Demagnetisation field of the masked disk (paper Sec. II.B).

``demag_direct`` is the plain definition: for every cell i of the disk,
H_alpha(i) = sum over disk cells j of sum_beta K_alpha,beta(r_i - r_j) m_beta(j).
It costs O(N^2) and is meant for small disks.

``demag_fft`` evaluates the same sum as the paper does, by zero-padded FFT
convolution on a P x P grid with P >= 2D - 1: the kernel is laid out at wrapped
displacements (u mod P, v mod P) for |u|, |v| <= D - 1 and zero elsewhere, its
transform is taken once, and every evaluation transforms m, multiplies, and
transforms back, keeping the D x D box.  With P >= 2D - 1 the circular
convolution equals the linear one, so the two functions agree to rounding.

Arrays are float64 torch tensors shaped [..., 3, D, D] (components x, y, z).
"""
from __future__ import annotations

import torch

from .geometry import Disk
from .greens import kernels


def demag_direct(m: torch.Tensor, disk: Disk) -> torch.Tensor:
    mask = disk.mask
    xs = disk.x[mask]
    ys = disk.y[mask]
    u = xs[:, None] - xs[None, :]                 # r_i - r_j, [N, N]
    v = ys[:, None] - ys[None, :]
    Kxx, Kyy, Kxy, Kzz = kernels(u, v, disk.ell)
    mm = m[..., :, mask]                          # [..., 3, N]
    mx, my, mz = mm[..., 0, :], mm[..., 1, :], mm[..., 2, :]
    hx = mx @ Kxx.T + my @ Kxy.T
    hy = mx @ Kxy.T + my @ Kyy.T
    hz = mz @ Kzz.T
    H = torch.zeros_like(m)
    H[..., 0, mask] = hx
    H[..., 1, mask] = hy
    H[..., 2, mask] = hz
    return H


def kernel_spectra(disk: Disk):
    """Transforms of the four wrapped kernels on the P x P grid (computed once)."""
    cached = getattr(disk, "_oracle_spectra", None)
    if cached is not None:
        return cached
    D, P = disk.D, disk.P
    d = torch.arange(-(D - 1), D, dtype=torch.float64)
    v, u = torch.meshgrid(d, d, indexing="ij")   # rows: y displacement, cols: x displacement
    K = kernels(u, v, disk.ell)
    iv = (v.long() % P)
    iu = (u.long() % P)
    spectra = []
    for k in K:
        w = torch.zeros(P, P, dtype=torch.float64)
        w[iv, iu] = k
        spectra.append(torch.fft.rfft2(w))
    disk._oracle_spectra = tuple(spectra)
    return disk._oracle_spectra


def demag_fft(m: torch.Tensor, disk: Disk) -> torch.Tensor:
    D, P = disk.D, disk.P
    Sxx, Syy, Sxy, Szz = kernel_spectra(disk)
    mm = disk.apply_mask(m)
    F = torch.fft.rfft2(mm, s=(P, P))             # zero-padded transform, [..., 3, P, P/2+1]
    Fx, Fy, Fz = F[..., 0, :, :], F[..., 1, :, :], F[..., 2, :, :]
    G = torch.stack([Sxx * Fx + Sxy * Fy, Sxy * Fx + Syy * Fy, Szz * Fz], dim=-3)
    H = torch.fft.irfft2(G, s=(P, P))[..., :D, :D]
    return disk.apply_mask(H)
