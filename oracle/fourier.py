"""Wavevector grids for periodic boxes (FP64, torch CPU).

Test infrastructure (see ``oracle/__init__``).

The FFT convention is torch's / numpy's: forward transforms are unnormalised,
inverse transforms carry 1/N^3; axes are (x, y, z) in C order and the last axis
of a real-input transform keeps modes nz = 0..N/2.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64


def mode_numbers(n: int):
    """Integer mode numbers (nx, ny, nz) broadcastable to the rfftn half grid."""
    full = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64).round()
    half = torch.arange(n // 2 + 1, dtype=F64)
    return full.view(n, 1, 1), full.view(1, n, 1), half.view(1, 1, n // 2 + 1)


def wavevectors(n: int, box: float):
    """k_x, k_y, k_z = 2 pi n / L (h/Mpc) on the rfftn half grid, and k^2."""
    nx, ny, nz = mode_numbers(n)
    kf = 2.0 * math.pi / box
    kx, ky, kz = kf * nx, kf * ny, kf * nz
    return kx, ky, kz, kx * kx + ky * ky + kz * kz


def kept_modes(n: int):
    """Boolean mask of modes kept by every k-space operator of the method.

    Reading (the paper does not say): the k = 0 mode and every mode with any
    |n_i| = N/2 (a Nyquist index) are set to zero, so that each i*k operator is odd
    and its result is exactly representable as a real field.
    """
    nx, ny, nz = mode_numbers(n)
    nyq = n // 2
    keep = (nx.abs() != nyq) & (ny.abs() != nyq) & (nz.abs() != nyq)
    keep = keep & ~((nx == 0) & (ny == 0) & (nz == 0))
    return keep


def inverse_laplacian(n: int, box: float):
    """Multiplier of d^-2: -1/k^2 on kept modes, 0 elsewhere."""
    _, _, _, k2 = wavevectors(n, box)
    keep = kept_modes(n)
    safe = torch.where(keep, k2, torch.ones_like(k2))
    return torch.where(keep, -1.0 / safe, torch.zeros_like(k2))


def rfft3(x: torch.Tensor) -> torch.Tensor:
    return torch.fft.rfftn(x, dim=(-3, -2, -1))


def irfft3(xk: torch.Tensor, n: int) -> torch.Tensor:
    return torch.fft.irfftn(xk, s=(n, n, n), dim=(-3, -2, -1))
