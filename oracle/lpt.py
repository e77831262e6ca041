"""Second-order Lagrangian perturbation theory displacements s1, s2 (FP64, torch CPU).

Test infrastructure (see ``oracle/__init__``).

Paper passages: Section 2 (2LPT initial conditions computed with standard Fourier
techniques) and Appendix A.3 (s1, s2 are the Zel'dovich and second-order
displacement fields at a = 1, stored per particle).

Conventions (readings, the paper defers 2LPT to the literature):
* delta is the linear density contrast at a = 1 on the particle grid
  q = (i, j, k) * L / Np, z fastest.
* phi solves lap(phi) = delta; s1 = -grad(phi), so delta = -div(s1):
  s1_k = i k delta_k / k^2.
* S = sum_{i<j} (phi_ii phi_jj - phi_ij^2) (no dealiasing), lap(phi2) = S and
  s2 = grad(phi2): s2_k = -i k S_k / k^2.  With this sign D2 is negative
  (D2 ~ -3/7 D1^2) and the second-order term of the trajectory is D2 s2.
* Every k-space operator zeroes k = 0 and every mode with a Nyquist index.

Gaussian field from white noise w ~ N(0, 1) per grid cell: delta_k = w_k
sqrt(P(k) / dp^3), dp = L / Np, which gives <|delta_k|^2> = Np^3 P(k) / dp^3 for
the unnormalised DFT.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import cosmology as cosmo
from .fourier import F64, irfft3, kept_modes, rfft3, wavevectors


def _as_t(x) -> torch.Tensor:
    return torch.as_tensor(np.asarray(x) if not isinstance(x, torch.Tensor) else x).to(F64)


def delta_k_from_noise(w, cfg: cosmo.Config, amplitude: float | None = None) -> torch.Tensor:
    """Half-spectrum of the a = 1 linear field from white noise w (Np^3 values)."""
    n = cfg.np_side
    w = _as_t(w).reshape(n, n, n)
    _, _, _, k2 = wavevectors(n, cfg.box)
    k = torch.sqrt(k2)
    pk = torch.as_tensor(cosmo.linear_power(k.numpy(), cfg, amplitude), dtype=F64)
    dp3 = (cfg.box / n) ** 3
    mult = torch.sqrt(pk / dp3)
    mult = torch.where(kept_modes(n), mult, torch.zeros_like(mult))
    return rfft3(w) * mult


def lpt_from_delta_k(dk: torch.Tensor, n: int, box: float):
    """(s1, s2), each of shape (3, n, n, n), from the half spectrum of delta."""
    kx, ky, kz, k2 = wavevectors(n, box)
    keep = kept_modes(n)
    safe = torch.where(keep, k2, torch.ones_like(k2))
    dk = torch.where(keep, dk, torch.zeros_like(dk))
    kv = (kx, ky, kz)
    s1 = torch.stack([irfft3(1j * kj * dk / safe, n) for kj in kv])
    phi = {}
    for i in range(3):
        for j in range(i, 3):
            phi[i, j] = irfft3(kv[i] * kv[j] * dk / safe, n)
    src = (phi[0, 0] * phi[1, 1] + phi[1, 1] * phi[2, 2] + phi[2, 2] * phi[0, 0]
           - phi[0, 1] ** 2 - phi[1, 2] ** 2 - phi[0, 2] ** 2)
    sk = torch.where(keep, rfft3(src), torch.zeros_like(dk))
    s2 = torch.stack([irfft3(-1j * kj * sk / safe, n) for kj in kv])
    return s1, s2


def lpt_from_delta(delta, box: float):
    """(s1, s2) from a real linear density field on the n^3 particle grid."""
    delta = _as_t(delta)
    n = delta.shape[-1]
    return lpt_from_delta_k(rfft3(delta), n, box)


def lpt_from_noise(w, cfg: cosmo.Config, amplitude: float | None = None):
    """(s1, s2) of the Gaussian field with the BBKS spectrum drawn from noise w."""
    return lpt_from_delta_k(delta_k_from_noise(w, cfg, amplitude), cfg.np_side, cfg.box)


def lagrangian_grid(n: int, box: float) -> torch.Tensor:
    """q = (i, j, k) * L / n as a (3, n, n, n) tensor (corner-registered grid)."""
    ax = torch.arange(n, dtype=F64) * (box / n)
    gx, gy, gz = torch.meshgrid(ax, ax, ax, indexing="ij")
    return torch.stack([gx, gy, gz])


def linear_delta_rms(cfg: cosmo.Config) -> float:
    """rms of the a = 1 linear density over the box modes (diagnostic only)."""
    n = cfg.np_side
    _, _, _, k2 = wavevectors(n, cfg.box)
    pk = torch.as_tensor(cosmo.linear_power(torch.sqrt(k2).numpy(), cfg), dtype=F64)
    pk = torch.where(kept_modes(n), pk, torch.zeros_like(pk))
    w = torch.full_like(pk, 2.0)
    w[..., 0] = 1.0
    return math.sqrt(float((w * pk).sum()) / cfg.box**3)
