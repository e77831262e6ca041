"""Particle-mesh force of eq. (eom): -(3/2) Om a d_x d_x^-2 delta  (FP64, torch CPU).

Test infrastructure (see ``oracle/__init__``).

Paper passages: Section 2 (a PM code, forces on a mesh finer than the particle
grid), Appendix A.1 eq. (eom) (the force), Appendix A.3.2 eq. (KDKALC) (the
force evaluated at a_c inside the kick).

Readings (the paper names neither the assignment scheme nor the Green's function):
* Cloud-in-cell assignment on a cell-centred periodic mesh: mesh value c is the
  cell centred at (c + 1/2) * L/Nm.  A particle at x has mesh coordinate
  u = x / dx - 1/2 (mod Nm); with i = floor(u), f = u - i it gives weight
  (1 - f) to cell i and f to cell i + 1 along each axis, the product over axes.
  Mass per particle (Nm/Np)^3, so the mean density is 1 per cell.
* Continuum Poisson kernel -1/k^2 and spectral gradient i k; k = 0 and every
  Nyquist-index mode are zero; no window deconvolution or extra softening.
* The force is interpolated back with the same cloud-in-cell weights.

With those readings g = i k delta_k / k^2 is minus the gradient of d^-2 delta, and
the force of eq. (eom) is F = (3/2) Om a * g, interpolated to the particles.
"""
from __future__ import annotations

import torch

from .fourier import F64, irfft3, kept_modes, rfft3, wavevectors
from .lpt import lagrangian_grid


def mesh_coordinates(s: torch.Tensor, n_p: int, n_m: int, box: float) -> torch.Tensor:
    """u = (q + s) / dx - 1/2 for displacements s of shape (3, Np, Np, Np)."""
    q = lagrangian_grid(n_p, box)
    return (q + s) * (n_m / box) - 0.5


def cic_stencil(u: torch.Tensor, n_m: int):
    """The 8 (flat cell index, weight) pairs of every particle.

    u: (3, P) mesh coordinates.  Returns idx (8, P) int64 and w (8, P) float64.
    floor() is piecewise constant, so autograd differentiates through the weights.
    """
    i0 = torch.floor(u)
    f = u - i0
    i0 = i0.to(torch.int64)
    idx, wts = [], []
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                cx = torch.remainder(i0[0] + dx, n_m)
                cy = torch.remainder(i0[1] + dy, n_m)
                cz = torch.remainder(i0[2] + dz, n_m)
                wx = f[0] if dx else 1.0 - f[0]
                wy = f[1] if dy else 1.0 - f[1]
                wz = f[2] if dz else 1.0 - f[2]
                idx.append((cx * n_m + cy) * n_m + cz)
                wts.append(wx * wy * wz)
    return torch.stack(idx), torch.stack(wts)


def cic_deposit(s: torch.Tensor, n_p: int, n_m: int, box: float) -> torch.Tensor:
    """Density rho (Nm, Nm, Nm), mean 1, of particles at q + s."""
    u = mesh_coordinates(s, n_p, n_m, box).reshape(3, -1)
    idx, w = cic_stencil(u, n_m)
    mass = (n_m / n_p) ** 3
    rho = torch.zeros(n_m**3, dtype=F64)
    rho = rho.index_add(0, idx.reshape(-1), (w * mass).reshape(-1))
    return rho.reshape(n_m, n_m, n_m)


def cic_deposit_points(x: torch.Tensor, n_m: int, box: float, mass: float = 1.0) -> torch.Tensor:
    """CIC density of arbitrary points x (3, P) in [0, L) (same convention)."""
    u = x.reshape(3, -1) * (n_m / box) - 0.5
    idx, w = cic_stencil(u, n_m)
    rho = torch.zeros(n_m**3, dtype=F64)
    rho = rho.index_add(0, idx.reshape(-1), (w * mass).reshape(-1))
    return rho.reshape(n_m, n_m, n_m)


def gradient_fields(rho: torch.Tensor, box: float) -> torch.Tensor:
    """g_j = irfft(i k_j rho_k / k^2), shape (3, Nm, Nm, Nm); k = 0 and Nyquist zeroed."""
    n = rho.shape[-1]
    kx, ky, kz, k2 = wavevectors(n, box)
    keep = kept_modes(n)
    safe = torch.where(keep, k2, torch.ones_like(k2))
    rk = rfft3(rho)
    rk = torch.where(keep, rk, torch.zeros_like(rk))
    return torch.stack([irfft3(1j * kj * rk / safe, n) for kj in (kx, ky, kz)])


def potential_field(rho: torch.Tensor, box: float) -> torch.Tensor:
    """d^-2 delta on the mesh (diagnostic; the method only needs its gradient)."""
    n = rho.shape[-1]
    _, _, _, k2 = wavevectors(n, box)
    keep = kept_modes(n)
    safe = torch.where(keep, k2, torch.ones_like(k2))
    rk = torch.where(keep, rfft3(rho), torch.zeros_like(k2, dtype=torch.complex128))
    return irfft3(-rk / safe, n)


def cic_gather(fields: torch.Tensor, s: torch.Tensor, n_p: int, box: float) -> torch.Tensor:
    """Interpolate mesh fields (c, Nm, Nm, Nm) to the particles; returns (c, P)."""
    n_m = fields.shape[-1]
    u = mesh_coordinates(s, n_p, n_m, box).reshape(3, -1)
    idx, w = cic_stencil(u, n_m)
    flat = fields.reshape(fields.shape[0], -1)
    return (flat[:, idx] * w.unsqueeze(0)).sum(dim=1)


def pm_force(s: torch.Tensor, a: float, n_p: int, n_m: int, box: float, omega_m: float) -> torch.Tensor:
    """F = (3/2) Om a g at every particle, shape (3, Np, Np, Np); s is (3, Np, Np, Np)."""
    rho = cic_deposit(s, n_p, n_m, box)
    g = gradient_fields(rho, box)
    f = cic_gather(g, s, n_p, box)
    return (1.5 * omega_m * a) * f.reshape(3, n_p, n_p, n_p)
