"""Shell-averaged power spectrum of a particle distribution (FP64, torch CPU).

Test infrastructure (see ``oracle/__init__``).

Section 3.1 compares models through P(k) of the z = 0 density.  This estimator is
applied identically to any set of final positions (reading; the paper gives no
estimator details):

* CIC deposit of the positions on the Nm^3 cell-centred mesh (the force mesh
  convention), delta = rho / mean(rho) - 1;
* P_b = < |delta_k|^2 > L^3 / Nm^6 over all modes of the full grid with
  round(|n|) = b, 1 <= b <= Nm/2;
* no window deconvolution, no shot-noise subtraction.

Section 3.1 also compares a model's density with the truth's through the
cross-correlation coefficient rho(k) = P_x / sqrt(P_a P_b) (reading: the printed
denominator lacks the square root, which the derivation in Appendix B has) and
n_max(k) = (2/3) rho / sqrt(1 - rho^2), eq. (nmax).  P_x is the shell average of
Re(delta_a,k delta_b,k^*) with the same weights as P.

Pinned in the tests by a single-mode closed form, Parseval's theorem, the mode
counts of the shells, identities of the cross spectrum (rho = +-1 for proportional
fields, bilinearity, symmetry, Cauchy-Schwarz, independent fields uncorrelated) and
the normalisation of eq. (nmax) that Appendix B fixes (n_max = 2 where 10% of the
power is residual).  The paper's figures print no values that could be compared.
"""
from __future__ import annotations

import torch

from .fourier import F64, mode_numbers, rfft3
from .pm import cic_deposit_points


def power_from_delta(delta: torch.Tensor, box: float):
    """(P_b, mode count n_b) for b = 1..N/2 of a real mesh field delta (N^3)."""
    n = delta.shape[-1]
    dk = rfft3(delta.to(F64))
    p = (dk.real**2 + dk.imag**2) * (box**3 / float(n) ** 6)
    nx, ny, nz = mode_numbers(n)
    shell = torch.round(torch.sqrt(nx * nx + ny * ny + nz * nz)).to(torch.int64)
    # modes with 0 < nz < N/2 stand for themselves and their conjugate partner
    mult = torch.full_like(p, 2.0)
    mult[..., 0] = 1.0
    if n % 2 == 0:
        mult[..., n // 2] = 1.0
    nb = n // 2
    shell = shell.expand_as(p).reshape(-1)
    mult = mult.reshape(-1)
    sel = (shell >= 1) & (shell <= nb)
    cnt = torch.zeros(nb + 1, dtype=F64).index_add(0, shell[sel], mult[sel])
    tot = torch.zeros(nb + 1, dtype=F64).index_add(0, shell[sel], (mult * p.reshape(-1))[sel])
    return tot[1:] / cnt[1:], cnt[1:]


def power_of_positions(x, n_m: int, box: float):
    """P_b of points x (3, P), any shape flattening to (3, P), positions in [0, L)."""
    x = torch.as_tensor(x, dtype=F64).reshape(3, -1)
    rho = cic_deposit_points(torch.remainder(x, box), n_m, box)
    delta = rho / rho.mean() - 1.0
    return power_from_delta(delta, box)


def cross_power_from_delta(da: torch.Tensor, db: torch.Tensor, box: float):
    """(P_a, P_b, P_x, n_b) for b = 1..N/2 of two real mesh fields on the same N^3 mesh,
    P_x the shell average of Re(delta_a,k conj(delta_b,k))."""
    n = da.shape[-1]
    ka = rfft3(da.to(F64))
    kb = rfft3(db.to(F64))
    norm = box**3 / float(n) ** 6
    pa = (ka.real**2 + ka.imag**2) * norm
    pb = (kb.real**2 + kb.imag**2) * norm
    px = (ka.real * kb.real + ka.imag * kb.imag) * norm
    nx, ny, nz = mode_numbers(n)
    shell = torch.round(torch.sqrt(nx * nx + ny * ny + nz * nz)).to(torch.int64)
    mult = torch.full_like(pa, 2.0)
    mult[..., 0] = 1.0
    if n % 2 == 0:
        mult[..., n // 2] = 1.0
    nb = n // 2
    shell = shell.expand_as(pa).reshape(-1)
    mult = mult.reshape(-1)
    sel = (shell >= 1) & (shell <= nb)

    def shell_mean(v):
        tot = torch.zeros(nb + 1, dtype=F64).index_add(0, shell[sel], (mult * v.reshape(-1))[sel])
        return tot[1:]

    cnt = torch.zeros(nb + 1, dtype=F64).index_add(0, shell[sel], mult[sel])[1:]
    return shell_mean(pa) / cnt, shell_mean(pb) / cnt, shell_mean(px) / cnt, cnt


def correlation(pa, pb, px):
    """rho = P_x / sqrt(P_a P_b) and n_max = (2/3) rho / sqrt(1 - rho^2), eq. (nmax)."""
    rho = px / torch.sqrt(pa * pb)
    return rho, (2.0 / 3.0) * rho / torch.sqrt(1.0 - rho * rho)


def cross_power_of_positions(xa, xb, n_m: int, box: float):
    """(P_a, P_b, P_x, n_b) of two point sets, each deposited as in power_of_positions."""
    def delta(x):
        x = torch.as_tensor(x, dtype=F64).reshape(3, -1)
        rho = cic_deposit_points(torch.remainder(x, box), n_m, box)
        return rho / rho.mean() - 1.0
    return cross_power_from_delta(delta(xa), delta(xb), box)
