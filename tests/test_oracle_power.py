"""Pins of the oracle's shell-averaged power spectrum (CPU only)."""
import math

import pytest
import torch

from oracle import power
from oracle.fourier import F64


@pytest.mark.parametrize("nvec", [(1, 0, 0), (0, 2, 2), (3, -1, 4)])
def test_single_mode_power(nvec):
    # delta = A cos(k.x): the shell of |n| holds total power A^2 L^3 / 2
    n, box, amp = 16, 100.0, 0.2
    ax = (torch.arange(n, dtype=F64) + 0.5) * box / n
    x = torch.stack(torch.meshgrid(ax, ax, ax, indexing="ij"))
    k = 2 * math.pi / box * torch.tensor(nvec, dtype=F64)
    delta = amp * torch.cos((k.view(3, 1, 1, 1) * x).sum(0))
    pk, cnt = power.power_from_delta(delta, box)
    b = round(math.sqrt(sum(v * v for v in nvec)))
    assert (pk[b - 1] * cnt[b - 1]).item() == pytest.approx(amp**2 * box**3 / 2, rel=1e-12)
    others = torch.cat([pk[: b - 1], pk[b:]])
    assert others.abs().max().item() < 1e-20


def test_mode_counts_cover_the_sphere():
    n = 16
    pk, cnt = power.power_from_delta(torch.zeros(n, n, n, dtype=F64), 1.0)
    # number of integer vectors with round(|n|) = b inside the full grid
    full = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64).round()
    nx, ny, nz = torch.meshgrid(full, full, full, indexing="ij")
    sh = torch.round(torch.sqrt(nx**2 + ny**2 + nz**2)).to(torch.int64)
    for b in range(1, n // 2 + 1):
        assert cnt[b - 1].item() == (sh == b).sum().item()
