"""Pins of the oracle's 2LPT fields (CPU only).

Closed forms: a single plane wave has s1 analytic and S = 0; two plane waves give
S = A B (1 - mu^2) cos(k1 q) cos(k2 q) and the matching s2.  Statistics: the
realised linear field from white noise has the input P(k) on average.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cosmology as cosmo
from oracle import lpt
from oracle.fourier import F64


def _grid(n, box):
    return lpt.lagrangian_grid(n, box)


def test_single_plane_wave():
    n, box, amp = 16, 50.0, 0.3
    q = _grid(n, box)
    nvec = torch.tensor([1.0, 2.0, -1.0], dtype=F64)
    k = 2 * math.pi / box * nvec
    phase = (k.view(3, 1, 1, 1) * q).sum(0)
    delta = amp * torch.cos(phase)
    s1, s2 = lpt.lpt_from_delta(delta, box)
    # delta = -div s1 with s1 = -grad phi, lap phi = delta:  s1 = -A k sin(k.q) / k^2
    expect = -amp * k.view(3, 1, 1, 1) / (k @ k) * torch.sin(phase)
    torch.testing.assert_close(s1, expect, atol=1e-13, rtol=0)
    assert s2.abs().max() < 1e-13


@pytest.mark.parametrize("n1,n2", [((1, 0, 0), (0, 2, 0)), ((1, 1, 0), (1, 0, 2)), ((2, -1, 1), (0, 1, 1))])
def test_two_plane_waves_second_order(n1, n2):
    n, box, A, B = 16, 80.0, 0.4, -0.7
    q = _grid(n, box)
    kf = 2 * math.pi / box
    k1 = kf * torch.tensor(n1, dtype=F64)
    k2 = kf * torch.tensor(n2, dtype=F64)
    p1 = (k1.view(3, 1, 1, 1) * q).sum(0)
    p2 = (k2.view(3, 1, 1, 1) * q).sum(0)
    delta = A * torch.cos(p1) + B * torch.cos(p2)
    s1, s2 = lpt.lpt_from_delta(delta, box)
    mu2 = float((k1 @ k2) ** 2 / ((k1 @ k1) * (k2 @ k2)))
    # phi_ij = A k1i k1j/k1^2 cos p1 + B k2i k2j/k2^2 cos p2  =>
    # S = (tr^2 - tr(Phi^2))/2 = A B (1 - mu^2) cos p1 cos p2
    # phi2 = -(AB(1-mu^2)/2) [cos(p1+p2)/|k1+k2|^2 + cos(p1-p2)/|k1-k2|^2], s2 = grad phi2
    c = 0.5 * A * B * (1.0 - mu2)
    kp, km = k1 + k2, k1 - k2
    expect = c * (kp.view(3, 1, 1, 1) * torch.sin(p1 + p2) / (kp @ kp)
                  + km.view(3, 1, 1, 1) * torch.sin(p1 - p2) / (km @ km))
    torch.testing.assert_close(s2, expect, atol=1e-13, rtol=0)
    s1_expect = -(A * k1.view(3, 1, 1, 1) / (k1 @ k1) * torch.sin(p1)
                  + B * k2.view(3, 1, 1, 1) / (k2 @ k2) * torch.sin(p2))
    torch.testing.assert_close(s1, s1_expect, atol=1e-13, rtol=0)


def test_nyquist_and_mean_modes_are_removed():
    n, box = 8, 10.0
    q = _grid(n, box)
    # a Nyquist wave along x and a constant: both must produce zero displacement
    delta = torch.cos(math.pi * q[0] * n / box) + 0.5
    s1, s2 = lpt.lpt_from_delta(delta, box)
    assert s1.abs().max() < 1e-14 and s2.abs().max() < 1e-14


def test_realised_spectrum_matches_input():
    # <|delta_k|^2> dp^3 / Np^3 = P(k) for delta_k = w_k sqrt(P / dp^3); averaged
    # over all kept modes of 6 seeds the ratio is 1 within sampling error.
    cfg = cosmo.Config(np_side=32)
    n = cfg.np_side
    from oracle.fourier import kept_modes, wavevectors
    _, _, _, k2 = wavevectors(n, cfg.box)
    pk = torch.as_tensor(cosmo.linear_power(torch.sqrt(k2).numpy(), cfg), dtype=F64)
    keep = kept_modes(n)
    ratios = []
    for seed in range(6):
        w = np.random.default_rng(100 + seed).standard_normal(n**3)
        dk = lpt.delta_k_from_noise(w, cfg)
        r = (dk.abs() ** 2) * (cfg.box / n) ** 3 / n**3 / torch.where(keep, pk, torch.ones_like(pk))
        ratios.append(r[keep])
    mean = torch.cat(ratios).mean().item()
    assert abs(mean - 1.0) < 0.02


def test_displacement_divergence_is_minus_delta():
    # delta = -div s1 at first order; check with a centred spectral-free finite
    # difference on a smooth low-mode field (second-order accurate).
    n, box = 64, 100.0
    q = _grid(n, box)
    kf = 2 * math.pi / box
    delta = 0.2 * torch.cos(kf * q[0] + 2 * kf * q[1]) - 0.1 * torch.sin(kf * q[2])
    s1, _ = lpt.lpt_from_delta(delta, box)
    h = box / n
    div = sum((torch.roll(s1[d], -1, d) - torch.roll(s1[d], 1, d)) / (2 * h) for d in range(3))
    err = (div + delta).abs().max().item()
    assert err < 2e-2 * delta.abs().max().item()
