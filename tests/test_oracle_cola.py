"""Pins of the oracle's COLA evolution (CPU only).

* Linear growth (Section 2: the large scales follow the exact growth factor for
  any number of steps): at tiny amplitude the final P(k) at the lowest shell is
  (D1(1)/D1(a_0))^2 times the initial one, up to the PM force error, which must
  vanish as the resolution grows, at second order in k dp for odd mesh/particle
  ratios and first order for even ones (the particle lattice's image at the
  mesh Nyquist frequency is treated asymmetrically by the spectral gradient).
* Zel'dovich motion of a 1D plane wave is exact before shell crossing: x = q +
  D1(a) s1; the deviation is the PM force error and falls with resolution.
* Momentum: sum of v_res and of s_res stay zero.
* v_res(a_0) = 0 after L-(a_0) (eq. Lops).
* 2LPT sign convention: the Eulerian density of x = q + D1 s1 + D2 s2 at second
  order reproduces the perturbation-theory kernel
  F2(k1, k2) = 5/7 + mu/2 (k1/k2 + k2/k1) + 2/7 mu^2 (Einstein-de Sitter).
"""
import math

import numpy as np
import pytest
import torch

from oracle import cola, lpt, power
from oracle import cosmology as cosmo
from oracle.fourier import F64, irfft3, rfft3, wavevectors


def _linear_growth_deviation(n_p, ratio, seed=1301):
    cfg = cosmo.Config(np_side=n_p, nm_side=ratio * n_p)
    w = np.random.default_rng(seed).standard_normal(n_p**3)
    amp = cosmo.power_amplitude(cfg) * 1e-8      # |s| << cell: linear regime
    s1, s2 = lpt.lpt_from_noise(w, cfg, amp)
    tab = cosmo.step_table(cfg)
    st0 = cola.initial_state(s1, s2, tab)
    x, _, _ = cola.evolve(s1, s2, cfg, tab)
    q = lpt.lagrangian_grid(n_p, cfg.box)
    p0, _ = power.power_of_positions(q + st0.s, n_p, cfg.box)
    p1, _ = power.power_of_positions(x, n_p, cfg.box)
    target = (tab.grow["D1"][-1] / tab.grow["D1"][0]) ** 2
    return float(p1[0] / p0[0] / target - 1.0)


def test_linear_growth_odd_ratio_second_order():
    d32 = _linear_growth_deviation(32, 1)
    d64 = _linear_growth_deviation(64, 1)
    assert abs(d64) < 1e-2
    assert 3.0 < d32 / d64 < 5.0


def test_linear_growth_even_ratio_first_order():
    d16 = _linear_growth_deviation(16, 2)
    d32 = _linear_growth_deviation(32, 2)
    assert abs(d32) < 0.08
    assert 1.6 < d16 / d32 < 2.4


def _zeldovich_deviation(n_p, ratio):
    cfg = cosmo.Config(np_side=n_p, nm_side=ratio * n_p)
    q = lpt.lagrangian_grid(n_p, cfg.box)
    k = 2 * math.pi / cfg.box
    amp = 0.5 / k                      # D1(1) A k = 0.5 < 1: no shell crossing
    s1 = torch.zeros(3, n_p, n_p, n_p, dtype=F64)
    s1[0] = amp * torch.sin(k * q[0])
    x, _, s = cola.evolve(s1, torch.zeros_like(s1), cfg)
    return ((s - s1).abs().max() / amp).item()


def test_zeldovich_plane_wave_converges():
    d = [_zeldovich_deviation(n, 1) for n in (16, 32, 64)]
    assert d[0] / d[1] > 1.8 and d[1] / d[2] > 1.8
    assert d[2] < 0.02


def test_momentum_and_initial_velocity():
    cfg = cosmo.Config()
    n = cfg.np_side
    w = np.random.default_rng(1301).standard_normal(n**3)
    s1, s2 = lpt.lpt_from_noise(w, cfg)
    tab = cosmo.step_table(cfg)
    x, v, s, states = cola.evolve(s1, s2, cfg, tab, keep_states=True)
    assert states[0].v.abs().max().item() == 0.0
    for st in states[1:]:
        tot = st.v.reshape(3, -1).sum(1).abs().max().item()
        assert tot < 1e-10 * st.v.abs().sum().item()
        # sum s1 = sum s2 = 0, so sum s = sum s_res
        tot_s = st.s.reshape(3, -1).sum(1).abs().max().item()
        assert tot_s < 1e-10 * st.s.abs().sum().item()
    assert x.min().item() >= 0.0 and x.max().item() < cfg.box


@pytest.mark.parametrize("n1,n2", [((1, 0, 0), (0, 1, 0)), ((1, 1, 0), (1, 0, 0)), ((2, 1, 0), (-1, 1, 1))])
def test_2lpt_reproduces_second_order_kernel(n1, n2):
    eds = cosmo.Config(omega_m=1.0, omega_l=0.0)
    g = cosmo.growth([0.5], eds)
    d2_over_d1sq = g["D2"][0] / g["D1"][0] ** 2          # -3/7 in EdS
    n, box, A, B = 32, 100.0, 0.3, 0.2
    q = lpt.lagrangian_grid(n, box)
    kf = 2 * math.pi / box
    k1 = kf * torch.tensor(n1, dtype=F64)
    k2 = kf * torch.tensor(n2, dtype=F64)
    p1 = (k1.view(3, 1, 1, 1) * q).sum(0)
    p2 = (k2.view(3, 1, 1, 1) * q).sum(0)
    dl = A * torch.cos(p1) + B * torch.cos(p2)
    s1, s2 = lpt.lpt_from_delta(dl, box)
    # spectral derivatives of the oracle's fields
    kx, ky, kz, _ = wavevectors(n, box)
    kv = (kx, ky, kz)
    d = lambda f, j: irfft3(1j * kv[j] * rfft3(f), n)
    grad_s1 = [[d(s1[i], j) for j in range(3)] for i in range(3)]
    div_s2 = sum(d(s2[j], j) for j in range(3))
    tr2 = sum(grad_s1[i][j] * grad_s1[j][i] for i in range(3) for j in range(3))
    grad_dl = [d(dl, j) for j in range(3)]
    # Eulerian density at second order, per D1^2:
    # -(D2/D1^2) div s2 + (delta^2 + s1_ij s1_ji)/2 - s1 . grad delta
    d2 = -d2_over_d1sq * div_s2 + 0.5 * (dl * dl + tr2) - sum(s1[j] * grad_dl[j] for j in range(3))
    for kk, sgn in ((k1 + k2, 1.0), (k1 - k2, -1.0)):
        proj = 2.0 * (d2 * torch.cos((kk.view(3, 1, 1, 1) * q).sum(0))).mean().item()
        ka, kb = k1, sgn * k2
        mu = float(ka @ kb) / math.sqrt(float(ka @ ka) * float(kb @ kb))
        ra = math.sqrt(float(ka @ ka) / float(kb @ kb))
        f2 = 5.0 / 7.0 + 0.5 * mu * (ra + 1.0 / ra) + 2.0 / 7.0 * mu * mu
        assert proj == pytest.approx(f2 * A * B, rel=1e-9, abs=1e-12)
