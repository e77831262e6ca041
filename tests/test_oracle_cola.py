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
* Variants: the modified, standard (eq. KDKALCstd) and plain PM (eq. KDKStd)
  schemes converge to one trajectory at second order; the standard COLA scheme
  keeps linear growth exact with few steps, plain PM does not.
* v_res(a_0) = 0 after L-(a_0) (eq. Lops).
* LPT motion is integrated exactly (Section 2 and Appendix A.3: COLA integrates
  only the residual about the LPT trajectory): with the force replaced by the 2LPT
  acceleration T^2[D1] s1 + T^2[D2] s2, every step lands on s = D1 s1 + D2 s2 with
  v_res = 0, and the output velocity is T[D1] s1 + T[D2] s2, for any step count.
  This pins every first- and second-order term of the kick, the drift and L+-.
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


def _plane_wave_run(scheme, n_steps, log_a, n_p=16):
    cfg = cosmo.Config(np_side=n_p, nm_side=n_p, scheme=scheme, n_steps=n_steps, log_a_steps=log_a)
    q = lpt.lagrangian_grid(n_p, cfg.box)
    k = 2 * math.pi / cfg.box
    amp = 0.5 / k
    s1 = torch.zeros(3, n_p, n_p, n_p, dtype=F64)
    s1[0] = amp * torch.sin(k * q[0])
    _, v, s = cola.evolve(s1, torch.zeros_like(s1), cfg)
    return s, v, amp


def test_all_schemes_converge_to_one_trajectory():
    # eqs. (KDKALC), (KDKALCstd) and (KDKStd) discretise the same equation of
    # motion T^2[s] = F(s, a) with the same mesh force, so with more steps each
    # approaches one trajectory, at second order in the step, on either grid.
    s_ref, v_ref, amp = _plane_wave_run("modified", 160, False)
    vscale = v_ref.abs().max().item()
    for scheme in ("pm", "standard", "modified"):
        for log_a in (False, True):
            errs = []
            for n in (20, 80):
                s, v, _ = _plane_wave_run(scheme, n, log_a)
                errs.append(max((s - s_ref).abs().max().item() / amp, (v - v_ref).abs().max().item() / vscale))
            assert errs[1] < 5e-4, (scheme, log_a, errs)
            assert errs[0] / errs[1] > 6.0, (scheme, log_a, errs)


def test_standard_cola_exact_in_linear_regime_and_pm_is_not():
    # Both COLA discretisations take the linear growth from D1, D2 and leave only
    # the (here vanishing) residual to the steps: 3 standard steps give the same
    # lowest-shell growth as 10 modified steps, up to the PM force error.  The plain
    # PM leapfrog (eq. KDKStd) integrates the growth itself and carries a step error;
    # uniform in log a it does better than uniform in a (Appendix A.2).
    d_mod = _linear_growth_deviation_cfg(32, 1)
    d_std = _linear_growth_deviation_cfg(32, 1, scheme="standard", n_steps=3)
    d_pm_a = _linear_growth_deviation_cfg(32, 1, scheme="pm", n_steps=10)
    d_pm_log = _linear_growth_deviation_cfg(32, 1, scheme="pm", n_steps=10, log_a_steps=True)
    d_u1 = _linear_growth_deviation_cfg(32, 1, u1_drift=True, n_steps=3)
    assert abs(d_mod) < 0.04
    assert abs(d_std - d_mod) < 0.01
    assert abs(d_u1 - d_mod) < 0.01
    assert abs(d_pm_a - d_mod) > 0.01
    assert abs(d_pm_log - d_mod) < 0.5 * abs(d_pm_a - d_mod)


def _linear_growth_deviation_cfg(n_p, ratio, seed=1301, **kw):
    cfg = cosmo.Config(np_side=n_p, nm_side=ratio * n_p, **kw)
    w = np.random.default_rng(seed).standard_normal(n_p**3)
    amp = cosmo.power_amplitude(cfg) * 1e-8
    s1, s2 = lpt.lpt_from_noise(w, cfg, amp)
    tab = cosmo.step_table(cfg)
    st0 = cola.initial_state(s1, s2, tab)
    x, _, _ = cola.evolve(s1, s2, cfg, tab)
    q = lpt.lagrangian_grid(n_p, cfg.box)
    p0, _ = power.power_of_positions(q + st0.s, n_p, cfg.box)
    p1, _ = power.power_of_positions(x, n_p, cfg.box)
    return float(p1[0] / p0[0] / ((tab.grow["D1"][-1] / tab.grow["D1"][0]) ** 2) - 1.0)


def test_pm_state_carries_the_full_velocity():
    # eq. (KDKStd) is eq. (KDKALCstd) with s1 = s2 = 0: no L-, the state starts with
    # the 2LPT velocity T[s](a_0) and its LPT fields are zero.
    cfg = cosmo.Config(np_side=8, nm_side=8, scheme="pm")
    w = np.random.default_rng(5).standard_normal(8**3)
    s1, s2 = lpt.lpt_from_noise(w, cfg)
    tab = cosmo.step_table(cfg)
    st = cola.initial_state(s1, s2, tab, lpt_frame=False)
    g = tab.grow
    assert torch.equal(st.v, g["TD1"][0] * s1 + g["TD2"][0] * s2)
    assert st.s1.abs().max().item() == 0.0 and st.s2.abs().max().item() == 0.0


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


@pytest.mark.parametrize("kw", [{"n_steps": 10}, {"n_steps": 3}, {"n_steps": 7, "n_lpt": 1.5},
                                {"scheme": "standard", "n_steps": 4}, {"log_a_steps": True, "n_steps": 5},
                                {"u1_drift": True, "n_steps": 6}, {"omega_m": 0.25, "omega_l": 0.75}])
def test_lpt_motion_is_integrated_exactly(kw, monkeypatch):
    cfg = cosmo.Config(np_side=8, nm_side=16, **kw)
    tab = cosmo.step_table(cfg)
    g = torch.Generator().manual_seed(5)
    s1 = torch.randn(3, 8, 8, 8, generator=g, dtype=F64)
    s2 = 0.3 * torch.randn(3, 8, 8, 8, generator=g, dtype=F64)

    def lpt_acceleration(s, a, *args):
        gr = cosmo.growth([a], cfg)
        return float(gr["T2D1"][0]) * s1 + float(gr["T2D2"][0]) * s2

    monkeypatch.setattr(cola, "pm_force", lpt_acceleration)
    x, v_phys, s, states = cola.evolve(s1, s2, cfg, tab, keep_states=True)
    D1, D2 = tab.grow["D1"], tab.grow["D2"]
    scale = float(s1.abs().max())
    for i, st in enumerate(states):
        assert (st.s - (D1[i] * s1 + D2[i] * s2)).abs().max().item() < 1e-12 * scale, i
        assert st.v.abs().max().item() < 1e-12 * scale, i
    n = cfg.n_steps
    assert (s - (D1[n] * s1 + D2[n] * s2)).abs().max().item() < 1e-12 * scale
    v_lpt = tab.grow["TD1"][n] * s1 + tab.grow["TD2"][n] * s2
    assert (v_phys - v_lpt).abs().max().item() < 1e-12 * scale
    x_lpt = torch.remainder(lpt.lagrangian_grid(8, cfg.box) + D1[n] * s1 + D2[n] * s2, cfg.box)
    d = x - x_lpt
    d = d - cfg.box * torch.round(d / cfg.box)
    assert d.abs().max().item() < 1e-12 * cfg.box
