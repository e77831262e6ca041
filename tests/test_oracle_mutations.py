"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in the oracle (a dropped term, a wrong sign, a wrong
index or evaluation point, a transposed operand) for the duration of the case and
requires a named pin to fail.  The pins themselves are the tests in
test_oracle_cosmology, test_oracle_lpt, test_oracle_pm and test_oracle_cola; nothing
here changes the oracle outside the case.
"""
import pytest

from oracle import cola, lpt, pm
from oracle import cosmology as cosmo
from tests import test_oracle_cola as pins_cola
from tests import test_oracle_cosmology as pins_cosmo
from tests import test_oracle_lpt as pins_lpt
from tests import test_oracle_pm as pins_pm


def _kick_without_second_order(st, i, table, cfg):
    a = float(table.a[i])
    force = cola.pm_force(st.s, a, cfg.np_side, cfg.nm_side, cfg.box, cfg.omega_m)
    acc = force - table.grow["T2D1"][i] * st.s1                       # T^2[D2] s2 dropped
    return cola.State(s=st.s, v=st.v + table.alpha[i] * acc, s1=st.s1, s2=st.s2)


def _kick_with_wrong_sign(st, i, table, cfg):
    a = float(table.a[i])
    force = cola.pm_force(st.s, a, cfg.np_side, cfg.nm_side, cfg.box, cfg.omega_m)
    acc = force + table.grow["T2D1"][i] * st.s1 - table.grow["T2D2"][i] * st.s2
    return cola.State(s=st.s, v=st.v + table.alpha[i] * acc, s1=st.s1, s2=st.s2)


def _drift_without_second_order(st, i, table):
    s = st.s + table.beta[i] * st.v + table.dD1[i] * st.s1             # dD2 s2 dropped
    return cola.State(s=s, v=st.v, s1=st.s1, s2=st.s2)


def _drift_with_next_index(st, i, table):
    j = min(i + 1, len(table.beta) - 1)
    s = st.s + table.beta[i] * st.v + table.dD1[j] * st.s1 + table.dD2[j] * st.s2
    return cola.State(s=s, v=st.v, s1=st.s1, s2=st.s2)


def _finish_without_lplus(st, table, cfg):
    n = cfg.n_steps
    st = cola.kick(st, n, table, cfg)
    x = cola.torch.remainder(cola.lagrangian_grid(cfg.np_side, cfg.box) + st.s, cfg.box)
    return x, st.v, st.s                                                # L+(a_n) dropped


def _lpt_motion_pin():
    with pytest.MonkeyPatch.context() as inner:
        pins_cola.test_lpt_motion_is_integrated_exactly({"n_steps": 3}, inner)


@pytest.mark.parametrize("name,fn", [("kick", _kick_without_second_order), ("kick", _kick_with_wrong_sign),
                                     ("drift", _drift_without_second_order), ("drift", _drift_with_next_index),
                                     ("finish", _finish_without_lplus)])
def test_cola_step_mistakes_are_caught(name, fn, monkeypatch):
    monkeypatch.setattr(cola, name, fn)
    with pytest.raises(AssertionError):
        _lpt_motion_pin()


def test_cic_weights_swapped_are_caught(monkeypatch):
    orig = pm.cic_stencil

    def swapped(u, n_m):
        idx, w = orig(u, n_m)
        return idx, w[[4, 5, 6, 7, 0, 1, 2, 3]]        # (1 - f) and f exchanged along x
    monkeypatch.setattr(pm, "cic_stencil", swapped)
    with pytest.raises(AssertionError):
        pins_pm.test_single_particle_stencils()


def test_gradient_sign_is_caught(monkeypatch):
    orig = pm.gradient_fields
    monkeypatch.setattr(pm, "gradient_fields", lambda rho, box: -orig(rho, box))
    with pytest.raises(AssertionError):
        pins_pm.test_single_mode_potential_and_gradient((2, -1, 5))


def test_transposed_axes_are_caught(monkeypatch):
    orig = pm.mesh_coordinates
    monkeypatch.setattr(pm, "mesh_coordinates", lambda s, n_p, n_m, box: orig(s, n_p, n_m, box)[[1, 0, 2]])
    with pytest.raises(AssertionError):
        pins_pm.test_gather_reproduces_linear_fields()


def test_second_order_lpt_sign_is_caught(monkeypatch):
    orig = lpt.lpt_from_delta_k

    def flipped(dk, n, box):
        s1, s2 = orig(dk, n, box)
        return s1, -s2
    monkeypatch.setattr(lpt, "lpt_from_delta_k", flipped)
    with pytest.raises(AssertionError):
        pins_lpt.test_two_plane_waves_second_order((1, 1, 0), (1, 0, 2))


def test_kick_factor_at_the_wrong_time_is_caught(monkeypatch):
    orig = cosmo.kick_factor
    monkeypatch.setattr(cosmo, "kick_factor", lambda a_i, a_f, a_c, cfg: orig(a_i, a_f, a_f, cfg))
    with pytest.raises(AssertionError):
        pins_cosmo.test_toy_model_is_integrated_exactly(3, -2.5)


def test_drift_factor_at_the_wrong_time_is_caught(monkeypatch):
    orig = cosmo.drift_factor
    monkeypatch.setattr(cosmo, "drift_factor", lambda a_i, a_f, a_c, cfg: orig(a_i, a_f, a_i, cfg))
    with pytest.raises(AssertionError):
        pins_cosmo.test_toy_model_is_integrated_exactly(3, -2.5)


def test_nyquist_modes_kept_are_caught(monkeypatch):
    from oracle import fourier

    def without_nyquist_mask(n):
        nx, ny, nz = fourier.mode_numbers(n)
        return ~((nx == 0) & (ny == 0) & (nz == 0))
    monkeypatch.setattr(pm, "kept_modes", without_nyquist_mask)
    with pytest.raises(AssertionError):
        pins_pm.test_modes_with_a_nyquist_index_give_no_force(1)


def test_force_without_its_time_factor_is_caught(monkeypatch):
    orig = pm.pm_force
    wrong = lambda s, a, n_p, n_m, box, om: orig(s, 1.0, n_p, n_m, box, om)    # (3/2) Om instead of (3/2) Om a
    monkeypatch.setattr(pm, "pm_force", wrong)
    monkeypatch.setattr(cola, "pm_force", wrong)
    with pytest.raises(AssertionError):
        pins_cola.test_zeldovich_plane_wave_converges()


def test_second_order_growth_normalised_once_is_caught(monkeypatch):
    # D2 (and its derivatives) divided by D1raw(1) instead of D1raw(1)^2
    import numpy as np
    orig = cosmo.growth

    def once(a, cfg):
        g = dict(orig(a, cfg))
        raw = float(cosmo._growth_raw(np.array([1.0]), cfg)[0][0])
        for key in ("D2", "TD2", "T2D2"):
            g[key] = g[key] * raw
        return g
    monkeypatch.setattr(cosmo, "growth", once)
    with pytest.raises(AssertionError):
        pins_cosmo.test_d2_matches_standard_fit()


def test_time_variable_with_the_wrong_exponent_is_caught(monkeypatch):
    orig = cosmo.u_of_a
    monkeypatch.setattr(cosmo, "u_of_a", lambda a, cfg: orig(a, cfg) ** -1)   # a^-n instead of a^n
    with pytest.raises(AssertionError):
        pins_cosmo.test_toy_model_is_integrated_exactly(3, -2.5)


def test_unmutated_oracle_passes_the_same_pins():
    # the cases above fail only because of what they plant
    _lpt_motion_pin()
    pins_pm.test_single_particle_stencils()
    pins_pm.test_single_mode_potential_and_gradient((2, -1, 5))
    pins_pm.test_gather_reproduces_linear_fields()
    pins_lpt.test_two_plane_waves_second_order((1, 1, 0), (1, 0, 2))
    pins_cosmo.test_toy_model_is_integrated_exactly(3, -2.5)
    pins_pm.test_modes_with_a_nyquist_index_give_no_force(1)
    pins_cola.test_zeldovich_plane_wave_converges()
    pins_cosmo.test_d2_matches_standard_fit()


# --- spectrum normalisation and second-order growth -----------------------------------
from tests import test_oracle_spectrum as pins_spec   # noqa: E402


def _bbks(k, cfg, gamma, c=(2.34, 3.89, 16.1, 5.46, 6.71)):
    import numpy as np
    q = np.asarray(k, dtype=np.float64) / gamma
    x = c[0] * q
    with np.errstate(divide="ignore", invalid="ignore"):
        lead = np.where(x > 1e-8, np.log1p(x) / np.where(x > 0, x, 1.0), 1.0 - 0.5 * x)
    return lead * (1.0 + c[1] * q + (c[2] * q) ** 2 + (c[3] * q) ** 3 + (c[4] * q) ** 4) ** -0.25


def test_shape_parameter_with_h_squared_is_caught(monkeypatch):
    monkeypatch.setattr(cosmo, "bbks_transfer", lambda k, cfg: _bbks(k, cfg, cfg.omega_m * cfg.h**2))
    with pytest.raises(AssertionError):
        pins_spec.test_bbks_depends_on_k_over_omega_m_h(0.3, 0.7, 0.3, 0.5)
    with pytest.raises(AssertionError):
        pins_spec.test_power_amplitude_matches_independent_value()


@pytest.mark.parametrize("coeffs", [(2.34, 3.98, 16.1, 5.46, 6.71), (2.34, 3.89, 16.1, 5.64, 6.71),
                                    (2.43, 3.89, 16.1, 5.46, 6.71)])
def test_mistyped_transfer_coefficient_is_caught(coeffs, monkeypatch):
    monkeypatch.setattr(cosmo, "bbks_transfer", lambda k, cfg: _bbks(k, cfg, cfg.omega_m * cfg.h, coeffs))
    with pytest.raises(AssertionError):
        pins_spec.test_power_amplitude_matches_independent_value()


def test_tophat_without_its_factor_three_is_caught(monkeypatch):
    orig = cosmo.tophat_window
    monkeypatch.setattr(cosmo, "tophat_window", lambda x: orig(x) / 3.0)
    with pytest.raises(AssertionError):
        with pytest.MonkeyPatch.context() as inner:
            pins_spec.test_tophat_variance_of_white_noise(inner)
    with pytest.raises(AssertionError):
        pins_spec.test_power_amplitude_matches_independent_value()


def test_second_order_growth_off_by_1e4_is_caught(monkeypatch):
    orig = cosmo.growth

    def off(a, cfg):
        g = dict(orig(a, cfg))
        g["D2"] = g["D2"] * (1.0 + 1e-4)
        return g
    monkeypatch.setattr(cosmo, "growth", off)
    with pytest.raises(AssertionError):
        pins_spec.test_d2_matches_variation_of_parameters(0.3, 0.7)
    with pytest.raises(AssertionError):
        pins_spec.test_step_table_matches_independent_values()


def test_unmutated_spectrum_pins_pass():
    with pytest.MonkeyPatch.context() as inner:
        pins_spec.test_tophat_variance_of_white_noise(inner)
    pins_spec.test_bbks_depends_on_k_over_omega_m_h(0.3, 0.7, 0.3, 0.5)
    pins_spec.test_power_amplitude_matches_independent_value()
    pins_spec.test_d2_matches_variation_of_parameters(0.3, 0.7)
    pins_spec.test_step_table_matches_independent_values()
