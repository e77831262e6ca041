"""Pins of the oracle's background, growth and step coefficients (CPU only).

Each check compares the oracle against something other than itself: closed forms
of the Einstein-de Sitter case, the Heath integral for D1, the standard D2 fit,
the toy-model exactness of the modified kick/drift (Appendix A.3.2, eq. toyKDK)
integrated independently, the exact cases and second-order convergence of the
standard kick/drift (eqs. KDKStd, KDKALCstd), and the constants the paper states.
"""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import cosmology as cosmo

LCDM = cosmo.Config()
EDS = cosmo.Config(omega_m=1.0, omega_l=0.0)


def test_eds_growth_closed_forms():
    # Omega_m = 1: D1 = a, T[D1] = a^(3/2), T^2[D1] = (3/2) a^2,
    # D2 = -3/7 a^2, T[D2] = -(6/7) a^(5/2), T^2[D2] = -(15/7) a^3.
    a = np.array([0.05, 0.1, 0.37, 0.64, 1.0])
    g = cosmo.growth(a, EDS)
    np.testing.assert_allclose(g["D1"], a, rtol=1e-10)
    np.testing.assert_allclose(g["TD1"], a**1.5, rtol=1e-10)
    np.testing.assert_allclose(g["T2D1"], 1.5 * a**2, rtol=1e-10)
    np.testing.assert_allclose(g["D2"], -3.0 / 7.0 * a**2, rtol=1e-9)
    np.testing.assert_allclose(g["TD2"], -6.0 / 7.0 * a**2.5, rtol=1e-9)
    np.testing.assert_allclose(g["T2D2"], -15.0 / 7.0 * a**3, rtol=1e-9)


def _heath(a, om, ol):
    """Heath (1977) integral: D1 proportional to E(a) int_0^a da' / (a' E(a'))^3,
    and its exact a-derivative, for matter + curvature + Lambda."""
    ok = 1.0 - om - ol
    e = lambda x: np.sqrt(om / x**3 + ok / x**2 + ol)
    integ = lambda x: quad(lambda y: 1.0 / (y * e(y)) ** 3, 0.0, x, epsabs=0, epsrel=1e-13, limit=200)[0]
    de = lambda x: (-3.0 * om / x**4 - 2.0 * ok / x**3) / (2.0 * e(x))
    d = np.array([e(x) * integ(x) for x in a])
    dd = np.array([de(x) * integ(x) + e(x) / (x * e(x)) ** 3 for x in a])
    return d, dd, e


@pytest.mark.parametrize("om,ol", [(0.3, 0.7), (0.25, 0.75), (0.3, 0.6)])
def test_d1_matches_heath_integral(om, ol):
    cfg = cosmo.Config(omega_m=om, omega_l=ol)
    a = np.array([0.1, 0.19, 0.5, 0.82, 1.0])
    d, dd, e = _heath(np.concatenate([a, [1.0]]), om, ol)
    norm = d[-1]
    g = cosmo.growth(a, cfg)
    np.testing.assert_allclose(g["D1"], d[:-1] / norm, rtol=1e-10)
    q = a**3 * e(a)
    np.testing.assert_allclose(g["TD1"], q * dd[:-1] / norm, rtol=1e-9)


def test_d2_matches_standard_fit():
    # D2 ~ -3/7 D1^2 Om(a)^(-1/143), Om(a) = Om a^-3 / E(a)^2.
    a = np.linspace(0.1, 1.0, 10)
    g = cosmo.growth(a, LCDM)
    om_a = LCDM.omega_m / a**3 / cosmo.hubble_e(a, LCDM) ** 2
    fit = -3.0 / 7.0 * g["D1"] ** 2 * om_a ** (-1.0 / 143.0)
    np.testing.assert_allclose(g["D2"], fit, rtol=1e-3)


def test_paper_constants():
    rows = {}
    with open("tests/golden/paper_constants.txt") as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            rows[name] = val
    cfg = cosmo.Config()
    assert cfg.a_init == pytest.approx(1.0 / (1.0 + float(rows["z_initial"])))
    assert cfg.n_steps == int(rows["n_steps"])
    assert cfg.n_lpt == float(rows["n_lpt"])
    assert cfg.box == float(rows["box_mpc_h"])
    a, am = cosmo.time_grid(cfg)
    assert rows["timestep_spacing"] == "uniform_in_a"
    np.testing.assert_allclose(np.diff(a), (1.0 - 0.1) / 10, rtol=1e-14)
    np.testing.assert_allclose(am, 0.5 * (a[1:] + a[:-1]), rtol=1e-15)
    assert a[0] == pytest.approx(0.1) and a[-1] == pytest.approx(1.0)


def _run_scalar_kdk(force_of_a, v0, cfg, table):
    """Scalar particle advanced with the oracle's merged-kick / drift factors."""
    s, v = 0.0, v0
    for i in range(cfg.n_steps):
        v += table.alpha[i] * force_of_a(table.a[i])
        s += table.beta[i] * v
    v += table.alpha[cfg.n_steps] * force_of_a(table.a[cfg.n_steps])
    return s, v


def _exact_scalar(force_of_a, v0, cfg):
    """ds/da = v/Q, dv/da = f(a)/Q integrated by an adaptive ODE solver."""
    rhs = lambda a, y: [y[1] / float(cosmo.q_of_a(a, cfg)), force_of_a(a) / float(cosmo.q_of_a(a, cfg))]
    sol = solve_ivp(rhs, (cfg.a_init, cfg.a_final), [0.0, v0], method="DOP853", rtol=1e-12, atol=1e-14)
    return sol.y[0, -1], sol.y[1, -1]


@pytest.mark.parametrize("n_steps,n_lpt", [(10, -2.5), (3, -2.5), (1, -2.5), (7, 1.5), (10, -4.0)])
def test_toy_model_is_integrated_exactly(n_steps, n_lpt):
    # Appendix A.3.2: if the residual acceleration is c T[u](a) then v = c u(a) and
    # s = c int u/Q da are reproduced exactly, for any step size.
    cfg = cosmo.Config(n_steps=n_steps, n_lpt=n_lpt)
    table = cosmo.step_table(cfg)
    c = 0.37
    f = lambda a: c * float(cosmo.tu_of_a(a, cfg))
    v0 = c * float(cosmo.u_of_a(cfg.a_init, cfg))
    s_num, v_num = _run_scalar_kdk(f, v0, cfg, table)
    s_ex, v_ex = _exact_scalar(f, v0, cfg)
    assert v_num == pytest.approx(c * float(cosmo.u_of_a(cfg.a_final, cfg)), rel=1e-12)
    assert v_num == pytest.approx(v_ex, rel=1e-9)
    assert s_num == pytest.approx(s_ex, rel=1e-9)


def test_generic_force_converges_at_second_order():
    # For an acceleration not proportional to T[u] the scheme is a consistent
    # second-order integrator: halving the step divides the error by ~4.
    errs = []
    f = lambda a: 0.8 * a + 0.3
    for n in (20, 40, 80):
        cfg = cosmo.Config(n_steps=n)
        s_num, v_num = _run_scalar_kdk(f, 0.0, cfg, cosmo.step_table(cfg))
        s_ex, v_ex = _exact_scalar(f, 0.0, cfg)
        errs.append(abs(s_num - s_ex) / abs(s_ex))
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


@pytest.mark.parametrize("ai,af,ac", [(0.1, 0.19, 0.145), (0.37, 0.64, 0.37), (0.5, 1.0, 1.0)])
def test_standard_factors_eds_closed_forms(ai, af, ac):
    # eqs. (KDKStd), (KDKALCstd) with Omega_m = 1, Q = a^(3/2):
    # int 1/Q da = 2 (a_i^-1/2 - a_f^-1/2), int (a/a_c)/Q da = 2 (a_f^1/2 - a_i^1/2) / a_c.
    assert cosmo.drift_factor_std(ai, af, EDS) == pytest.approx(2 * (ai**-0.5 - af**-0.5), rel=1e-12)
    assert cosmo.kick_factor_std(ai, af, ac, EDS) == pytest.approx(2 * (af**0.5 - ai**0.5) / ac, rel=1e-12)


def test_log_a_grid():
    # Appendix A.2: steps uniform in log a (constant ratio), midpoints arithmetic.
    cfg = cosmo.Config(log_a_steps=True, a_init=0.02, n_steps=7)
    a, am = cosmo.time_grid(cfg)
    np.testing.assert_allclose(a[1:] / a[:-1], (1.0 / 0.02) ** (1.0 / 7), rtol=1e-13)
    assert a[0] == 0.02 and a[-1] == 1.0
    np.testing.assert_allclose(am, 0.5 * (a[1:] + a[:-1]), rtol=1e-15)


@pytest.mark.parametrize("scheme", ["standard", "pm"])
@pytest.mark.parametrize("log_a", [False, True])
def test_standard_merged_factors_tile_the_run(scheme, log_a):
    # The merged kicks cover [a_0, a_n] once and the drifts [a_0, a_n] once, so in
    # Einstein-de Sitter sum_i alpha_i a_i = 2 (a_n^1/2 - a_0^1/2) and
    # sum_i beta_i = 2 (a_0^-1/2 - a_n^-1/2), for any grid.
    cfg = cosmo.Config(omega_m=1.0, omega_l=0.0, scheme=scheme, log_a_steps=log_a, n_steps=6)
    t = cosmo.step_table(cfg)
    assert float(np.sum(t.alpha * t.a)) == pytest.approx(2 * (1.0 - 0.1**0.5), rel=1e-12)
    assert float(np.sum(t.beta)) == pytest.approx(2 * (0.1**-0.5 - 1.0), rel=1e-12)


def test_unknown_scheme_rejected():
    with pytest.raises(ValueError):
        cosmo.step_table(cosmo.Config(scheme="leapfrog"))


@pytest.mark.parametrize("scheme", ["standard", "pm"])
def test_standard_kick_exact_for_a_proportional_force(scheme):
    # eq. (KDKStd): the kick holds d d^-2 delta fixed over its interval, so a force
    # F(a) = c a (fixed d d^-2 delta) is integrated exactly: v_n = v_0 + c int a/Q da.
    # A zero force leaves v fixed and the drift exact: s_n = v_0 int 1/Q da.
    for log_a in (False, True):
        cfg = cosmo.Config(scheme=scheme, log_a_steps=log_a, n_steps=4)
        table = cosmo.step_table(cfg)
        c, v0 = 0.61, 0.23
        ia = quad(lambda x: x / float(cosmo.q_of_a(x, cfg)), 0.1, 1.0, epsabs=0, epsrel=1e-13)[0]
        i1 = quad(lambda x: 1.0 / float(cosmo.q_of_a(x, cfg)), 0.1, 1.0, epsabs=0, epsrel=1e-13)[0]
        _, v_num = _run_scalar_kdk(lambda a: c * a, v0, cfg, table)
        assert v_num == pytest.approx(v0 + c * ia, rel=1e-12)
        s_num, v_num = _run_scalar_kdk(lambda a: 0.0, v0, cfg, table)
        assert v_num == v0
        assert s_num == pytest.approx(v0 * i1, rel=1e-12)


@pytest.mark.parametrize("log_a", [False, True])
def test_standard_leapfrog_converges_at_second_order(log_a):
    errs = []
    f = lambda a: 0.8 * a**2 + 0.3
    for n in (20, 40, 80):
        cfg = cosmo.Config(n_steps=n, scheme="standard", log_a_steps=log_a)
        s_num, _ = _run_scalar_kdk(f, 0.1, cfg, cosmo.step_table(cfg))
        s_ex, _ = _exact_scalar(f, 0.1, cfg)
        errs.append(abs(s_num - s_ex) / abs(s_ex))
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert 3.0 < errs[1] / errs[2] < 5.0


def test_u1_drift_variant():
    # The footnote's variant of eq. (KDKALC): u = 1 in the drift, u = a^nLPT in the
    # kick.  EdS drift factor 2 (a_i^-1/2 - a_f^-1/2); kick factors unchanged; a
    # residual acceleration c T[u](a) is still kicked exactly, and a constant velocity
    # is now drifted exactly.
    base = cosmo.Config(omega_m=1.0, omega_l=0.0, n_steps=5)
    var = cosmo.Config(omega_m=1.0, omega_l=0.0, n_steps=5, u1_drift=True)
    tb, tv = cosmo.step_table(base), cosmo.step_table(var)
    np.testing.assert_array_equal(tb.alpha, tv.alpha)
    a = tv.a
    np.testing.assert_allclose(tv.beta, 2 * (a[:-1] ** -0.5 - a[1:] ** -0.5), rtol=1e-12)
    cfg = cosmo.Config(n_steps=4, u1_drift=True)
    table = cosmo.step_table(cfg)
    c = 0.37
    f = lambda x: c * float(cosmo.tu_of_a(x, cfg))
    _, v_num = _run_scalar_kdk(f, 0.0, cfg, table)
    assert v_num == pytest.approx(c * float(cosmo.u_of_a(cfg.a_final, cfg) - cosmo.u_of_a(cfg.a_init, cfg)),
                                  rel=1e-12)
    i1 = quad(lambda x: 1.0 / float(cosmo.q_of_a(x, cfg)), cfg.a_init, cfg.a_final, epsabs=0, epsrel=1e-13)[0]
    s_num, _ = _run_scalar_kdk(lambda x: 0.0, 0.29, cfg, table)
    assert s_num == pytest.approx(0.29 * i1, rel=1e-12)


def test_lpt_velocity_cancels_at_start():
    # L-(a_0) applied to the 2LPT velocity gives v_res(a_0) = 0 (eq. Lops); the
    # T[D] used there must be the derivative of the D used for positions.
    table = cosmo.step_table(LCDM)
    g = table.grow
    h = 1e-5
    a0 = LCDM.a_init
    gp, gm = cosmo.growth([a0 + h], LCDM), cosmo.growth([a0 - h], LCDM)
    q0 = float(cosmo.q_of_a(a0, LCDM))
    assert g["TD1"][0] == pytest.approx(q0 * (gp["D1"][0] - gm["D1"][0]) / (2 * h), rel=1e-8)
    assert g["TD2"][0] == pytest.approx(q0 * (gp["D2"][0] - gm["D2"][0]) / (2 * h), rel=1e-8)


def test_bbks_limits_and_sigma8():
    cfg = LCDM
    assert float(cosmo.bbks_transfer(1e-9, cfg)) == pytest.approx(1.0, abs=1e-7)
    # sigma8 of the normalised spectrum, recomputed by a trapezoid rule on a fine
    # log-k grid (a different quadrature from the one used to normalise).
    amp = cosmo.power_amplitude(cfg)
    lnk = np.linspace(np.log(1e-5), np.log(1e3), 400001)
    k = np.exp(lnk)
    integ = k**3 * cosmo.linear_power(k, cfg, amp) * cosmo.tophat_window(8.0 * k) ** 2
    sig2 = np.trapezoid(integ, lnk) / (2 * np.pi**2)
    assert np.sqrt(sig2) == pytest.approx(cfg.sigma8, rel=1e-6)
