"""Independent pins of the oracle's spectrum normalisation and growth tables (CPU only).

The linear spectrum (Section 2: initial conditions from a Gaussian field) enters the
method as P(k) = A k^ns T(k)^2, with T the BBKS fit and A fixed by sigma8.  The growth
factors D1, D2 and the step coefficients come from Appendix A.1 and A.3.  Each check
below compares the oracle with something it does not compute itself:

* the top-hat variance of white noise, sigma_R^2 = 3 A / (4 pi R^3) (the integral of
  the squared spherical Bessel function j1 is pi/6), which fixes the window and the
  quadrature of the sigma8 normalisation independently of the transfer function;
* the BBKS fit depends on k only through k / Gamma with Gamma = Om h;
* the amplitude and the whole 10-step table of an independent calculation
  (``tests/golden/reference_scalars.txt``);
* D2 and T[D2] by variation of parameters: with the growing mode D+ (Heath integral)
  and the decaying mode D- = E(a) = H/H0 of the linear growth equation, the
  second-order growth factor is a double quadrature, with no ODE solver involved.
"""
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import cosmology as cosmo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reference_scalars.txt")
LCDM = cosmo.Config()


def _golden():
    rows, final, td, amp = [], None, {}, None
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0] == "amplitude":
                amp = float(f[1])
            elif f[0] == "row":
                rows.append([float(x) for x in f[1:]])
            elif f[0] == "final":
                final = [float(x) for x in f[1:]]
            elif f[0] == "td":
                td[float(f[1])] = (float(f[2]), float(f[3]))
    return amp, np.array(rows), final, td


def test_tophat_variance_of_white_noise(monkeypatch):
    # With T = 1 and ns = 0 the spectrum is white, P = A.  Then
    #   sigma_R^2 = (A / 2 pi^2) int_0^inf k^2 W(kR)^2 dk = (A / 2 pi^2 R^3) * 9 int_0^inf j1(x)^2 dx
    # and int_0^inf j1^2 = pi / 6, so sigma_R^2 = 3 A / (4 pi R^3): the variance of white
    # noise averaged over a sphere of volume 4 pi R^3 / 3.  The oracle integrates k over
    # [1e-5, 1e3] h/Mpc; x = 8k then stops at X = 8000, and the missing tail is
    # 9 int_X^inf j1^2 = 9 / (2X) + O(X^-2) (j1 ~ -cos x / x), a 1.2e-4 relative effect
    # that the expected value includes.
    monkeypatch.setattr(cosmo, "bbks_transfer", lambda k, cfg: np.ones_like(np.asarray(k, dtype=np.float64)))
    cfg = cosmo.Config(n_s=0.0)
    a = cosmo.power_amplitude(cfg)
    r, x_max = 8.0, 8.0 * 1e3
    integral = 1.5 * np.pi - 4.5 / x_max
    sigma2 = a / (2 * np.pi**2 * r**3) * integral
    assert sigma2 == pytest.approx(cfg.sigma8**2, rel=1e-6)
    # and the untruncated closed form, to the size of the tail
    assert 3 * a / (4 * np.pi * r**3) == pytest.approx(cfg.sigma8**2, rel=2e-4)


@pytest.mark.parametrize("om,h,om2,h2", [(0.3, 0.7, 0.3, 0.5), (0.3, 0.7, 0.25, 0.7), (0.3, 0.7, 0.4, 0.6)])
def test_bbks_depends_on_k_over_omega_m_h(om, h, om2, h2):
    # The BBKS fit is a function of q = k / Gamma alone, with Gamma = Om h (no baryon
    # correction): T(k; Om, h) = T(k Om' h' / (Om h); Om', h').
    k = np.geomspace(1e-4, 50.0, 41)
    c1 = cosmo.Config(omega_m=om, h=h)
    c2 = cosmo.Config(omega_m=om2, h=h2)
    np.testing.assert_allclose(cosmo.bbks_transfer(k, c1),
                               cosmo.bbks_transfer(k * (om2 * h2) / (om * h), c2), rtol=1e-13)
    # and it decreases from 1
    t = cosmo.bbks_transfer(np.concatenate([[1e-9], k]), c1)
    assert np.all(np.diff(t) < 0) and t[0] == pytest.approx(1.0, abs=1e-7)


def test_power_amplitude_matches_independent_value():
    amp, _, _, _ = _golden()
    assert cosmo.power_amplitude(LCDM) == pytest.approx(amp, rel=5e-5)


def test_step_table_matches_independent_values():
    _, rows, final, td = _golden()
    t = cosmo.step_table(LCDM)
    g = t.grow
    for r in rows:
        i = int(r[0])
        got = [t.a[i], g["D1"][i], g["D2"][i], g["T2D1"][i], g["T2D2"][i], t.alpha[i], t.beta[i],
               t.dD1[i], t.dD2[i]]
        np.testing.assert_allclose(got, r[1:], rtol=0, atol=1e-9, err_msg=f"row {i}")
    n = int(final[0])
    got = [t.a[n], g["D1"][n], g["D2"][n], g["T2D1"][n], g["T2D2"][n], t.alpha[n]]
    np.testing.assert_allclose(got, final[1:], rtol=0, atol=1e-9, err_msg="final row")
    for a, (td1, td2) in td.items():
        gg = cosmo.growth([a], LCDM)
        np.testing.assert_allclose([gg["TD1"][0], gg["TD2"][0]], [td1, td2], rtol=0, atol=6e-9)


def _second_order_by_quadrature(a_eval, om, ol):
    """D2 and T[D2] at a_eval from variation of parameters (normalised by D1raw(1)^2).

    The growth equation Q (Q D')' - c D = f with c = (3/2) Om a has the growing mode
    D+ (Heath: E(a) int_0^a da' / (a' E)^3) and the decaying mode D- = E(a), Wronskian
    W = D+ D-' - D+' D- = C / Q.  The solution of f = -c D+^2 that vanishes faster
    than D+ as a -> 0 is
      D2(a) = (1/C) [D-(a) I+(a) - D+(a) I-(a)],  I+-(a) = int_0^a D+-(a') f(a') / Q(a') da',
    and T[D2] = Q D2' = (Q / C) [D-'(a) I+(a) - D+'(a) I-(a)].
    """
    ok = 1.0 - om - ol
    e = lambda x: np.sqrt(om / x**3 + ok / x**2 + ol)
    de = lambda x: (-3.0 * om / x**4 - 2.0 * ok / x**3) / (2.0 * e(x))
    q = lambda x: x**3 * e(x)
    heath_int = lambda x: quad(lambda y: 1.0 / (y * e(y)) ** 3, 0.0, x, epsabs=0, epsrel=1e-13, limit=200)[0]
    dplus = lambda x: e(x) * heath_int(x)
    dplus_p = lambda x: de(x) * heath_int(x) + e(x) / (x * e(x)) ** 3
    f = lambda x: -1.5 * om * x * dplus(x) ** 2
    cw = q(1.0) * (dplus(1.0) * de(1.0) - dplus_p(1.0) * e(1.0))
    d1 = dplus(1.0)
    d2, td2 = [], []
    for a in a_eval:
        ip = quad(lambda x: dplus(x) * f(x) / q(x), 0.0, a, epsabs=0, epsrel=1e-12, limit=200)[0]
        im = quad(lambda x: e(x) * f(x) / q(x), 0.0, a, epsabs=0, epsrel=1e-12, limit=200)[0]
        d2.append((e(a) * ip - dplus(a) * im) / cw / d1**2)
        td2.append(q(a) * (de(a) * ip - dplus_p(a) * im) / cw / d1**2)
    return np.array(d2), np.array(td2)


def test_decaying_mode_solves_the_growth_equation():
    # E(a) = H/H0 solves Q (Q D')' = (3/2) Om a D for matter + curvature + Lambda:
    # checked by central differences of Q dE/da (exact derivative) in a.
    for om, ol in [(0.3, 0.7), (0.3, 0.6)]:
        ok = 1.0 - om - ol
        e = lambda x: np.sqrt(om / x**3 + ok / x**2 + ol)
        de = lambda x: (-3.0 * om / x**4 - 2.0 * ok / x**3) / (2.0 * e(x))
        qde = lambda x: x**3 * e(x) * de(x)
        for a in (0.1, 0.45, 1.0):
            h = 1e-5 * a
            lhs = a**3 * e(a) * (qde(a + h) - qde(a - h)) / (2 * h)
            assert lhs == pytest.approx(1.5 * om * a * e(a), rel=1e-8)


@pytest.mark.parametrize("om,ol", [(0.3, 0.7), (0.25, 0.75), (0.3, 0.6)])
def test_d2_matches_variation_of_parameters(om, ol):
    a = np.array([0.1, 0.37, 0.73, 1.0])
    d2, td2 = _second_order_by_quadrature(a, om, ol)
    g = cosmo.growth(a, cosmo.Config(omega_m=om, omega_l=ol))
    np.testing.assert_allclose(g["D2"], d2, rtol=1e-9)
    np.testing.assert_allclose(g["TD2"], td2, rtol=1e-8)
