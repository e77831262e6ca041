"""Background, growth factors, spectrum and COLA step coefficients (FP64, scipy).

Test infrastructure (see ``oracle/__init__``).

Paper passages followed:

* Appendix A.1, eq. (eom): T = Q(a) d/da with Q(a) = a^3 H(a)/H0, and
  T^2[s] = -(3/2) Om a d_x d_x^-2 delta.  Linearising that equation gives the
  growth equations T^2[D1] = (3/2) Om a D1 and, at second order,
  T^2[D2] = (3/2) Om a (D2 - D1^2) (the standard 2LPT growth equation; the paper
  calls computing D1, T[D1], T^2[D1], ... "a straightforward exercise",
  end of Appendix A.3).
* Appendix A.3: D1(1) = 1 normalisation.  D2 is normalised with the same
  constant squared, so D2 ~ -3/7 D1^2 (reading: only D2*s2 enters the method,
  and s2 is built from the D1-normalised field).
* Appendix A.3.2, eq. (KDKALC): u(a) = a^nLPT, kick factor
  (u(a_f) - u(a_i)) / T[u](a_c), drift factor int u/Q da / u(a_c).
* eq. (ALCtimestep) and the text after it: timesteps uniform in a, with
  a_{i+1/2} the arithmetic midpoint (Appendix A.2).  Consecutive half-kicks that
  share a_c = a_i are merged into one kick (exact: same force, factors add).
* Variants (``Config.scheme``): eq. (KDKALCstd), the standard COLA discretisation,
  kick factor int (a/a_c)/Q da and drift factor int 1/Q da; eq. (KDKStd), the plain
  PM leapfrog, which is eq. (KDKALCstd) with s1 = s2 = 0 (Appendix A.3.1).  Its
  kick carries -(3/2) Om d d^-2 delta without the factor a_c, so with the force
  F = -(3/2) Om a_c d d^-2 delta the factor is again int (a/a_c)/Q da.
  ``Config.log_a_steps``: a_i uniform in log a (Appendix A.2), midpoints still
  arithmetic (the choice stated there for small steps).  ``Config.u1_drift``: the
  footnote's variant of eq. (KDKALC), u = A + B a^nLPT with B << A, i.e. u = 1 in the
  drift (factor int 1/Q da) and u = a^nLPT in the kick.

Readings of the variants: eq. (KDKALCstd) is printed with a minus sign in front of
the kick integral while the bracket it multiplies is already the acceleration; read
with a plus sign, which is what setting s1 = s2 = 0 must give to recover eq.
(KDKStd), as the text after it states, and what eq. (KDKALC) has.  eq. (KDKStd)
prints d_x d_x^2; read d_x d_x^-2 as in eq. (eom).

Readings where the paper is silent: flat-or-curved FRW with matter, curvature and
Lambda and no radiation, E^2 = Om a^-3 + Ok a^-2 + OL; BBKS transfer function with
shape parameter Gamma = Om h (no baryon correction); sigma8 normalisation of the
z = 0 linear spectrum with a top-hat of radius 8 Mpc/h.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.integrate import quad, solve_ivp


@dataclass(frozen=True)
class Config:
    """Run parameters of the method (Section 2, Appendix A.3) plus the cosmology."""

    np_side: int = 32          # particles per side (Lagrangian grid)
    nm_side: int = 64          # force-mesh cells per side
    box: float = 100.0         # L in Mpc/h
    omega_m: float = 0.3
    omega_l: float = 0.7
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    a_init: float = 0.1        # z = 9
    a_final: float = 1.0
    n_steps: int = 10
    n_lpt: float = -2.5
    scheme: str = "modified"   # "modified" eq. (KDKALC), "standard" eq. (KDKALCstd), "pm" eq. (KDKStd)
    log_a_steps: bool = False  # a_i uniform in log a instead of in a
    u1_drift: bool = False     # "modified" with u = 1 in the drift (footnote on u(a), Appendix A.3.2)

    @property
    def omega_k(self) -> float:
        return 1.0 - self.omega_m - self.omega_l


def hubble_e(a, cfg: Config):
    """E(a) = H(a)/H0 for matter + curvature + Lambda (no radiation)."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(cfg.omega_m / a**3 + cfg.omega_k / a**2 + cfg.omega_l)


def q_of_a(a, cfg: Config):
    """Q(a) = a^3 H(a)/H0, eq. (eom)."""
    a = np.asarray(a, dtype=np.float64)
    return a**3 * hubble_e(a, cfg)


# ----------------------------------------------------------------------------------
# Growth factors: integrate y = (D1, T[D1], D2, T[D2]) in a with dD/da = T[D]/Q and
# dT[D]/da = T^2[D]/Q.  Growing-mode start deep in matter domination.
# ----------------------------------------------------------------------------------
_A_START = 1e-5


def _growth_rhs(a, y, cfg: Config):
    d1, v1, d2, v2 = y
    q = float(q_of_a(a, cfg))
    src = 1.5 * cfg.omega_m * a
    return [v1 / q, src * d1 / q, v2 / q, src * (d2 - d1 * d1) / q]


def _growth_raw(a_eval, cfg: Config):
    """Unnormalised solution at the sorted points a_eval (all >= _A_START)."""
    a0 = _A_START
    q0 = float(q_of_a(a0, cfg))
    y0 = [a0, q0, -3.0 / 7.0 * a0 * a0, -6.0 / 7.0 * a0 * q0]
    sol = solve_ivp(_growth_rhs, (a0, float(a_eval[-1])), y0, method="DOP853",
                    t_eval=a_eval, rtol=1e-13, atol=1e-30, args=(cfg,))
    if not sol.success:
        raise RuntimeError(sol.message)
    return sol.y


def growth(a, cfg: Config) -> dict:
    """D1, D2, T[D1], T[D2], T^2[D1], T^2[D2] at scale factors ``a`` (FP64 arrays).

    Normalised so that D1(1) = 1; D2 carries the same normalisation squared.
    T^2[D] is taken from the right-hand sides of the growth equations (never by
    finite differences).
    """
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    pts = np.unique(np.concatenate([a, [1.0]]))
    d1, v1, d2, v2 = _growth_raw(pts, cfg)
    c = d1[np.searchsorted(pts, 1.0)]
    idx = np.searchsorted(pts, a)
    D1, V1 = d1[idx] / c, v1[idx] / c
    D2, V2 = d2[idx] / c**2, v2[idx] / c**2
    src = 1.5 * cfg.omega_m * a
    return {
        "D1": D1, "D2": D2, "TD1": V1, "TD2": V2,
        "T2D1": src * D1, "T2D2": src * (D2 - D1 * D1),
    }


# ----------------------------------------------------------------------------------
# Time grid and COLA kick / drift coefficients, eq. (KDKALC) and eq. (ALCtimestep).
# ----------------------------------------------------------------------------------
def time_grid(cfg: Config):
    """a_i (i = 0..n), uniform in a or in log a, and the midpoints a_{i+1/2} (i = 0..n-1)."""
    n = cfg.n_steps
    t = np.arange(n + 1, dtype=np.float64) / n
    if cfg.log_a_steps:
        a = cfg.a_init * (cfg.a_final / cfg.a_init) ** t
    else:
        a = cfg.a_init + (cfg.a_final - cfg.a_init) * t
    a[-1] = cfg.a_final
    return a, 0.5 * (a[:-1] + a[1:])


def u_of_a(a, cfg: Config):
    """u(a) = a^nLPT (Appendix A.3.2 ansatz)."""
    return np.asarray(a, dtype=np.float64) ** cfg.n_lpt


def tu_of_a(a, cfg: Config):
    """T[u](a) = Q(a) du/da = Q(a) nLPT a^(nLPT-1)."""
    a = np.asarray(a, dtype=np.float64)
    return q_of_a(a, cfg) * cfg.n_lpt * a ** (cfg.n_lpt - 1.0)


def kick_factor(a_i, a_f, a_c, cfg: Config) -> float:
    """Modified kick K(a_i, a_f; a_c) factor: (u(a_f) - u(a_i)) / T[u](a_c)."""
    return float((u_of_a(a_f, cfg) - u_of_a(a_i, cfg)) / tu_of_a(a_c, cfg))


def drift_factor(a_i, a_f, a_c, cfg: Config) -> float:
    """Modified drift D(a_i, a_f; a_c) factor: int_{a_i}^{a_f} u/Q da / u(a_c)."""
    val, _ = quad(lambda x: float(u_of_a(x, cfg) / q_of_a(x, cfg)), a_i, a_f,
                  epsabs=0.0, epsrel=1e-13, limit=200)
    return val / float(u_of_a(a_c, cfg))


def kick_factor_std(a_i, a_f, a_c, cfg: Config) -> float:
    """Standard kick factor, eqs. (KDKALCstd) and (KDKStd): int_{a_i}^{a_f} (a/a_c)/Q da."""
    val, _ = quad(lambda x: float(x / q_of_a(x, cfg)), a_i, a_f, epsabs=0.0, epsrel=1e-13, limit=200)
    return val / a_c


def drift_factor_std(a_i, a_f, cfg: Config) -> float:
    """Standard drift factor, eqs. (KDKALCstd) and (KDKStd): int_{a_i}^{a_f} 1/Q da."""
    val, _ = quad(lambda x: float(1.0 / q_of_a(x, cfg)), a_i, a_f, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


@dataclass
class StepTable:
    a: np.ndarray            # a_0 .. a_n
    a_mid: np.ndarray        # a_{1/2} .. a_{n-1/2}
    alpha: np.ndarray        # merged kick factor at a_i, i = 0..n
    beta: np.ndarray         # drift factor for step i, i = 0..n-1
    dD1: np.ndarray          # D1(a_{i+1}) - D1(a_i)
    dD2: np.ndarray          # D2(a_{i+1}) - D2(a_i)
    grow: dict = field(default_factory=dict)   # growth() evaluated at a_0..a_n


def step_table(cfg: Config) -> StepTable:
    """All per-step scalars of the evolution (ALCtimestep) with the scheme's factors.

    Step i (0 <= i < n) = kick at a_i over [a_{i-1/2}, a_{i+1/2}] (over
    [a_0, a_{1/2}] for i = 0) followed by the drift over [a_i, a_{i+1}] with
    a_c = a_{i+1/2}.  The closing half-kick over [a_{n-1/2}, a_n] uses alpha[n].
    """
    if cfg.scheme not in ("modified", "standard", "pm"):
        raise ValueError(f"unknown scheme {cfg.scheme!r}")
    std = cfg.scheme != "modified"
    a, am = time_grid(cfg)
    n = cfg.n_steps
    alpha = np.empty(n + 1)
    # K(a_{i-1/2}, a_i; a_i) followed by K(a_i, a_{i+1/2}; a_i) are merged.
    for i in range(n + 1):
        lo = a[0] if i == 0 else am[i - 1]
        hi = a[n] if i == n else am[i]
        alpha[i] = kick_factor_std(lo, hi, a[i], cfg) if std else kick_factor(lo, hi, a[i], cfg)
    # u = 1 in eq. (KDKALC)'s drift gives int 1/Q da, the standard drift factor
    plain_drift = std or cfg.u1_drift
    beta = np.array([drift_factor_std(a[i], a[i + 1], cfg) if plain_drift else drift_factor(a[i], a[i + 1], am[i], cfg)
                     for i in range(n)])
    g = growth(a, cfg)
    return StepTable(a=a, a_mid=am, alpha=alpha, beta=beta,
                     dD1=np.diff(g["D1"]), dD2=np.diff(g["D2"]), grow=g)


# ----------------------------------------------------------------------------------
# Linear power spectrum at z = 0: BBKS transfer function, sigma8 normalisation.
# ----------------------------------------------------------------------------------
def bbks_transfer(k, cfg: Config):
    """Bardeen, Bond, Kaiser & Szalay (1986) transfer function, q = k / (Om h)."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (cfg.omega_m * cfg.h)
    x = 2.34 * q
    with np.errstate(divide="ignore", invalid="ignore"):
        lead = np.where(x > 1e-8, np.log1p(x) / np.where(x > 0, x, 1.0), 1.0 - 0.5 * x)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return lead * poly ** -0.25


def tophat_window(x):
    """Fourier transform of a unit-volume spherical top-hat, 3 (sin x - x cos x)/x^3."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    full = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs**3
    return np.where(small, 1.0 - x * x / 10.0, full)


def _unnormalised_power(k, cfg: Config):
    k = np.asarray(k, dtype=np.float64)
    return k ** cfg.n_s * bbks_transfer(k, cfg) ** 2


def power_amplitude(cfg: Config) -> float:
    """A such that P(k) = A k^ns T(k)^2 has sigma(R = 8 Mpc/h) = sigma8.

    sigma^2 = (1 / 2 pi^2) int k^2 P(k) W(kR)^2 dk, integrated over ln k on
    [1e-5, 1e3] h/Mpc in pieces so the oscillating tail is resolved.
    """
    def integrand(lnk):
        k = np.exp(lnk)
        return k**3 * float(_unnormalised_power(k, cfg)) * float(tophat_window(8.0 * k)) ** 2

    edges = np.linspace(np.log(1e-5), np.log(1e3), 401)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        tot += quad(integrand, lo, hi, epsabs=0.0, epsrel=1e-10, limit=200)[0]
    return cfg.sigma8**2 / (tot / (2.0 * np.pi**2))


def linear_power(k, cfg: Config, amplitude: float | None = None):
    """P(k) in (Mpc/h)^3 at z = 0 (a = 1, where D1 = 1)."""
    amp = power_amplitude(cfg) if amplitude is None else amplitude
    return amp * _unnormalised_power(k, cfg)
