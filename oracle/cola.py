"""COLA time evolution, eqs. (ALCtimestep), (Lops), (KDKALC)  (FP64, torch CPU).

Test infrastructure (see ``oracle/__init__``).

State per particle: displacement s = x - q and the residual velocity
v = v_res = T[s_res] measured by an LPT observer (Appendix A.3), stored as
(3, Np, Np, Np) tensors.  s1, s2 are constant per particle (Appendix A.3, end).

Evolution from a_0 to a_n (eq. ALCtimestep):
  L-(a_0), then for i = 0..n-1:  K(a_i, a_{i+1/2}; a_i)  D(a_i, a_{i+1}; a_{i+1/2})
  K(a_{i+1/2}, a_{i+1}; a_{i+1}), then L+(a_n).
The closing half-kick of step i and the opening half-kick of step i+1 share
a_c = a_{i+1} and the same force, so they are applied as one kick whose factor is
the sum of the two; one force evaluation per step plus one at a_n.

Kick (KDKALC):  v += alpha * (F(s, a_c) - T^2[D1](a_c) s1 - T^2[D2](a_c) s2)
Drift (KDKALC): s += beta * v + (D1(a_f) - D1(a_i)) s1 + (D2(a_f) - D2(a_i)) s2
L+- (Lops):     v +-= T[D1](a) s1 + T[D2](a) s2

Config.scheme "standard" uses the same operators with the factors of eq.
(KDKALCstd) (taken from the step table).  Config.scheme "pm" is the plain PM
leapfrog of eq. (KDKStd): the operators above with s1 = s2 = 0, so that L+- do
nothing, the state is the full displacement s and the full velocity v = T[s], and
the kick adds the plain force; the particles still start on the 2LPT trajectory.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import cosmology as cosmo
from .fourier import F64
from .lpt import lagrangian_grid, lpt_from_noise
from .pm import pm_force


@dataclass
class State:
    s: torch.Tensor    # (3, Np, Np, Np) displacement from the Lagrangian grid
    v: torch.Tensor    # (3, Np, Np, Np) residual velocity v_res
    s1: torch.Tensor
    s2: torch.Tensor


def initial_state(s1, s2, table: cosmo.StepTable, lpt_frame: bool = True) -> State:
    """2LPT position and velocity at a_0, then L-(a_0): v_res(a_0) = 0 (eq. Lops).

    lpt_frame False (eq. KDKStd): the operators act with s1 = s2 = 0, so the state
    keeps the 2LPT velocity and carries zero LPT fields.
    """
    g = table.grow
    s = g["D1"][0] * s1 + g["D2"][0] * s2
    v = g["TD1"][0] * s1 + g["TD2"][0] * s2          # T[s] of the 2LPT trajectory
    if not lpt_frame:
        return State(s=s, v=v, s1=torch.zeros_like(s1), s2=torch.zeros_like(s2))
    v = v - (g["TD1"][0] * s1 + g["TD2"][0] * s2)     # L-(a_0)
    return State(s=s, v=v, s1=s1, s2=s2)


def kick(st: State, i: int, table: cosmo.StepTable, cfg: cosmo.Config) -> State:
    """Merged kick at a_i with factor alpha_i (eq. KDKALC)."""
    a = float(table.a[i])
    g = table.grow
    force = pm_force(st.s, a, cfg.np_side, cfg.nm_side, cfg.box, cfg.omega_m)
    acc = force - g["T2D1"][i] * st.s1 - g["T2D2"][i] * st.s2
    return State(s=st.s, v=st.v + table.alpha[i] * acc, s1=st.s1, s2=st.s2)


def drift(st: State, i: int, table: cosmo.StepTable) -> State:
    """Drift D(a_i, a_{i+1}; a_{i+1/2}) (eq. KDKALC)."""
    s = st.s + table.beta[i] * st.v + table.dD1[i] * st.s1 + table.dD2[i] * st.s2
    return State(s=s, v=st.v, s1=st.s1, s2=st.s2)


def step(st: State, i: int, table: cosmo.StepTable, cfg: cosmo.Config) -> State:
    """One step: kick at a_i, then drift to a_{i+1}."""
    return drift(kick(st, i, table, cfg), i, table)


def finish(st: State, table: cosmo.StepTable, cfg: cosmo.Config):
    """Closing half-kick at a_n, then L+(a_n).  Returns (x mod L, v_phys, s)."""
    n = cfg.n_steps
    st = kick(st, n, table, cfg)
    g = table.grow
    v_phys = st.v + g["TD1"][n] * st.s1 + g["TD2"][n] * st.s2     # L+(a_n)
    x = torch.remainder(lagrangian_grid(cfg.np_side, cfg.box) + st.s, cfg.box)
    return x, v_phys, st.s


def evolve(s1, s2, cfg: cosmo.Config, table: cosmo.StepTable | None = None,
           keep_states: bool = False):
    """Full evolution from given LPT fields.  Returns (x, v_phys, s[, states])."""
    table = cosmo.step_table(cfg) if table is None else table
    st = initial_state(s1, s2, table, lpt_frame=cfg.scheme != "pm")
    states = [st]
    for i in range(cfg.n_steps):
        st = step(st, i, table, cfg)
        if keep_states:
            states.append(st)
    x, v, s = finish(st, table, cfg)
    return (x, v, s, states) if keep_states else (x, v, s)


def run(w, cfg: cosmo.Config, amplitude: float | None = None, keep_states: bool = False):
    """2LPT initial conditions from white noise w, then the COLA evolution."""
    s1, s2 = lpt_from_noise(w, cfg, amplitude)
    return evolve(s1, s2, cfg, keep_states=keep_states)


def to_flat(t: torch.Tensor) -> torch.Tensor:
    """(3, Np, Np, Np) -> (3, Np^3) in particle order p = (i Np + j) Np + k."""
    return t.reshape(3, -1)


def from_flat(t, n: int) -> torch.Tensor:
    return torch.as_tensor(t, dtype=F64).reshape(3, n, n, n)
