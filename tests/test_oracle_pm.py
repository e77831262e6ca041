"""Pins of the oracle's particle-mesh force (CPU only).

Cloud-in-cell: mass conservation, single-particle stencils, uniform lattices.
Poisson + gradient: the analytic field of a single Fourier mode.  Whole force:
momentum conservation, zero self-force, exact interpolation of linear fields and
the deposit/gather adjoint identity.
"""
import math

import pytest
import torch

from oracle import pm
from oracle.fourier import F64
from oracle.lpt import lagrangian_grid


def _clustered_displacements(n_p, box, seed, scale=3.0):
    g = torch.Generator().manual_seed(seed)
    s = scale * torch.randn(3, n_p, n_p, n_p, generator=g, dtype=F64)
    # pull a chunk of the particles into a tight clump to exercise many-per-cell
    clump = torch.rand(n_p, n_p, n_p, generator=g, dtype=F64) < 0.2
    q = lagrangian_grid(n_p, box)
    centre = torch.tensor([0.3, 0.6, 0.1], dtype=F64).view(3, 1, 1, 1) * box
    s = torch.where(clump, centre - q + 0.5 * torch.randn(3, n_p, n_p, n_p, generator=g, dtype=F64), s)
    return s


def test_mass_is_conserved():
    n_p, n_m, box = 16, 32, 50.0
    s = _clustered_displacements(n_p, box, 1, scale=20.0)
    rho = pm.cic_deposit(s, n_p, n_m, box)
    assert rho.sum().item() == pytest.approx(n_m**3, rel=1e-13)
    assert rho.min().item() >= 0.0


def test_single_particle_stencils():
    n_m, box = 8, 8.0           # dx = 1
    # at a cell centre (c + 1/2) dx: all mass in cell c
    rho = pm.cic_deposit_points(torch.tensor([[2.5], [3.5], [7.5]], dtype=F64), n_m, box, mass=1.0)
    assert rho[2, 3, 7].item() == pytest.approx(1.0, abs=1e-15)
    assert rho.sum().item() == pytest.approx(1.0, abs=1e-15)
    # at a cell corner: 1/8 to each of the 8 cells sharing it, across the periodic edge
    rho = pm.cic_deposit_points(torch.tensor([[0.0], [4.0], [2.0]], dtype=F64), n_m, box, mass=1.0)
    for cx in (7, 0):
        for cy in (3, 4):
            for cz in (1, 2):
                assert rho[cx, cy, cz].item() == pytest.approx(0.125, abs=1e-15)
    # linear weights along one axis
    rho = pm.cic_deposit_points(torch.tensor([[1.75], [0.5], [0.5]], dtype=F64), n_m, box, mass=1.0)
    assert rho[1, 0, 0].item() == pytest.approx(0.75, abs=1e-15)
    assert rho[2, 0, 0].item() == pytest.approx(0.25, abs=1e-15)


def test_all_particles_at_one_point_deposit_as_one_particle():
    """Displacements s = x0 - q carry every lattice point to x0 (some across the
    periodic box): the deposit must equal that of one particle holding all the mass."""
    n_p, n_m, box = 8, 16, 16.0
    x0 = [3.25, 12.75, 0.5]
    q = torch.arange(n_p, dtype=F64) * (box / n_p)
    qx, qy, qz = torch.meshgrid(q, q, q, indexing="ij")
    s = torch.stack([x0[0] - qx, x0[1] - qy, x0[2] - qz])
    rho = pm.cic_deposit(s, n_p, n_m, box)
    one = pm.cic_deposit_points(torch.tensor(x0, dtype=F64).view(3, 1), n_m, box, mass=float(n_m**3))
    assert torch.allclose(rho, one, rtol=0, atol=1e-9)
    assert int((one != 0).sum()) == 4   # z fraction 0: four cells


@pytest.mark.parametrize("ratio", [1, 2])
def test_unperturbed_lattice_is_uniform_and_force_free(ratio):
    n_p, box = 8, 40.0
    n_m = ratio * n_p
    s = torch.zeros(3, n_p, n_p, n_p, dtype=F64)
    rho = pm.cic_deposit(s, n_p, n_m, box)
    torch.testing.assert_close(rho, torch.ones_like(rho), atol=1e-14, rtol=0)
    f = pm.pm_force(s, 1.0, n_p, n_m, box, 0.3)
    assert f.abs().max().item() < 1e-13


def test_lattice_ratio_three_is_force_free_by_symmetry():
    n_p, box = 6, 30.0
    s = torch.zeros(3, n_p, n_p, n_p, dtype=F64)
    f = pm.pm_force(s, 1.0, n_p, 3 * n_p, box, 0.3)
    assert f.abs().max().item() < 1e-13


@pytest.mark.parametrize("nvec", [(1, 0, 0), (0, 3, 0), (2, -1, 5), (-7, 4, 1)])
def test_single_mode_potential_and_gradient(nvec):
    n, box, amp = 16, 70.0, 0.37
    dx = box / n
    ax = (torch.arange(n, dtype=F64) + 0.5) * dx       # cell centres
    x = torch.stack(torch.meshgrid(ax, ax, ax, indexing="ij"))
    k = 2 * math.pi / box * torch.tensor(nvec, dtype=F64)
    phase = (k.view(3, 1, 1, 1) * x).sum(0)
    rho = 1.0 + amp * torch.cos(phase)
    g = pm.gradient_fields(rho, box)
    k2 = float(k @ k)
    # d^-2 delta = -A cos / k^2 and g = -grad(d^-2 delta) = -A k sin / k^2
    expect = -amp * k.view(3, 1, 1, 1) / k2 * torch.sin(phase)
    torch.testing.assert_close(g, expect, atol=1e-13, rtol=0)
    phi = pm.potential_field(rho, box)
    torch.testing.assert_close(phi, -amp * torch.cos(phase) / k2, atol=1e-13, rtol=0)


def test_momentum_is_conserved():
    n_p, n_m, box = 16, 32, 60.0
    s = _clustered_displacements(n_p, box, 7, scale=8.0)
    f = pm.pm_force(s, 0.8, n_p, n_m, box, 0.3)
    tot = f.reshape(3, -1).sum(1)
    scale = f.abs().sum().item()
    assert tot.abs().max().item() < 1e-12 * scale


def test_single_particle_feels_no_self_force():
    n_m, box = 16, 16.0
    for pos in ([3.3, 7.9, 0.2], [0.0, 0.5, 15.99], [8.25, 8.75, 1.1]):
        x = torch.tensor(pos, dtype=F64).view(3, 1)
        rho = pm.cic_deposit_points(x, n_m, box, mass=5.0)
        g = pm.gradient_fields(rho, box)
        u = x * (n_m / box) - 0.5
        idx, w = pm.cic_stencil(u, n_m)
        f = (g.reshape(3, -1)[:, idx] * w).sum(1)
        assert f.abs().max().item() < 1e-13


def test_gather_reproduces_linear_fields():
    n_p, n_m, box = 8, 16, 16.0                # dx = 1
    ax = (torch.arange(n_m, dtype=F64) + 0.5)
    x = torch.stack(torch.meshgrid(ax, ax, ax, indexing="ij"))
    fld = torch.stack([0.3 * x[0] - 0.2 * x[1] + 0.1 * x[2] + 1.0, 2.0 * x[2], -x[0] + x[1]])
    g = torch.Generator().manual_seed(3)
    s = 0.4 * torch.rand(3, n_p, n_p, n_p, generator=g, dtype=F64)
    q = lagrangian_grid(n_p, box)
    pos = q + s
    interior = ((pos > 1.0) & (pos < n_m - 1.0)).all(0).reshape(-1)
    got = pm.cic_gather(fld, s, n_p, box)[:, interior]
    p = pos.reshape(3, -1)[:, interior]
    exp = torch.stack([0.3 * p[0] - 0.2 * p[1] + 0.1 * p[2] + 1.0, 2.0 * p[2], -p[0] + p[1]])
    torch.testing.assert_close(got, exp, atol=1e-12, rtol=0)


def test_deposit_and_gather_are_adjoint():
    # sum_c rho_c g_c = m sum_p (gather g)_p for any mesh field g
    n_p, n_m, box = 8, 16, 20.0
    s = _clustered_displacements(n_p, box, 11, scale=4.0)
    fld = torch.randn(1, n_m, n_m, n_m, generator=torch.Generator().manual_seed(5), dtype=F64)
    rho = pm.cic_deposit(s, n_p, n_m, box)
    lhs = (rho * fld[0]).sum().item()
    rhs = (n_m / n_p) ** 3 * pm.cic_gather(fld, s, n_p, box).sum().item()
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_modes_with_a_nyquist_index_give_no_force(axis):
    # reading of the k-space operators: every mode with any |n_i| = N/2 is zeroed.
    # (-1)^c along one axis times cos(k y') along another is a single mode pair with
    # a Nyquist index and a non-zero wavenumber elsewhere: its force vanishes, while
    # keeping it would give a gradient along the other axis.
    n, box, amp = 16, 50.0, 0.3
    c = torch.arange(n, dtype=F64)
    alt = (-1.0) ** c
    other = (axis + 1) % 3
    x = (c + 0.5) * box / n
    k = 2 * math.pi / box * 2
    shape_a = [1, 1, 1]
    shape_a[axis] = n
    shape_o = [1, 1, 1]
    shape_o[other] = n
    rho = (1.0 + amp * alt.view(shape_a) * torch.cos(k * x).view(shape_o)).expand(n, n, n).contiguous()
    g = pm.gradient_fields(rho, box)
    assert g.abs().max().item() < 1e-14
    # the same field without the Nyquist factor has the full gradient -amp sin(k x) / k
    g2 = pm.gradient_fields((1.0 + amp * torch.cos(k * x).view(shape_o)).expand(n, n, n).contiguous(), box)
    expect = amp / k * torch.sin(k * x).abs().max().item()
    assert g2[other].abs().max().item() == pytest.approx(expect, rel=1e-12)
