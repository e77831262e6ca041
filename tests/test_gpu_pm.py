"""GPU parity of the CIC deposit and the PM force against the FP64 oracle.

Tolerances (derived from FP32 arithmetic): CIC weights carry ~1e-7 relative error;
the deposit rounds each of a cell's n contributions to 2^-32 and sums them exactly in
64-bit fixed point, then converts the cell to FP32 within one ulp, so the summation adds
at most n 2^-33 + 2^-23 of the cell's value (the bar below allows 1e-5, the bound an
arbitrary-order FP32 sum of n <= 10^4 terms would need, sqrt(n) 2^-24).  On
top of that the mesh coordinate t = s/dx - 1/2 is an FP32 number, so each weight
carries an absolute error of a few ulp(t) ~ |t| 2^-23: a cell reached by up to
8 such weights of mass m gets 8 m |t|max 2^-22 more.  The force adds the FFT
error (~1e-6 relative L2): bars rel L2 <= 1e-5 and max error <= 1e-4 of the rms.
"""
import numpy as np
import pytest
import torch

import paper_1301_0322_amd as cola
from oracle import pm
from paper_1301_0322_amd import inputs
from tests.gpu_util import announce, dev, host, max_rel_to_rms, rel_l2

pytestmark = pytest.mark.gpu

CASES = [(32, 64, 100.0), (16, 48, 50.0), (32, 32, 100.0), (24, 96, 80.0), (64, 128, 100.0)]


def _state(np_side, box, seed, rms):
    return inputs.displacements(np_side, box, seed, rms=rms)


# rms 0.3: lattice-like (one LDS pass per tile); 6: multi-pass boxes; 40: boxes
# spanning the periodic box (direct global path)
@pytest.mark.parametrize("np_side,nm,box", CASES)
@pytest.mark.parametrize("rms", [0.3, 6.0, 40.0])
def test_density_matches_oracle(np_side, nm, box, rms):
    announce(f"density np={np_side} nm={nm} rms={rms}")
    s = _state(np_side, box, 11, rms)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        rho = torch.empty(nm**3, dtype=torch.float32, device="cuda")
        plan.density(dev(s), rho, plan.workspace())
        got = host(rho).reshape(nm, nm, nm)
    ref = pm.cic_deposit(torch.from_numpy(s.astype(np.float64)).reshape(3, np_side, np_side, np_side),
                         np_side, nm, box).numpy()
    mass = (nm / np_side) ** 3
    t_max = np.abs(s).max() * nm / box + 1.0
    viol = np.abs(got - ref) / (1e-5 * ref + 8 * mass * t_max * 2.0**-22)
    worst = np.unravel_index(np.argmax(viol), viol.shape)
    print(f"[density np={np_side} nm={nm} rms={rms}] max |diff| {np.abs(got - ref).max():.3e} "
          f"(mean density 1), bar use {viol.max():.3f}", flush=True)
    assert viol.max() <= 1.0, (worst, float(got[worst]), float(ref[worst]), int((viol > 1).sum()))
    assert got.sum() == pytest.approx(nm**3, rel=1e-5)


@pytest.mark.parametrize("np_side,nm,box", CASES)
@pytest.mark.parametrize("rms", [0.3, 6.0, 40.0])
def test_pm_force_matches_oracle(np_side, nm, box, rms):
    announce(f"pm_force np={np_side} nm={nm} rms={rms}")
    s = _state(np_side, box, 5, rms)
    a = 0.55
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        acc = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
        plan.pm_force(dev(s), a, acc, plan.workspace())
        got = host(acc)
    ref = pm.pm_force(torch.from_numpy(s.astype(np.float64)).reshape(3, np_side, np_side, np_side), a,
                      np_side, nm, box, 0.3).reshape(3, -1).numpy()
    assert rel_l2(got, ref) < 1e-5
    assert max_rel_to_rms(got, ref) < 1e-4


def test_unperturbed_lattice_feels_no_force():
    announce("pm_force lattice")
    with cola.Plan(cola.Config(np=32, nm=64)) as plan:
        s = torch.zeros((3, 32**3), dtype=torch.float32, device="cuda")
        acc = torch.empty_like(s)
        plan.pm_force(s, 1.0, acc, plan.workspace())
        assert host(acc.abs().max()) < 1e-6


def _collapsed(np_side, nm, x0):
    """Displacements that put every particle at the point x0, in a box of nm unit cells
    (Lagrangian points q = i box/np; s = x0 - q, exact in FP32 for these sizes)."""
    q = np.arange(np_side) * (nm / np_side)
    qx, qy, qz = np.meshgrid(q, q, q, indexing="ij")
    return np.stack([x0[0] - qx, x0[1] - qy, x0[2] - qz]).reshape(3, -1).astype(np.float32)


def _point_density(nm, total, x0):
    """CIC of a single point mass on unit cells centred at c + 1/2 (the deposit's
    definition with all the mass in one particle)."""
    rho = np.zeros((nm, nm, nm))
    t = np.asarray(x0, dtype=np.float64) - 0.5
    c = np.floor(t).astype(int)
    f = t - c
    for a in (0, 1):
        for b in (0, 1):
            for e in (0, 1):
                w = (f[0] if a else 1 - f[0]) * (f[1] if b else 1 - f[1]) * (f[2] if e else 1 - f[2])
                rho[(c[0] + a) % nm, (c[1] + b) % nm, (c[2] + e) % nm] += total * w
    return rho


@pytest.mark.parametrize("np_side,nm", [(32, 64), (128, 256), (256, 512)])
def test_density_of_all_particles_at_one_point(np_side, nm):
    """The degenerate deposit: every particle in one cell of one tile (the whole particle
    set on the crowded-tile list, every LDS add on the same four cells).  The CIC
    fractions 1/4, 3/4 and 0 make each share and each sum exact, so the density must
    equal the point-mass closed form exactly: four cells holding nm^3 times 3/16, 9/16,
    1/16 and 3/16, every other cell zero."""
    announce(f"density all particles at one point np={np_side} nm={nm}")
    x0 = (10.75, 20.25, 30.5)
    s = _collapsed(np_side, nm, x0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=float(nm))) as plan:
        ws = plan.workspace()
        rho = torch.empty(nm**3, dtype=torch.float32, device="cuda")
        plan.density(dev(s), rho, ws)
        got = host(rho).reshape(nm, nm, nm)
        del ws, rho
        torch.cuda.empty_cache()
    ref = _point_density(nm, float(nm) ** 3, x0)
    assert np.count_nonzero(ref) == 4
    assert np.array_equal(got, ref.astype(np.float32)), (np.argwhere(got != ref)[:4], got[got != ref][:4])


def test_density_full_size_matches_oracle():
    """256^3 particles on the 512^3 mesh in the benchmarked launch configuration
    (bin depth 32), every cell against the oracle's FP64 deposit, same bar as the
    small cases; the clumped fifth of the particles puts tiles on the crowded list."""
    np_side, nm, box = 256, 512, 100.0
    announce("density 256/512")
    s = _state(np_side, box, 1302, 2.0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        assert plan.get_tuning()[2] == 32
        rho = torch.empty(nm**3, dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        plan.density(dev(s), rho, ws)
        got = host(rho).reshape(nm, nm, nm)
        del ws, rho
        torch.cuda.empty_cache()
    ref = pm.cic_deposit(torch.from_numpy(s.astype(np.float64)).reshape(3, np_side, np_side, np_side),
                         np_side, nm, box).numpy()
    mass = (nm / np_side) ** 3
    t_max = np.abs(s).max() * nm / box + 1.0
    viol = np.abs(got - ref) / (1e-5 * ref + 8 * mass * t_max * 2.0**-22)
    worst = np.unravel_index(np.argmax(viol), viol.shape)
    assert viol.max() <= 1.0, (worst, float(got[worst]), float(ref[worst]), int((viol > 1).sum()))
    assert got.astype(np.float64).sum() == pytest.approx(nm**3, rel=1e-6)
    assert ref.max() > 1000.0      # the clump: many particles per cell


def test_pm_force_full_size_matches_oracle():
    """256^3 particles on the 512^3 mesh, the benchmarked configuration."""
    np_side, nm, box = 256, 512, 100.0
    announce("pm_force 256/512")
    s = _state(np_side, box, 1302, 2.0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        acc = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        sd = dev(s)
        plan.pm_force(sd, 0.82, acc, ws)
        got = host(acc)
        # momentum conservation of the FP32 force at full size
        tot = np.abs(got.astype(np.float64).sum(axis=1)).max()
        assert tot < 1e-5 * np.abs(got).sum() / 3
        del ws, sd, acc
        torch.cuda.empty_cache()
    ref = pm.pm_force(torch.from_numpy(s).double().reshape(3, np_side, np_side, np_side), 0.82, np_side, nm,
                      box, 0.3).reshape(3, -1).numpy()
    assert rel_l2(got, ref) < 1e-5
    assert max_rel_to_rms(got, ref) < 2e-4


def test_pm_force_paper_mesh_full_size_matches_oracle():
    """256^3 particles on the paper's 768^3 mesh (3x per side), against the oracle,
    bars of the 512^3 case."""
    np_side, nm, box = 256, 768, 100.0
    announce("pm_force 256/768")
    s = _state(np_side, box, 1302, 2.0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        acc = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        plan.pm_force(dev(s), 0.82, acc, ws)
        got = host(acc)
        del ws, acc
        torch.cuda.empty_cache()
    ref = pm.pm_force(torch.from_numpy(s).double().reshape(3, np_side, np_side, np_side), 0.82, np_side, nm,
                      box, 0.3).reshape(3, -1).numpy()
    assert rel_l2(got, ref) < 1e-5
    assert max_rel_to_rms(got, ref) < 2e-4


@pytest.mark.parametrize("np_side,nm", [(32, 64), (128, 256)])
def test_fft_tile_shapes_agree(np_side, nm):
    """Every valid strided-pass tile width gives the same force bit for bit: the width
    sets how many columns one block transforms, not the arithmetic of a column."""
    s = dev(_state(np_side, 100.0, 9, 2.0))
    outs = {}
    for wy, wx in [(0, 0), (4, 4), (8, 8), (16, 16), (8, 16), (16, 8)]:
        announce(f"pm_force tiles y={wy} x={wx} nm={nm}")
        with cola.Plan(cola.Config(np=np_side, nm=nm)) as plan:
            plan.set_fft_tile(0, wy)
            plan.set_fft_tile(1, wx)
            acc = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
            plan.pm_force(s, 0.7, acc, plan.workspace())
            outs[(wy, wx)] = host(acc)
    ref = outs[(0, 0)]
    for key, got in outs.items():
        assert np.array_equal(got, ref), (key, rel_l2(got, ref))


def test_fft_tile_rejects_invalid_width():
    with cola.Plan(cola.Config(np=16, nm=16)) as plan:
        with pytest.raises(cola.ColaError):
            plan.set_fft_tile(0, 16)      # 16 does not divide nm/2 = 8
        with pytest.raises(cola.ColaError):
            plan.set_fft_tile(2, 8)


def test_binding_rejects_short_or_mistyped_buffers():
    with cola.Plan(cola.Config(np=16, nm=32)) as plan:
        s = torch.zeros(3, 16**3, device="cuda")
        rho = torch.empty(32**3, device="cuda")
        ws = plan.workspace()
        with pytest.raises(ValueError, match="ws"):
            plan.density(s, rho, ws[: ws.numel() // 2])
        with pytest.raises(ValueError, match="rho"):
            plan.density(s, rho[:-1], ws)
        with pytest.raises(ValueError, match="4-byte"):
            plan.density(s.double(), rho, ws)
        with pytest.raises(ValueError, match="contiguous"):
            plan.pm_force(torch.zeros(16**3, 3, device="cuda").t(), 0.5, s, ws)
        p = cola.Particles.empty(16)
        p.s2 = p.s2[:, :-1]
        with pytest.raises(ValueError, match="particles.s2"):
            plan.step(0, p, ws)
        plan.density(s, rho, ws)              # the well-formed call still runs
        torch.cuda.synchronize()
        assert abs(float(rho.double().sum()) - 32**3) < 1e-2


@pytest.mark.timeout(900)
def test_pm_force_large_mesh_matches_oracle():
    """The 1024^3 mesh of the large box (400 Mpc/h): 256^3 particles with Gaussian
    displacements of 8 Mpc/h rms (20 cells, the scale of the large box's z = 0
    displacements), force of eq. (eom) against the oracle's FP64 force at every
    particle.  Bars of the 512^3 case; the FFT error grows only as log n.

    No clump here: the clumped inputs pull a fifth of the particles across the box,
    to mesh coordinates |t| ~ 700 cells, where the FP32 rounding of t (|t| 2^-24 per
    rounding) moves the CIC weights by ~1e-4 of a cell and the force by about 1e-5
    relative; that is the precision of FP32 displacements, not of the FFT, and the
    density test below keeps the clump."""
    np_side, nm, box = 256, 1024, 400.0
    announce("pm_force 256/1024")
    s = inputs.displacements(np_side, box, 1303, rms=8.0, clump_frac=0.0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        acc = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        sd = dev(s)
        plan.pm_force(sd, 0.64, acc, ws)
        got = host(acc)
        del ws, sd, acc
        torch.cuda.empty_cache()
    announce("pm_force 256/1024: oracle")
    ref = pm.pm_force(torch.from_numpy(s).double().reshape(3, np_side, np_side, np_side), 0.64, np_side, nm,
                      box, 0.3).reshape(3, -1).numpy()
    e2, em = rel_l2(got, ref), max_rel_to_rms(got, ref)
    print(f"[pm_force 256/1024] rel L2 {e2:.3e}, max / rms {em:.3e}, "
          f"max |t| {np.abs(s).max() * nm / box:.0f} cells", flush=True)
    assert e2 < 1e-5
    assert em < 2e-4


@pytest.mark.timeout(900)
def test_density_large_box_matches_oracle():
    """The large-box workload's particle and mesh counts (512^3 particles on the 1024^3
    mesh, 400 Mpc/h; a fifth of the particles pulled into one clump): every one of the
    2^30 cells against the oracle's FP64 deposit, bar of the small cases.  This is also
    the parity check of the particle-index decode at np = 512."""
    np_side, nm, box = 512, 1024, 400.0
    announce("density 512/1024")
    s = _state(np_side, box, 1303, 4.0)
    with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
        rho = torch.empty(nm**3, dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        sd = dev(s)
        plan.density(sd, rho, ws)
        got = host(rho).reshape(nm, nm, nm)
        del ws, sd, rho
        torch.cuda.empty_cache()
    announce("density 512/1024: oracle")
    ref = pm.cic_deposit(torch.from_numpy(s).double().reshape(3, np_side, np_side, np_side), np_side, nm,
                         box).numpy()
    mass = (nm / np_side) ** 3
    t_max = np.abs(s).max() * nm / box + 1.0
    diff = np.abs(got - ref)
    viol = diff / (1e-5 * ref + 8 * mass * t_max * 2.0**-22)
    worst = np.unravel_index(np.argmax(viol), viol.shape)
    print(f"[density 512/1024] max |diff| {diff.max():.3e} (mean density 1), "
          f"max |diff| / rho {float((diff[ref > 1e-3] / ref[ref > 1e-3]).max()):.3e} where rho > 1e-3, "
          f"bar use {viol.max():.3f}", flush=True)
    assert viol.max() <= 1.0, (worst, float(got[worst]), float(ref[worst]), int((viol > 1).sum()))
    assert got.astype(np.float64).sum() == pytest.approx(nm**3, rel=1e-6)
