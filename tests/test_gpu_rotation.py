"""Rotated half-spectrum planes between the y passes and the x pass.

With rotation on, row y of x-plane x is stored at row (y + r x) mod n, r the x pass's
inner DFT length; only where rows sit in the workspace changes, never the arithmetic
of a transform, so every result must equal the plain-plane result bit for bit.  The
1024^3 mesh (rotated by default) is also compared with the oracle in test_gpu_pm.
"""
import numpy as np
import pytest
import torch

import paper_1301_0322_amd as cola
from paper_1301_0322_amd import inputs
from tests.gpu_util import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu

# inner DFT length of the x pass (the rotation in rows per plane) for each mesh size
R2 = {16: 4, 24: 8, 32: 8, 48: 8, 64: 8, 96: 16, 128: 16, 192: 16, 256: 16, 384: 16, 512: 32, 768: 24,
      1024: 32}


def _force(cfg, s, rot):
    with cola.Plan(cfg) as plan:
        plan.set_fft_rotation(rot)
        rows = plan.get_fft_rotation()
        acc = torch.empty((3, cfg.np**3), dtype=torch.float32, device="cuda")
        ws = plan.workspace()
        plan.pm_force(s, 0.61, acc, ws)
        out = host(acc)
        del ws, acc
        torch.cuda.empty_cache()
    return out, rows


@pytest.mark.parametrize("np_side,nm", [(16, 16), (16, 48), (32, 64), (48, 96), (64, 128), (96, 192),
                                        (128, 256), (96, 384), (128, 512), (128, 768)])
def test_force_is_identical_with_rotated_planes(np_side, nm):
    announce(f"rotation pm_force np={np_side} nm={nm}")
    cfg = cola.Config(np=np_side, nm=nm)
    s = dev(inputs.displacements(np_side, cfg.box, 21, rms=3.0))
    plain, r0 = _force(cfg, s, 0)
    rotated, r1 = _force(cfg, s, 1)
    assert (r0, r1) == (0, R2[nm])
    assert np.array_equal(plain, rotated), rel_l2(rotated, plain)
    assert np.abs(plain).max() > 0


@pytest.mark.timeout(600)
def test_force_is_identical_with_rotated_planes_large_mesh():
    """1024^3, where rotation is the default: plain planes give the same force."""
    announce("rotation pm_force np=128 nm=1024")
    cfg = cola.Config(np=128, nm=1024, box=400.0)
    s = dev(inputs.displacements(128, cfg.box, 22, rms=8.0, clump_frac=0.0))
    default, rd = _force(cfg, s, -1)
    plain, r0 = _force(cfg, s, 0)
    assert (rd, r0) == (32, 0)
    assert np.array_equal(plain, default), rel_l2(default, plain)


@pytest.mark.parametrize("n", [32, 64, 96])
def test_2lpt_is_identical_with_rotated_planes(n):
    """np = nm, so the plan's setting also governs the 2LPT transforms."""
    announce(f"rotation 2lpt n={n}")
    cfg = cola.Config(np=n, nm=n)
    w = dev(inputs.white_noise(n, 31))
    outs = []
    for rot in (0, 1):
        with cola.Plan(cfg) as plan:
            plan.set_fft_rotation(rot)
            p = cola.Particles.empty(n)
            plan.init_2lpt(w, p, plan.workspace())
            outs.append([host(t) for t in (p.s, p.v, p.s1, p.s2)])
    for name, a, b in zip(("s", "v", "s1", "s2"), *outs):
        assert np.array_equal(a, b), (name, rel_l2(b, a))


def test_adjoint_is_identical_with_rotated_planes():
    """Checkpointed run and its adjoint (transposed x passes, np = nm = 32).  Both the
    forward deposit and the adjoint's weighted deposits sum 64-bit fixed point, so the
    run and its gradient must agree bit for bit."""
    announce("rotation adjoint n=32")
    n = 32
    cfg = cola.Config(np=n, nm=n)
    w = dev(inputs.white_noise(n, 41))
    rng = np.random.default_rng(5)
    g_rho = dev(rng.standard_normal(n**3).astype(np.float32))
    grads = []
    for rot in (0, 1):
        with cola.Plan(cfg) as plan:
            plan.set_fft_rotation(rot)
            ws = plan.workspace()
            p = cola.Particles.empty(n)
            ckpt = torch.empty((cfg.n_steps + 1, 3, n**3), dtype=torch.float32, device="cuda")
            x = torch.empty((3, n**3), dtype=torch.float32, device="cuda")
            v = torch.empty_like(x)
            plan.run_checkpointed(w, p, x, v, ckpt, ws)
            g = torch.empty_like(w)
            plan.run_adjoint(w, ckpt, g_rho, g, plan.adjoint_workspace())
            grads.append((host(g), host(x)))
    assert np.array_equal(grads[0][1], grads[1][1])
    assert np.array_equal(grads[0][0], grads[1][0]), rel_l2(grads[1][0], grads[0][0])

