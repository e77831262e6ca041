"""The oracle's reference gradient (FP64 autograd through the whole run) against
central finite differences of the oracle itself (CPU only).

The loss L = sum_c (rho_c - rho_target_c)^2 of the final CIC density is piecewise
smooth (CIC weights have kinks at cell boundaries); small steps stay on one
smooth piece.  Bar: 1e-6 relative per direction.
"""
import numpy as np
import pytest
import torch

from oracle import cola as ocola
from oracle import cosmology as cosmo
from oracle import lpt, pm
from oracle.fourier import F64


def _loss(w, cfg, target):
    s1, s2 = lpt.lpt_from_noise(w, cfg)
    _, _, s = ocola.evolve(s1, s2, cfg)
    rho = pm.cic_deposit(s, cfg.np_side, cfg.nm_side, cfg.box)
    return ((rho - target) ** 2).sum()


def test_autograd_gradient_matches_central_differences():
    cfg = cosmo.Config(np_side=8, nm_side=16, n_steps=4)
    rng = np.random.default_rng(5)
    w0 = torch.tensor(rng.standard_normal(8**3), dtype=F64)
    target = torch.tensor(1.0 + 0.3 * rng.standard_normal((16, 16, 16)), dtype=F64)
    w = w0.clone().requires_grad_(True)
    loss = _loss(w, cfg, target)
    (grad,) = torch.autograd.grad(loss, w)
    for k in range(3):
        d = torch.tensor(rng.standard_normal(8**3), dtype=F64)
        d /= d.norm()
        eps = 1e-6
        with torch.no_grad():
            fd = (_loss(w0 + eps * d, cfg, target) - _loss(w0 - eps * d, cfg, target)) / (2 * eps)
        assert (grad @ d).item() == pytest.approx(fd.item(), rel=1e-6)


def test_stored_finite_differences_match_the_oracle_gradient():
    # tests/golden/adjoint_fd_128_256.txt holds, for 32 random directions of the
    # 128^3/256^3 differentiable workload, FP64 central differences of the oracle's loss
    # and the oracle's FP64 autograd directional derivatives (both written by
    # tests/golden/make_adjoint_fd.py): two independent routes to the same derivative,
    # which agree to the differences' accuracy (the eps sweep in the file's header)
    from tests.golden import make_adjoint_fd as fdg
    eps, loss, fd, ag = fdg.read_golden()
    assert eps == 1e-6 and len(fd) == fdg.N_DIR and ag is not None and len(ag) == fdg.N_DIR
    rms = np.sqrt(np.mean(fd**2))
    assert np.abs(fd - ag).max() <= 1e-4 * rms
