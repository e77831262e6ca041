"""Batched ensembles (one hipGraph, one branch per member) and the autotuner.

Every graph replay is checked against eager runs of the same members, with eager
work and synchronisations between replays.  The replays equal the eager runs bit for
bit: a graph replays the same kernels, the mass deposit sums 64-bit fixed point
(independent of particle order), and no result depends on the tile shapes.
"""
import numpy as np
import pytest
import torch

import paper_1301_0322_amd as cola
from paper_1301_0322_amd import inputs
from tests.gpu_util import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu

MEMBERS = [(16, 32, 101), (24, 48, 102), (16, 32, 103), (32, 64, 104)]


def test_ensemble_graph_replays_match_eager_runs():
    plans = [cola.Plan(cola.Config(np=n, nm=m)) for n, m, _ in MEMBERS]
    noises = [dev(inputs.white_noise(n, seed)) for n, _, seed in MEMBERS]
    eager = []
    for (n, m, _), w in zip(MEMBERS, noises):
        x, v, _ = cola.run(cola.Config(np=n, nm=m), w)
        eager.append((host(x), host(v)))
    announce("ensemble create")
    ens = cola.Ensemble(plans, noises)
    a = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for t in ens.x + ens.v:
            t.fill_(float("nan"))
        announce(f"ensemble launch {rep}")
        ens.launch()
        torch.cuda.synchronize()
        for k, (ex, ev) in enumerate(eager):
            gx, gv = host(ens.x[k]), host(ens.v[k])
            assert np.array_equal(gx, ex), (rep, k, rel_l2(gx, ex))
            assert np.array_equal(gv, ev), (rep, k, rel_l2(gv, ev))
        # eager work between replays
        a = (a @ a.T) / 512.0
        torch.cuda.synchronize()
    ens.close()
    for p in plans:
        p.close()


def test_autotune_picks_valid_shapes_and_caches(tmp_path):
    cache = str(tmp_path / "tune.txt")
    cfg = cola.Config(np=64, nm=128)
    w = dev(inputs.white_noise(64, 7))
    with cola.Plan(cfg) as ref_plan:
        p = cola.Particles.empty(64)
        ref_plan.init_2lpt(w, p, ref_plan.workspace())
        acc_ref = torch.empty_like(p.s)
        ref_plan.pm_force(p.s, 0.6, acc_ref, ref_plan.workspace())
    announce("autotune")
    with cola.Plan(cfg) as plan:
        assert plan.autotune(p, None, cache) is False
        y, x, tz = plan.get_tuning()
        assert y in (4, 8, 16) and x in (4, 8, 16) and tz in (8, 16, 32, 64)
        acc = torch.empty_like(p.s)
        plan.pm_force(p.s, 0.6, acc, plan.workspace())
        assert rel_l2(host(acc), host(acc_ref)) < 2e-6
    with cola.Plan(cfg) as plan2:
        assert plan2.autotune(p, None, cache) is True
        assert plan2.get_tuning() == (y, x, tz)
    assert "np=64 nm=128" in open(cache).read()
