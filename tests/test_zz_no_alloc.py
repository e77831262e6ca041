"""cola_density_noalloc (the allocation-free density for callers that cannot allocate)
against cola_density through the C-ABI.

The mass deposit sums 64-bit fixed point, so its result does not depend on the order
of the adds and both entry points give the same density bit for bit.  Two calls in a
row share the static scratch, the second with a smaller input; each is compared with
the workspace entry point on the same displacements.
"""
import numpy as np
import pytest
import torch

import paper_1301_0322_amd as cola
from paper_1301_0322_amd import inputs
from tests.gpu_util import announce, dev

pytestmark = pytest.mark.gpu

# (np, nm, box, seed, rms): the benchmarked 256^3/512^3 size first (binning buffers of
# 208 MB, most of the 256 MiB scratch), then a smaller one in the same scratch
CASES = [(256, 512, 100.0, 1302, 2.0), (32, 64, 100.0, 5, 6.0)]


def test_density_noalloc_matches_workspace_density():
    for np_side, nm, box, seed, rms in CASES:
        announce(f"density_noalloc np={np_side} nm={nm}")
        s = dev(inputs.displacements(np_side, box, seed, rms=rms))
        with cola.Plan(cola.Config(np=np_side, nm=nm, box=box)) as plan:
            ws = plan.workspace()
            ref = torch.empty(nm**3, dtype=torch.float32, device="cuda")
            plan.density(s, ref, ws)
            del ws
            got = torch.full_like(ref, float("nan"))
            plan.density_noalloc(s, got)
            torch.cuda.synchronize()
            same = torch.equal(got, ref)
            diff = (got - ref).abs().max().item()
            total = got.double().sum().item()
        assert same, (np_side, nm, diff)
        assert total == pytest.approx(nm**3, rel=1e-5)


def test_density_noalloc_rejects_tracing_plans():
    with cola.Plan(cola.Config(np=16, nm=32)) as plan:
        plan.trace_enable(1)
        s = torch.zeros((3, 16**3), dtype=torch.float32, device="cuda")
        rho = torch.empty(32**3, dtype=torch.float32, device="cuda")
        with pytest.raises(cola.ColaError) as e:
            plan.density_noalloc(s, rho)
        assert e.value.status == -1
