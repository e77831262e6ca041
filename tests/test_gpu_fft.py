"""GPU parity of the 3D real FFT passes against the oracle's FP64 FFT.

Tolerance: FP32 radix-2/3/4/8 Stockham passes with exactly-rounded twiddles have a
relative L2 error of order eps32 * log2(n^3) ~ 1e-6; the bar is 2e-6.
"""
import math

import numpy as np
import pytest
import torch

import paper_1301_0322_amd as cola
from oracle.fourier import irfft3, rfft3
from paper_1301_0322_amd import inputs
from tests.gpu_util import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu

PLANS = [(16, 48), (24, 96), (32, 64), (64, 128), (96, 192), (128, 384), (256, 512), (256, 768), (512, 1024)]


@pytest.mark.parametrize("np_side,nm", PLANS)
def test_r2c_matches_oracle(np_side, nm):
    with cola.Plan(cola.Config(np=np_side, nm=nm)) as plan:
        for n in sorted({np_side, nm}):
            if n > 512:
                continue  # host FP64 FFT of 1024^3 is covered by the roundtrip test
            announce(f"fft_r2c n={n}")
            x = inputs.mesh_field(n, seed=n)
            out = torch.empty(n**3, dtype=torch.float32, device="cuda")
            plan.fft_r2c(n, dev(x), out)
            got = host(out).view(np.complex64).reshape(n, n, n // 2)
            ref = rfft3(torch.from_numpy(x).double()).numpy()[..., : n // 2]
            err = rel_l2(got, ref)
            assert err < 2e-6, (n, err)


@pytest.mark.parametrize("np_side,nm", PLANS)
def test_c2r_matches_oracle(np_side, nm):
    with cola.Plan(cola.Config(np=np_side, nm=nm)) as plan:
        for n in sorted({np_side, nm}):
            if n > 512:
                continue
            announce(f"fft_c2r n={n}")
            x = inputs.mesh_field(n, seed=n + 1).astype(np.float64)
            half = rfft3(torch.from_numpy(x))
            half[..., n // 2] = 0
            ref = irfft3(half, n).numpy()
            src = np.ascontiguousarray(half[..., : n // 2].numpy().astype(np.complex64))
            inp = dev(src.view(np.float32).reshape(-1))
            out = torch.empty(n**3, dtype=torch.float32, device="cuda")
            plan.fft_c2r(n, inp, out)
            assert rel_l2(host(out).reshape(n, n, n), ref) < 2e-6
            # the input buffer is left untouched
            assert np.array_equal(host(inp), src.view(np.float32).reshape(-1))


def test_roundtrip_largest_mesh():
    n = 1024
    with cola.Plan(cola.Config(np=512, nm=n)) as plan:
        announce("fft roundtrip n=1024")
        g = torch.Generator(device="cuda").manual_seed(7)
        # band-limited field: build it from a half spectrum without the kz = n/2 plane
        x = torch.randn(n**3, generator=g, device="cuda", dtype=torch.float32)
        spec = torch.empty_like(x)
        plan.fft_r2c(n, x, spec)
        back = torch.empty_like(x)
        plan.fft_c2r(n, spec, back)
        spec2 = torch.empty_like(x)
        plan.fft_r2c(n, back, spec2)
        err = (torch.linalg.vector_norm((spec2 - spec).double()) / torch.linalg.vector_norm(spec.double())).item()
        assert err < 4e-6
        # Parseval on the projected field: sum back^2 = (2 sum|X|^2 - |X(kz=0)|^2) / n^3
        xs = spec.view(n, n, n // 2, 2).double()
        p = (xs**2).sum(-1)
        tot = 2 * p.sum() - p[..., 0].sum()
        assert math.isclose((back.double() ** 2).sum().item(), tot.item() / n**3, rel_tol=1e-5)
        del x, spec, back, spec2
        torch.cuda.empty_cache()


def test_fft_rejects_foreign_size():
    with cola.Plan(cola.Config(np=32, nm=64)) as plan:
        buf = torch.empty(128**3, dtype=torch.float32, device="cuda")
        with pytest.raises(cola.ColaError):
            plan.fft_r2c(128, buf, buf)


# ------------------------------------------------------------------------------------
# Every size, 768 and 1024 included, against an analytic spectrum: a sum of a few
# cosines f(j) = sum_m a_m cos(2 pi k_m.j / n + phi_m) has the DFT
# F(k) = (n^3 a_m / 2) e^{+-i phi_m} at k = +-k_m and zero elsewhere.  No host FFT is
# needed, so the largest meshes are compared element by element.  Modes have
# 1 <= kz <= n/2 - 1 (only +k_m lies in the stored half spectrum) except one kz = 0
# mode, whose conjugate partner (-kx, -ky, 0) is stored too.  Inputs are built on the
# device in float64 from exact integer phases, then rounded to float32.
# ------------------------------------------------------------------------------------
def _modes(n):
    h = n // 2
    return [((1, 2, 3), 1.0, 0.3), ((n - 5, 7, h - 1), 0.5, -1.1), ((h - 3, n - 1, 1), 0.25, 2.0),
            ((3, n - 4, 0), 0.75, 0.7)]


def _cosine_field(n):
    dev_ = torch.device("cuda")
    ax = torch.arange(n, device=dev_, dtype=torch.int64)
    f = torch.zeros((n, n, n), dtype=torch.float64, device=dev_)
    for (kx, ky, kz), a, ph in _modes(n):
        m = (kx * ax.view(n, 1, 1) + ky * ax.view(1, n, 1) + kz * ax.view(1, 1, n)) % n
        f += a * torch.cos(m.double() * (2 * math.pi / n) + ph)
        del m
    return f


def _expected_coefficients(n):
    """{(kx, ky, kz): complex} over the stored half spectrum (kz < n/2)."""
    out = {}
    for (kx, ky, kz), a, ph in _modes(n):
        c = 0.5 * a * n**3
        out[(kx, ky, kz)] = out.get((kx, ky, kz), 0) + c * complex(math.cos(ph), math.sin(ph))
        if kz == 0:
            key = ((-kx) % n, (-ky) % n, 0)
            out[key] = out.get(key, 0) + c * complex(math.cos(ph), -math.sin(ph))
    return out


ALL_SIZES = sorted({n for pair in PLANS for n in pair})


@pytest.mark.parametrize("n", ALL_SIZES)
def test_r2c_matches_analytic_spectrum(n):
    with cola.Plan(cola.Config(np=n, nm=n)) as plan:
        announce(f"fft_r2c analytic n={n}")
        x = _cosine_field(n).float().reshape(-1)
        out = torch.empty(n**3, dtype=torch.float32, device="cuda")
        plan.fft_r2c(n, x, out)
        del x
        spec = out.view(n, n, n // 2, 2)
        total = (spec.double() ** 2).sum().item()
        exp = _expected_coefficients(n)
        err2, ref2, at_modes = 0.0, 0.0, 0.0
        for (kx, ky, kz), c in exp.items():
            re, im = (float(v) for v in spec[kx, ky, kz].double().cpu())
            at_modes += re * re + im * im
            err2 += (re - c.real) ** 2 + (im - c.imag) ** 2
            ref2 += abs(c) ** 2
        leak2 = max(total - at_modes, 0.0)
        err = math.sqrt((err2 + leak2) / ref2)
        print(f"[r2c analytic n={n}] rel L2 {err:.3e} (leakage {math.sqrt(leak2 / ref2):.3e})", flush=True)
        del out, spec
        torch.cuda.empty_cache()
    assert err < 2e-6, err


@pytest.mark.parametrize("n", ALL_SIZES)
def test_c2r_matches_analytic_field(n):
    with cola.Plan(cola.Config(np=n, nm=n)) as plan:
        announce(f"fft_c2r analytic n={n}")
        half = torch.zeros((n, n, n // 2, 2), dtype=torch.float32, device="cuda")
        for (kx, ky, kz), c in _expected_coefficients(n).items():
            half[kx, ky, kz, 0] = c.real
            half[kx, ky, kz, 1] = c.imag
        out = torch.empty(n**3, dtype=torch.float32, device="cuda")
        plan.fft_c2r(n, half.view(-1), out)
        del half
        ref = _cosine_field(n)
        got = out.view(n, n, n).double()
        err = (torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref)).item()
        print(f"[c2r analytic n={n}] rel L2 {err:.3e}", flush=True)
        del out, ref, got
        torch.cuda.empty_cache()
    assert err < 2e-6, err
