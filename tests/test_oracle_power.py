"""Pins of the oracle's shell-averaged power spectrum (CPU only)."""
import math

import pytest
import torch

from oracle import power
from oracle.fourier import F64


@pytest.mark.parametrize("nvec", [(1, 0, 0), (0, 2, 2), (3, -1, 4)])
def test_single_mode_power(nvec):
    # delta = A cos(k.x): the shell of |n| holds total power A^2 L^3 / 2
    n, box, amp = 16, 100.0, 0.2
    ax = (torch.arange(n, dtype=F64) + 0.5) * box / n
    x = torch.stack(torch.meshgrid(ax, ax, ax, indexing="ij"))
    k = 2 * math.pi / box * torch.tensor(nvec, dtype=F64)
    delta = amp * torch.cos((k.view(3, 1, 1, 1) * x).sum(0))
    pk, cnt = power.power_from_delta(delta, box)
    b = round(math.sqrt(sum(v * v for v in nvec)))
    assert (pk[b - 1] * cnt[b - 1]).item() == pytest.approx(amp**2 * box**3 / 2, rel=1e-12)
    others = torch.cat([pk[: b - 1], pk[b:]])
    assert others.abs().max().item() < 1e-20


def test_mode_counts_cover_the_sphere():
    n = 16
    pk, cnt = power.power_from_delta(torch.zeros(n, n, n, dtype=F64), 1.0)
    # number of integer vectors with round(|n|) = b inside the full grid
    full = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64).round()
    nx, ny, nz = torch.meshgrid(full, full, full, indexing="ij")
    sh = torch.round(torch.sqrt(nx**2 + ny**2 + nz**2)).to(torch.int64)
    for b in range(1, n // 2 + 1):
        assert cnt[b - 1].item() == (sh == b).sum().item()


def _fields(n=16, seed=3):
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(n, n, n, generator=g, dtype=F64), torch.randn(n, n, n, generator=g, dtype=F64),
            torch.randn(n, n, n, generator=g, dtype=F64))


def test_cross_spectrum_identities():
    a, b, c = _fields()
    box = 50.0
    pa, pb, px, cnt = power.cross_power_from_delta(a, b, box)
    # the auto spectra agree with the single-field estimator
    pa_ref, cnt_ref = power.power_from_delta(a, box)
    assert torch.allclose(pa, pa_ref, rtol=1e-13) and torch.equal(cnt, cnt_ref)
    # a field against itself, a positive and a negative multiple: rho = 1, 1, -1
    for f, sign in ((a, 1.0), (2.5 * a, 1.0), (-0.7 * a, -1.0)):
        qa, qb, qx, _ = power.cross_power_from_delta(a, f, box)
        rho, _ = power.correlation(qa, qb, qx)
        assert torch.allclose(rho, torch.full_like(rho, sign), atol=1e-12)
    # bilinear in the second field, symmetric in the two
    _, _, x_bc, _ = power.cross_power_from_delta(a, b + c, box)
    _, _, x_c, _ = power.cross_power_from_delta(a, c, box)
    assert torch.allclose(x_bc, px + x_c, rtol=1e-10, atol=1e-12)
    _, _, x_ba, _ = power.cross_power_from_delta(b, a, box)
    assert torch.allclose(x_ba, px, rtol=1e-13)
    # Cauchy-Schwarz per shell
    assert bool((px.abs() <= torch.sqrt(pa * pb) * (1 + 1e-12)).all())


def test_independent_fields_are_uncorrelated():
    # white noise fields: rho in each shell is a mean of n_b independent terms of
    # zero mean, so |rho| stays within a few / sqrt(n_b)
    a, b, _ = _fields(n=32, seed=11)
    pa, pb, px, cnt = power.cross_power_from_delta(a, b, 1.0)
    rho, _ = power.correlation(pa, pb, px)
    sel = cnt >= 50
    assert bool((rho[sel].abs() < 5.0 / torch.sqrt(cnt[sel])).all())


def test_n_max_normalisation():
    # Appendix B fixes the coefficient 2/3 so that n_max = 2 when the residual power
    # P_eps = P_NL - R^2 P_M is 10% of P_NL; with R = P_x / P_M that is
    # rho^2 = 1 - P_eps / P_NL = 0.9.  Build such a pair mode by mode:
    # delta_M = delta_NL + eps with eps orthogonal to delta_NL in every mode.
    n, box = 16, 1.0
    a, _, _ = _fields(n=n, seed=5)
    ka = torch.fft.rfftn(a)
    # eps_k = i c sign(n_x) delta_k is Hermitian (a real field) and orthogonal per mode;
    # modes with n_x = 0 or n_x = n/2 get eps = 0, so only shells free of them are exact
    nx = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64).round().view(n, 1, 1)
    sgn = torch.sign(nx) * (nx.abs() != n // 2)
    c = 1.0 / 3.0                     # P_eps / P_NL = c^2 = 1/9 where eps is non-zero
    km = ka + 1j * c * sgn * ka
    m = torch.fft.irfftn(km, s=(n, n, n))
    pm_, pnl, px, _ = power.cross_power_from_delta(m, a, box)
    rho, nmax = power.correlation(pm_, pnl, px)
    # rho = 1 / sqrt(1 + c^2) = sqrt(0.9) on modes with eps; check the mode-level
    # identity on the whole-box sums restricted to n_x != 0, n/2
    w = (sgn != 0).expand(n, n, n // 2 + 1)
    mult = torch.full((n, n, n // 2 + 1), 2.0, dtype=F64)
    mult[..., 0] = 1.0
    mult[..., n // 2] = 1.0
    kmm = torch.fft.rfftn(m)
    sx = (mult * (kmm * ka.conj()).real)[w].sum()
    sm = (mult * kmm.abs() ** 2)[w].sum()
    sa = (mult * ka.abs() ** 2)[w].sum()
    r = sx / torch.sqrt(sm * sa)
    assert r.item() == pytest.approx(math.sqrt(0.9), rel=1e-12)
    _, nm = power.correlation(sm, sa, sx)
    assert nm.item() == pytest.approx(2.0, rel=1e-11)
    # per shell, rho lies between sqrt(0.9) (all modes with eps) and 1
    assert bool(((rho >= math.sqrt(0.9) - 1e-12) & (rho <= 1 + 1e-12)).all())


def test_parseval_over_the_shells():
    # a zero-mean field band-limited to |n| < N/4 puts all its power inside shells
    # 1..N/2, so sum_b P_b n_b = (L^3 / N^6) sum_k |delta_k|^2 = (L^3 / N^3) sum_x delta_x^2
    n, box = 16, 37.0
    g = torch.Generator().manual_seed(9)
    white = torch.randn(n, n, n, generator=g, dtype=F64)
    dk = torch.fft.rfftn(white)
    f = torch.fft.fftfreq(n, d=1.0 / n, dtype=F64)
    kz = torch.fft.rfftfreq(n, d=1.0 / n, dtype=F64)
    mag = torch.sqrt(f.view(n, 1, 1) ** 2 + f.view(1, n, 1) ** 2 + kz.view(1, 1, -1) ** 2)
    dk = torch.where((mag < n / 4) & (mag > 0), dk, torch.zeros_like(dk))
    delta = torch.fft.irfftn(dk, s=(n, n, n))
    pk, cnt = power.power_from_delta(delta, box)
    lhs = (pk * cnt).sum().item()
    rhs = box**3 / n**3 * (delta**2).sum().item()
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # and the cross estimator of a field with itself gives the same numbers
    pa, pb, px, cnt2 = power.cross_power_from_delta(delta, delta, box)
    assert torch.allclose(px, pk, rtol=1e-13) and torch.equal(cnt2, cnt)
