"""Host check of the particle-index decode's division by np.

The kernels split a Lagrangian index p = (ix np + iy) np + iz with two divisions by np,
each a multiply-shift by the constants that set_lattice_divisor (csrc/internal.hpp)
computes (Granlund and Montgomery 1994, round-up method).  This test builds a small host
program against that header, takes the constants from the library's own function and
checks the multiply-shift quotient against exact integer division:
  - for every np of the form 2^a 3^b up to 1024 (the supported sizes): every index
    p < np^3 and its second-level quotient, exhaustively;
  - for every np from 1 to 1024: the exactness condition of the method and dividends
    at and around every multiple of np near 0 and near 2^31, plus random ones.
The kernel's expression is restated here; the test also checks that the kernel source
still contains it verbatim.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1301_0322_amd", "csrc")
DEVICE_EXPR = "(unsigned)(((unsigned long long)x * lat.np_magic) >> (31 + lat.np_shift))"

PROGRAM = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include "internal.hpp"

static unsigned div_np(const cola::Lattice& lat, unsigned x) {
  return (unsigned)(((unsigned long long)x * lat.np_magic) >> (31 + lat.np_shift));
}

static int check(int np, unsigned x) {
  cola::Lattice l{};
  l.np = np;
  cola::set_lattice_divisor(l);
  if (div_np(l, x) != x / (unsigned)np) {
    std::printf("FAIL np=%d x=%u got=%u want=%u\n", np, x, div_np(l, x), x / (unsigned)np);
    return 1;
  }
  return 0;
}

int main() {
  long checked = 0;
  // every supported size: all Lagrangian indices and their second-level quotients
  const int sizes[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  for (int np : sizes) {
    cola::Lattice l{};
    l.np = np;
    cola::set_lattice_divisor(l);
    const unsigned long long n3 = (unsigned long long)np * np * np;
    for (unsigned long long p = 0; p < n3; ++p) {
      const unsigned q = div_np(l, (unsigned)p);
      if (q != (unsigned)(p / np)) { std::printf("FAIL np=%d p=%llu\n", np, p); return 1; }
      if (div_np(l, q) != q / (unsigned)np) { std::printf("FAIL np=%d q=%u\n", np, q); return 1; }
    }
    checked += (long)n3;
  }
  // every divisor up to 1024: the method's exactness condition and edge dividends < 2^31
  std::mt19937 rng(12345);
  for (int np = 1; np <= 1024; ++np) {
    cola::Lattice l{};
    l.np = np;
    cola::set_lattice_divisor(l);
    const unsigned long long m = l.np_magic, two = 1ULL << (31 + l.np_shift);
    if (!((1ULL << l.np_shift) >= (unsigned long long)np && m * (unsigned long long)np > two &&
          m * (unsigned long long)np <= two + (1ULL << l.np_shift))) {
      std::printf("FAIL condition np=%d\n", np);
      return 1;
    }
    const unsigned top = 0x7fffffffu;
    for (unsigned k = 0; k < 64; ++k) {
      const unsigned lo = k * (unsigned)np;
      const unsigned hi = (top / (unsigned)np - k) * (unsigned)np;
      for (int d = -1; d <= 1; ++d) {
        if (lo + d <= top && !(k == 0 && d < 0)) { if (check(np, lo + d)) return 1; }
        if (hi + d <= top) { if (check(np, hi + d)) return 1; }
      }
    }
    if (check(np, top)) return 1;
    for (int r = 0; r < 4096; ++r) if (check(np, rng() & top)) return 1;
    checked += 64 * 6 + 4097;
  }
  std::printf("OK %ld\n", checked);
  return 0;
}
"""


def test_kernel_division_expression_is_the_one_checked():
    src = open(os.path.join(CSRC, "kernels_particles.hip")).read()
    assert DEVICE_EXPR in src


@pytest.mark.timeout(600)
def test_lattice_divisor_is_exact(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    cpp = tmp_path / "divisor_check.cpp"
    exe = tmp_path / "divisor_check"
    cpp.write_text(PROGRAM)
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    # a host-only build: internal.hpp's HIP types come from the runtime headers
    subprocess.run([hipcc, "-x", "c++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
                    f"-I{CSRC}", str(cpp), "-o", str(exe)], check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout
