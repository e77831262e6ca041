"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

cola_api.cpp and cosmology.cpp are compiled for the host with both sanitizers (the
device objects are linked as built), and tests/host/abi_host_driver.c drives every
entry point that needs no GPU: plan creation for each size class and flag set,
workspace sizes, the step table, every setter with valid and invalid values, tracing
switches, rejected configurations and error strings.  The run must finish with no
sanitizer report, leaks included.
"""
import os
import shutil
import subprocess

import pytest

from paper_1301_0322_amd import build as cola_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1301_0322_amd", "csrc")
DEVICE_SOURCES = ["kernels_fft.hip", "kernels_particles.hip", "noalloc.hip"]
SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]


def _device_object(src, tmp_path):
    """The build's object for a device source if it is newer than every source, else a
    fresh compile with the build's flags."""
    obj = os.path.join(cola_build.BUILD, os.path.splitext(src)[0] + ".o")
    newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC))
    if os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj
    out = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
    _run([cola_build.HIPCC, *cola_build.FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out])
    return out


@pytest.mark.timeout(900)
def test_host_code_is_clean_under_sanitizers(tmp_path):
    hipcc = cola_build.HIPCC
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not found")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
              f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}"]
    objs = []
    for src in ("cola_api.cpp", "cosmology.cpp"):
        out = str(tmp_path / (os.path.splitext(src)[0] + "_san.o"))
        _run([hipcc, "-x", "c++", "-std=c++17", *common, *SAN, "-c", os.path.join(CSRC, src), "-o", out])
        objs.append(out)
    drv = str(tmp_path / "driver.o")
    _run([hipcc, "-x", "c", *common, *SAN, "-c", os.path.join(ROOT, "tests", "host", "abi_host_driver.c"), "-o", drv])
    exe = str(tmp_path / "driver")
    _run([hipcc, "--offload-arch=gfx950", *SAN, drv, *objs, *[_device_object(s, tmp_path) for s in DEVICE_SOURCES],
          "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert r.stdout.strip().endswith("OK"), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
