"""Writes tests/golden/adjoint_fd_128_256.txt: FP64 central differences of the loss of a
differentiable COLA run, computed with the oracle only.

Workload: 128^3 particles on a 256^3 mesh in a 100 Mpc/h box, 2LPT at z = 9 and 10
COLA steps to z = 0 (Section 2; eq. (ALCtimestep), eq. (KDKALC)); the loss is
L(w) = sum over the mesh of (rho(w) - rho_t)^2, rho the mean-1 CIC density of the
final positions and rho_t that of a second realization.  White noise w: seed 11
(inputs.white_noise), target noise: seed 12.  Directions: 32 unit vectors drawn from
numpy default_rng(DIR_SEED) standard normals, normalised.

For each direction d the file holds the central difference
  (L(w + eps d) - L(w - eps d)) / (2 eps)
at the eps chosen on the plateau of a sweep over 1e-2 .. 1e-6 (run with --sweep;
the sweep's table is written to the header).  The loss is piecewise smooth (cloud-in-
cell weights have kinks), so the difference quotient has a truncation error that
shrinks with eps until FP64 round-off of L / eps takes over.

With --autograd the script also writes, for the same directions, the oracle's exact
directional derivatives g.d (g = dL/dw by FP64 autograd through the oracle), read back
beside the stored differences: the two FP64 routes agree to the differences' accuracy.

Usage: python tests/golden/make_adjoint_fd.py [--sweep] [--eps EPS] [--autograd] [--threads N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cola as ocola            # noqa: E402
from oracle import cosmology as cosmo       # noqa: E402
from oracle import lpt, pm                  # noqa: E402
from paper_1301_0322_amd import inputs      # noqa: E402  (seeded inputs only; no method arithmetic)

NP, NM, BOX = 128, 256, 100.0
SEED_W, SEED_T = 11, 12
DIR_SEED = 4401
N_DIR = 32
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd_128_256.txt")
# The --sweep run that chose eps (directions 0 and 1): the quotient changes by 1.4% and
# 0.5% from 1e-2 to 1e-3 (larger steps cross more cloud-in-cell kinks) and by 7e-5 and
# 4e-5 from 1e-5 to 1e-6; 1e-6 is on the plateau, where FP64 round-off of L / eps
# (L ~ 3e9) is a few units, ~4e-5 of direction 0's quotient.
SWEEP = """eps     dir 0               dir 1
1e-02   104218.31953525543  447314.3164396286
1e-03   102771.91257476807  445263.36145401
1e-04   103064.4702911377   445773.83279800415
1e-05   103116.96529388426  445976.63879394525
1e-06   103110.07499694824  445994.37713623047"""


def config() -> cosmo.Config:
    return cosmo.Config(np_side=NP, nm_side=NM, box=BOX)


def final_density(w64: torch.Tensor, cfg: cosmo.Config, amp: float) -> torch.Tensor:
    s1, s2 = lpt.lpt_from_noise(w64, cfg, amp)
    _, _, s = ocola.evolve(s1, s2, cfg)
    return pm.cic_deposit(s, cfg.np_side, cfg.nm_side, cfg.box)


def target_density(cfg: cosmo.Config, amp: float) -> torch.Tensor:
    wt = torch.from_numpy(inputs.white_noise(NP, SEED_T).astype(np.float64))
    return final_density(wt, cfg, amp)


def loss(w64, cfg, amp, rho_t) -> float:
    return float(((final_density(w64, cfg, amp) - rho_t) ** 2).sum())


def oracle_gradient(cfg: cosmo.Config, amp: float, rho_t: torch.Tensor) -> np.ndarray:
    """dL/dw at the white noise of seed SEED_W by FP64 autograd through the oracle."""
    w = torch.from_numpy(inputs.white_noise(NP, SEED_W).astype(np.float64)).requires_grad_(True)
    (g,) = torch.autograd.grad(((final_density(w, cfg, amp) - rho_t) ** 2).sum(), w)
    return g.numpy()


def read_golden(path: str = OUT):
    """(eps, loss, fd per direction, autograd g.d per direction or None)."""
    eps, loss0, fd, ag = None, None, [], []
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if f[:2] == ["#", "eps"] and len(f) == 3:
                eps = float(f[2])
            elif f and f[0] == "loss":
                loss0 = float(f[1])
            elif f and f[0] == "dir":
                fd.append(float(f[2]))
            elif f and f[0] == "autograd":
                ag.append(float(f[2]))
    return eps, loss0, np.array(fd), (np.array(ag) if ag else None)


def write_golden(eps: float, l0: float, fd, ag=None, path: str = OUT):
    with open(path, "w") as fh:
        fh.write("# FP64 central differences of L(w) = sum (rho(w) - rho_t)^2, written by\n")
        fh.write(f"#   python tests/golden/make_adjoint_fd.py --eps {eps:g}\n")
        if ag is not None:
            fh.write("# and the oracle's autograd directional derivatives g.d, added by\n")
            fh.write("#   python tests/golden/make_adjoint_fd.py --autograd\n")
        fh.write(f"# np {NP} nm {NM} box {BOX} seed_w {SEED_W} seed_t {SEED_T} dir_seed {DIR_SEED} n_dir {N_DIR}\n")
        fh.write(f"# eps {eps!r}\n")
        fh.write("# eps sweep (--sweep):\n")
        for line in SWEEP.splitlines():
            fh.write(f"#   {line}\n")
        fh.write(f"loss {float(l0)!r}\n")
        for k, v in enumerate(fd):
            fh.write(f"dir {k} {float(v)!r}\n")
        if ag is not None:
            for k, v in enumerate(ag):
                fh.write(f"autograd {k} {float(v)!r}\n")


def directions() -> np.ndarray:
    rng = np.random.default_rng(DIR_SEED)
    d = rng.standard_normal((N_DIR, NP**3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--autograd", action="store_true")
    args = ap.parse_args()
    if args.threads:
        torch.set_num_threads(args.threads)
    cfg = config()
    amp = cosmo.power_amplitude(cfg)
    t0 = time.perf_counter()
    rho_t = target_density(cfg, amp)
    w0 = torch.from_numpy(inputs.white_noise(NP, SEED_W).astype(np.float64))
    l0 = loss(w0, cfg, amp, rho_t)
    print(f"L(w0) = {l0!r} ({time.perf_counter() - t0:.1f} s)", flush=True)
    dirs = directions()
    if args.autograd:
        eps, l_file, fd, _ = read_golden()
        if abs(l_file / l0 - 1.0) > 1e-12:
            raise SystemExit("the stored loss is not this workload's")
        g = oracle_gradient(cfg, amp, rho_t)
        ag = dirs @ g
        write_golden(eps, l_file, fd, ag)
        print("autograd g.d:", ag[:4], "... max |fd - g.d| / rms(fd):",
              float(np.abs(fd - ag).max() / np.sqrt(np.mean(fd**2))))
        return 0
    if args.sweep:
        for k in range(2):
            d = torch.from_numpy(dirs[k])
            for eps in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
                fd = (loss(w0 + eps * d, cfg, amp, rho_t) - loss(w0 - eps * d, cfg, amp, rho_t)) / (2 * eps)
                print(f"sweep dir {k} eps {eps:.0e} fd {fd!r}", flush=True)
        return 0
    if args.eps is None:
        raise SystemExit("--eps is required (choose it from --sweep)")
    rows = []
    for k in range(N_DIR):
        d = torch.from_numpy(dirs[k])
        fd = (loss(w0 + args.eps * d, cfg, amp, rho_t) - loss(w0 - args.eps * d, cfg, amp, rho_t)) / (2 * args.eps)
        rows.append(fd)
        print(f"dir {k} fd {fd!r} ({time.perf_counter() - t0:.0f} s)", flush=True)
    write_golden(args.eps, l0, rows)
    print("wrote", OUT)
    return 0


if __name__ == "__main__":
    sys.exit(main())
