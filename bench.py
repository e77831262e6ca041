#!/usr/bin/env python3
"""Benchmark of the COLA particle-mesh run on one MI355X.

A bench step is one pass of the whole hot path on one batch of synthetic input:
2LPT initial conditions from white noise, the COLA steps (CIC deposit, r2c FFT,
Poisson + gradient, three c2r FFTs, CIC gather + kick + drift) and the closing
kick with L+.  Inputs (the white noise) are resident in HBM before timing starts.

value = np^3 * n_steps / (seconds per bench step): whole-job particle-steps/s.
Also reported: the PM step time (each COLA step inside cola_run, HIP events
around the step), each kernel stage's time from HIP events on the launch stream, the roofline of the
dominant kernel (algorithmic bytes per launch / its mean duration against the
8 TB/s HBM peak) and the FP64 CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

CONFIGS = {
    # name: (np, nm, box, seed, description)
    "c0": (32, 64, 100.0, 1301, "32^3 particles / 64^3 mesh, 100 Mpc/h"),
    "c1": (256, 512, 100.0, 1302, "256^3 particles / 512^3 mesh, 100 Mpc/h"),
    "c2": (512, 1024, 400.0, 1303, "512^3 particles / 1024^3 mesh, 400 Mpc/h"),
    "c4": (128, 256, 100.0, 11, "128^3 particles / 256^3 mesh, 100 Mpc/h"),
    # the paper's own mesh refinement (3x per side)
    "c1_paper_mesh": (256, 768, 100.0, 1302, "256^3 particles / 768^3 mesh, 100 Mpc/h"),
}


def stage_bytes(np_side: int, nm: int) -> dict:
    """Algorithmic HBM bytes per launch of each stage (each array read and written
    once per pass; R = nm^3 reals, C = nm^2 (nm/2 + 1) complex, P = np^3)."""
    R = nm**3
    C = nm * nm * (nm // 2 + 1)
    P = np_side**3
    Rp = np_side**3
    Cp = np_side * np_side * (np_side // 2 + 1)
    return {
        "deposit": 12 * P + 4 * R,
        "fft_z_fwd": 4 * R + 8 * C,
        "fft_y_fwd": 16 * C,
        "fft_x_poisson": 8 * C + 16 * C,   # writes i n_x Phi and Phi
        "fft_y_inv": 16 * C,               # the x component
        "fft_y_inv_pair": 8 * C + 16 * C,  # Phi -> i n_y Phi and Phi
        "fft_z_inv": 8 * C + 4 * R,        # one force component per launch
        "gather_kick_drift": 12 * R + 72 * P,
        "gather_finish": 12 * R + 48 * P + 36 * P,
        "fill": 0,
        # 2LPT on the particle grid (per launch; the x and y passes handle 9 or 3 fields)
        "lpt_fft_z_fwd": 4 * Rp + 8 * Cp,
        "lpt_fft_y_fwd": 16 * Cp,
        "lpt_fft_x_mul": 8 * Cp + 6 * 8 * Cp,       # mean of the 9- and 3-output launches
        "lpt_fft_y_inv": 6 * 16 * Cp,
        "lpt_fft_z_inv": 3 * (8 * Cp + 4 * Rp) + 3 * 4 * Rp,
        "lpt_hessian": 6 * 8 * Cp + 4 * Rp,
    }


def b_alg_step(np_side: int, nm: int) -> int:
    """Bytes one PM step must move with this pass structure: deposit, z and y forward,
    the x pass (2 outputs), the y passes (x component; Phi -> y, z components), three z
    inverse passes, gather + kick + drift: 84 P + 32 R + 112 C."""
    R = nm**3
    C = nm * nm * (nm // 2 + 1)
    return 84 * np_side**3 + 32 * R + 112 * C


def b_alg_three_chains(np_side: int, nm: int) -> int:
    """The same with three independent inverse chains (one per force component):
    84 P + 32 R + 128 C."""
    R = nm**3
    C = nm * nm * (nm // 2 + 1)
    return 84 * np_side**3 + 32 * R + 128 * C


def csrc_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1301_0322_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(stage: str, workload: str):
    """HBM bytes per launch from the committed PMC summary, if it is for this
    kernel source and workload; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"pmc_{stage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != csrc_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# kernel of each timed stage, by bin depth, as rocprofv3 names it
STAGE_KERNEL = {"gather_kick_drift": "k_gather_sorted<{tz}, 1>",
                "deposit": "k_deposit_tiles<{tz}, unsigned long long, 1>"}


def read_profile_avg(stage: str, workload: str, tz: int):
    """Mean kernel duration (ms) of a stage's kernel in the committed rocprofv3
    kernel-trace summary, if it is for this kernel source, workload and bin depth."""
    path = os.path.join(ROOT, "profiles", f"kernel_trace_cola_run_{workload}.txt")
    if stage not in STAGE_KERNEL or not os.path.exists(path):
        return None
    name = STAGE_KERNEL[stage].format(tz=tz)
    digest = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_digest:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith(name + " ") and digest == csrc_digest():
                cols = line[len(name):].split()
                try:
                    return {"file": os.path.relpath(path, ROOT), "kernel": name, "calls": int(cols[0]),
                            "avg_ms": float(cols[1]) * 1e-3}
                except (IndexError, ValueError):
                    return None
    return None


# ------------------------------------------------------------------------------------
# rocprofv3 summaries (the text files under profiles/): --rocprof-trace DIR reads the
# kernel_trace.csv files of a `rocprofv3 --kernel-trace --output-format csv -d DIR` run,
# --rocprof-pmc DIR the counter_collection.csv files of a `--pmc` run.
# ------------------------------------------------------------------------------------
def _short_kernel_name(name: str) -> str:
    name = name.strip().strip('"')
    if name.startswith("void "):
        name = name[5:]
    depth, out = 0, []
    for ch in name:            # drop the argument list, keep template arguments
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).replace("cola::", "").strip()


def _csv_rows(directory: str, suffix: str):
    import csv
    rows = []
    for root, _, files in os.walk(directory):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(root, f), newline="") as fh:
                    rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {directory}")
    return rows


def rocprof_trace_summary(directory: str, per_dispatch=("k_deposit_tiles", "k_gather_sorted")) -> str:
    """Kernel table (calls, mean and total duration, share) of a kernel trace, and the
    duration of every dispatch, in launch order, of the kernels named in per_dispatch."""
    rows = _csv_rows(directory, "kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    stats, seq = {}, {}
    for r in rows:
        name = _short_kernel_name(r["Kernel_Name"])
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3   # us
        c, t = stats.get(name, (0, 0.0))
        stats[name] = (c + 1, t + dt)
        if any(name.startswith(k) for k in per_dispatch):
            seq.setdefault(name, []).append(dt)
    total = sum(t for _, t in stats.values())
    lines = [f"source_digest: {csrc_digest()}", "",
             f"{'kernel':<52} {'calls':>6} {'avg_us':>10} {'total_ms':>10} {'pct':>6}"]
    for name, (c, t) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{name:<52} {c:>6} {t / c:>10.1f} {t * 1e-3:>10.3f} {100 * t / total:>6.2f}")
    for name, v in seq.items():
        lines.append("")
        lines.append(f"per-dispatch us, {name} (launch order): " + " ".join(f"{x:.1f}" for x in v))
    return "\n".join(lines)


def rocprof_busy_summary(directory: str, gap_us: float = 2000.0, min_dispatches: int = 200) -> str:
    """GPU-busy fraction of each launch window of a kernel trace: dispatches are split
    into windows at idle gaps longer than gap_us (a host synchronisation between
    launches); for each window with at least min_dispatches kernels, busy = the length
    of the union of the kernel intervals, wall = last end - first start."""
    rows = _csv_rows(directory, "kernel_trace.csv")
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    windows, cur, last_end = [], [], None
    for a, b in iv:
        if cur and a - last_end > gap_us * 1e3:
            windows.append(cur)
            cur = []
        last_end = b if not cur else max(last_end, b)
        cur.append((a, b))
    if cur:
        windows.append(cur)
    lines = [f"source_digest: {csrc_digest()}", "",
             f"{'window':>6} {'dispatches':>10} {'wall_ms':>10} {'busy_ms':>10} {'busy_frac':>9} {'sum_kernel_ms':>13}"]
    for k, w in enumerate(windows):
        if len(w) < min_dispatches:
            continue
        busy, s0, e0 = 0, None, None
        for a, b in w:
            if s0 is None or a > e0:
                if s0 is not None:
                    busy += e0 - s0
                s0, e0 = a, b
            else:
                e0 = max(e0, b)
        busy += e0 - s0
        wall = max(b for _, b in w) - w[0][0]
        tot = sum(b - a for a, b in w)
        lines.append(f"{k:>6} {len(w):>10} {wall * 1e-6:>10.3f} {busy * 1e-6:>10.3f} {busy / wall:>9.3f} "
                     f"{tot * 1e-6:>13.3f}")
    return "\n".join(lines)


def _counter_values(directory: str, counter: str):
    """{short kernel name: [value per dispatch]} of one counter, and the values of the
    256 MiB calibration copy (--copy-calibration)."""
    out, calib = {}, []
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        name = _short_kernel_name(r["Kernel_Name"])
        out.setdefault(name, []).append(float(r["Counter_Value"]))
        if "copyBuffer" in name:
            calib.append(float(r["Counter_Value"]))
    return out, calib


def rocprof_hbm_summary(fetch_dir: str, write_dir: str, stage: str = "", tz: int = 32) -> str:
    """HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE run (KiB per
    dispatch), each scaled so that the 256 MiB device-to-device calibration copy of the
    same command reads and writes 256 MiB.  With stage, the key: value block that
    read_traffic() reads for that stage's kernel; else a table of every kernel."""
    fetch, fcal = _counter_values(fetch_dir, "FETCH_SIZE")
    write, wcal = _counter_values(write_dir, "WRITE_SIZE")
    kib = 256 * 1024
    # the calibration copy is the only copy whose WRITE_SIZE is 256 MiB
    wc = [v for v in wcal if abs(v - kib) < 0.01 * kib]
    if not wc:
        raise SystemExit("no 256 MiB calibration copy in the WRITE_SIZE run (use --copy-calibration)")
    fc = [v for v in fcal if abs(2 * v - kib) < 0.05 * kib or abs(v - kib) < 0.05 * kib]
    fscale, wscale = kib / fc[-1], kib / wc[-1]
    hbm = {k: (sum(fetch[k]) / len(fetch[k]), sum(write[k]) / len(write[k]), len(fetch[k]))
           for k in fetch if k in write}
    lines = [f"fetch_scale: {fscale:.4f}", f"write_scale: {wscale:.4f}", f"source_digest: {csrc_digest()}", ""]
    if stage:
        name = STAGE_KERNEL[stage].format(tz=tz)
        f, w, n = hbm[name]
        tot = f * 1024 * fscale + w * 1024 * wscale
        alg = stage_bytes(256, 512)[stage]
        lines += [f"kernel: {name}", f"launches_counted: {n}", f"fetch_kib_per_launch: {f:.1f}",
                  f"write_kib_per_launch: {w:.1f}", f"hbm_bytes_per_launch: {tot:.0f}",
                  f"algorithmic_bytes_per_launch: {alg}", f"traffic_over_algorithmic: {tot / alg:.2f}"]
    else:
        lines.append(f"{'kernel':<52} {'dispatches':>10} {'fetch_KiB':>12} {'write_KiB':>12} {'hbm_GB':>9}")
        for k, (f, w, n) in sorted(hbm.items(), key=lambda kv: -(kv[1][0] * fscale + kv[1][1] * wscale)):
            lines.append(f"{k:<52} {n:>10} {f:>12.1f} {w:>12.1f} {(f * fscale + w * wscale) * 1024 / 1e9:>9.3f}")
    return "\n".join(lines)


def rocprof_pmc_summary(directory: str) -> str:
    """Mean value per dispatch of every collected counter, per kernel."""
    rows = _csv_rows(directory, "counter_collection.csv")
    acc = {}
    for r in rows:
        name = _short_kernel_name(r["Kernel_Name"])
        key = (name, r["Counter_Name"])
        c, t = acc.get(key, (0, 0.0))
        acc[key] = (c + 1, t + float(r["Counter_Value"]))
    lines = [f"source_digest: {csrc_digest()}", "", f"{'kernel':<52} {'counter':<28} {'dispatches':>10} {'mean':>16}"]
    for (name, ctr), (c, t) in sorted(acc.items()):
        lines.append(f"{name:<52} {ctr:<28} {c:>10} {t / c:>16.1f}")
    return "\n".join(lines)


def cpu_baseline(np_side: int, nm: int, box: float, seed: int) -> dict:
    """The FP64 oracle on one COLA step of the same workload (ICs untimed)."""
    import numpy as np
    import torch
    from oracle import cola as ocola
    from oracle import cosmology as cosmo
    from oracle import lpt, philox

    cfg = cosmo.Config(np_side=np_side, nm_side=nm, box=box)
    w = philox.white_noise(seed, np_side**3)
    table = cosmo.step_table(cfg)
    s1, s2 = lpt.lpt_from_noise(w, cfg)
    st = ocola.initial_state(s1, s2, table)
    # COLA steps from the start of the run until about 10 s of CPU time have passed
    steps = 0
    t0 = time.perf_counter()
    while steps < cfg.n_steps and (steps == 0 or time.perf_counter() - t0 < 10.0):
        st = ocola.step(st, steps, table, cfg)
        steps += 1
    dt = time.perf_counter() - t0
    assert np.isfinite(st.s.sum().item())
    return {
        "value": steps * np_side**3 / dt, "unit": "particle-steps/s", "cores": torch.get_num_threads(),
        "threads": torch.get_num_threads(), "affinity_cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": f"the first {steps} COLA steps (PM force, kick, drift) of the {np_side}^3/{nm}^3 workload "
                  f"in FP64 torch-CPU, after oracle 2LPT ICs from the same Philox seed (ICs untimed); "
                  f"{dt:.1f} s",
    }


ENSEMBLE = [(64, 128, 16), (96, 192, 16), (128, 256, 16)]   # (np, nm, members), 100 Mpc/h


def timed(fn, stream, reps=1):
    """Milliseconds of fn() per repetition, HIP events on the launch stream."""
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def copy_bandwidth(stream, nbytes: int = 1 << 30) -> dict:
    """Measured device-to-device copy rate (read + write bytes per second) of a 1 GiB
    buffer, the practical streaming ceiling beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ms = timed(lambda: dst.copy_(src), stream, reps=5)
    del src, dst
    return {"bytes_moved": 2 * nbytes, "ms": ms, "gb_per_s": 2 * nbytes / (ms * 1e-3) / 1e9,
            "frac_of_peak": 2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_ensemble(stream) -> dict:
    """48 uneven-size realizations: one graph launch against the same runs issued
    one after another."""
    import torch
    import paper_1301_0322_amd as cola
    plans, noises = [], []
    seed = 1
    for np_side, nm, count in ENSEMBLE:
        for _ in range(count):
            pl = cola.Plan(cola.Config(np=np_side, nm=nm))
            w = torch.empty(np_side**3, dtype=torch.float32, device="cuda")
            pl.noise(seed, w)
            plans.append(pl)
            noises.append(w)
            seed += 1
    # tune each size once, share the choice
    tuned = {}
    for pl in plans:
        key = (pl.cfg.np, pl.cfg.nm)
        if key not in tuned:
            p = cola.Particles.empty(pl.cfg.np)
            pl.init_2lpt(noises[plans.index(pl)], p, pl.workspace())
            pl.autotune(p, None)
            tuned[key] = pl.get_tuning()
        y, x, tz = tuned[key]
        pl.set_fft_tile(0, y)
        pl.set_fft_tile(1, x)
        pl.set_bin_depth(tz)
    ens = cola.Ensemble(plans, noises)
    ens.launch()
    torch.cuda.synchronize()
    t_graph = timed(ens.launch, stream, reps=2)

    def sequential():
        for k, pl in enumerate(plans):
            pl.run(noises[k], ens.particles[k], ens.x[k], ens.v[k], ens.ws[k])
    sequential()
    torch.cuda.synchronize()
    t_seq = timed(sequential, stream, reps=2)
    work = sum(pl.cfg.np**3 * pl.cfg.n_steps for pl in plans)
    ens.close()
    return {"members": len(plans), "sizes": [list(e) for e in ENSEMBLE], "graph_ms": t_graph,
            "sequential_ms": t_seq, "graph_particle_steps_per_s": work / (t_graph * 1e-3),
            "sequential_particle_steps_per_s": work / (t_seq * 1e-3), "speedup": t_seq / t_graph}


def bench_paper_mesh(steps: int, config: str = "c1_paper_mesh") -> dict:
    """The in-run PM step of another configuration: the paper's 3x mesh (256^3
    particles on 768^3 cells) or the large box (512^3 on 1024^3, 400 Mpc/h)."""
    import torch

    import paper_1301_0322_amd as cola

    np_side, nm, box, seed, desc = CONFIGS[config]
    cfg = cola.Config(np=np_side, nm=nm, box=box)
    with cola.Plan(cfg) as plan:
        ws = plan.workspace()
        p = cola.Particles.empty(np_side)
        w = torch.empty(np_side**3, dtype=torch.float32, device="cuda")
        plan.noise(seed, w)
        x = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
        v = torch.empty_like(x)
        plan.run(w, p, x, v, ws)
        torch.cuda.synchronize()
        plan.trace_enable(2)
        for _ in range(steps):
            plan.run(w, p, x, v, ws)
        rec = plan.trace_read()["run_step"]
        plan.trace_enable(0)
        if not bool(torch.isfinite(x).all()):
            raise RuntimeError("non-finite positions at the 3x mesh")
    ms = rec[0] / rec[1]
    b_alg = b_alg_step(np_side, nm)
    return {"workload": desc, "pm_step_ms": ms, "particle_steps_per_s": np_side**3 / (ms * 1e-3),
            "b_alg_bytes": b_alg, "hbm_frac": b_alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "timed": f"each COLA step inside cola_run, HIP events around the step only, mean of {rec[1]} steps"}


def bench_adjoint(stream) -> dict:
    """128^3 / 256^3 differentiable run: forward with checkpoints + density against
    the hand-written adjoint; loss = sum (delta - delta_target)^2."""
    import torch
    import paper_1301_0322_amd as cola
    np_side, nm = 128, 256
    plan = cola.Plan(cola.Config(np=np_side, nm=nm))
    w = torch.empty(np_side**3, dtype=torch.float32, device="cuda")
    wt = torch.empty_like(w)
    plan.noise(11, w)
    plan.noise(12, wt)
    rho_t = cola.cola_density(wt, plan).detach()
    wd = w.clone().requires_grad_(True)

    def fwd():
        return cola.cola_density(wd, plan)

    def fwd_bwd():
        rho = fwd()
        ((rho - rho_t) ** 2).sum().backward()
    fwd_bwd()
    torch.cuda.synchronize()
    t_f = timed(lambda: fwd(), stream, reps=2)
    t_fb = timed(fwd_bwd, stream, reps=2)
    return {"config": f"{np_side}^3 particles / {nm}^3 mesh, 10 steps, loss sum (delta - delta_target)^2",
            "forward_ms": t_f, "forward_backward_ms": t_fb, "adjoint_ms": t_fb - t_f,
            "adjoint_over_forward": (t_fb - t_f) / t_f, "fwd_bwd_over_fwd": t_fb / t_f}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="GPUs (this build runs on one; N > 1 exits with a message)")
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (one step = one whole cola_run)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed cola_runs before the timed ones")
    ap.add_argument("--config", default="c1", choices=sorted(CONFIGS),
                    help="workload of the headline line (default c1: 256^3 particles, 512^3 mesh)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the FP64 oracle on the host")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 48-member ensemble figures")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 128^3 / 256^3 forward + adjoint figures")
    ap.add_argument("--autotune", action="store_true",
                    help="time the FFT tile widths and bin depth on the IC state first and keep the fastest "
                         "(default: the plan's defaults, the configuration the committed profiles cover)")
    ap.add_argument("--no-autotune", action="store_true", help="the default; kept for older command lines")
    ap.add_argument("--no-paper-mesh", action="store_true", help="skip the 256^3 / 768^3 and 512^3 / 1024^3 PM steps")
    ap.add_argument("--no-analysis", action="store_true", help="skip timing cola_cross_power")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy 256 MiB device to device once (a known-size kernel for HBM byte counters)")
    ap.add_argument("--rocprof-trace", metavar="DIR", help="print the summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--rocprof-pmc", metavar="DIR", help="print the summary of a rocprofv3 --pmc run and exit")
    ap.add_argument("--rocprof-busy", metavar="DIR",
                    help="print the GPU-busy fraction of each launch window of a rocprofv3 kernel trace and exit")
    ap.add_argument("--busy-gap-us", type=float, default=2000.0,
                    help="with --rocprof-busy: idle gap (us) that separates launch windows")
    ap.add_argument("--rocprof-hbm", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print HBM bytes per dispatch from a FETCH_SIZE and a WRITE_SIZE run and exit")
    ap.add_argument("--stage", default="", help="with --rocprof-hbm: the key: value block of this stage")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the 48-member ensemble (graph launches, then the same runs one by one)")
    args = ap.parse_args()
    if args.rocprof_hbm:
        print(rocprof_hbm_summary(*args.rocprof_hbm, stage=args.stage))
        return 0
    if args.rocprof_busy:
        print(rocprof_busy_summary(args.rocprof_busy, gap_us=args.busy_gap_us))
        return 0
    if args.rocprof_trace:
        print(rocprof_trace_summary(args.rocprof_trace))
        return 0
    if args.rocprof_pmc:
        print(rocprof_pmc_summary(args.rocprof_pmc))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU form of this method is described, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1301_0322_amd as cola

    np_side, nm, box, seed, desc = CONFIGS[args.config]
    torch.cuda.set_device(0)
    if args.ensemble_only:
        print(json.dumps({"ensemble": bench_ensemble(torch.cuda.current_stream())}), flush=True)
        return 0
    cfg = cola.Config(np=np_side, nm=nm, box=box)
    plan = cola.Plan(cfg)
    ws = plan.workspace()
    p = cola.Particles.empty(np_side)
    w = torch.empty(np_side**3, dtype=torch.float32, device="cuda")
    plan.noise(seed, w)
    x = torch.empty((3, np_side**3), dtype=torch.float32, device="cuda")
    v = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    if args.autotune and not args.no_autotune:
        plan.init_2lpt(w, p, ws)
        plan.autotune(p, None)
        ws = plan.workspace()
    # widths of 0 mean the built-in default (the widest column tile whose LDS fits)
    tuning = {k: (v if v else "default") for k, v in zip(("y_width", "x_width", "bin_depth"), plan.get_tuning())}
    tuning["source"] = "autotuned" if args.autotune and not args.no_autotune else "plan defaults"

    for _ in range(args.warmup):
        plan.run(w, p, x, v, ws)
    torch.cuda.synchronize()

    # timed region: K whole runs, HIP events on the launch stream around every kernel
    plan.trace_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.run(w, p, x, v, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    run_ms = e0.elapsed_time(e1) / args.steps
    stages = plan.trace_read()
    plan.trace_enable(False)
    if not np.isfinite(x.sum().item()):
        raise RuntimeError("non-finite positions")

    # PM step time inside the run: events around each COLA step of cola_run only
    # (deposit through gather + kick + drift), mean over every step of K runs
    plan.trace_enable(2)
    for _ in range(args.steps):
        plan.run(w, p, x, v, ws)
    steps_rec = plan.trace_read()["run_step"]
    plan.trace_enable(0)
    pm_step_ms = steps_rec[0] / steps_rec[1]

    # the same step through the public cola_step call, median over steps 1..n-1: plain
    # (the caller's Lagrangian-order arrays binned and packed from scratch each call)
    # and with resident steps (each call continues from the sorted state the previous
    # one left in the workspace)
    def public_steps(resident):
        plan.set_resident_steps(resident)
        plan.init_2lpt(w, p, ws)
        step_ms = []
        for i in range(cfg.n_steps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            plan.step(i, p, ws)
            b.record(stream)
            b.synchronize()
            if i > 0:
                step_ms.append(a.elapsed_time(b))
        # where a public step's time goes: the same calls with every kernel traced
        plan.init_2lpt(w, p, ws)
        plan.trace_enable(1)
        for i in range(cfg.n_steps):
            plan.step(i, p, ws)
        stages_ = {k: round(v[0] / cfg.n_steps, 4) for k, v in plan.trace_read().items()}
        plan.trace_enable(0)
        plan.set_resident_steps(0)
        return float(np.median(step_ms)), stages_

    api_step_ms, api_stages = public_steps(0)
    res_step_ms, res_stages = public_steps(1)

    sb = stage_bytes(np_side, nm)
    per_run = {k: {"ms": ms / args.steps, "launches": n // args.steps, "ms_per_launch": ms / n}
               for k, (ms, n) in stages.items()}
    dom = max(stages, key=lambda k: stages[k][0])
    dom_ms_launch = stages[dom][0] / stages[dom][1]
    dom_bytes = sb.get(dom, 0)
    achieved = dom_bytes / (dom_ms_launch * 1e-3) / 1e9
    workload = f"{args.config}"
    traffic = read_traffic(dom, workload)
    profile = read_profile_avg(dom, workload, plan.get_tuning()[2])
    b_alg = b_alg_step(np_side, nm)

    out = {
        "metric": f"particle-steps/s, {np_side}^3 COLA PM step (value: whole cola_run per bench step = 2LPT ICs "
                  f"+ {cfg.n_steps} PM steps + closing kick; the PM step alone under pm_step), % HBM roofline; "
                  f"adjoint/forward time",
        "value": np_side**3 * cfg.n_steps / (run_ms * 1e-3),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cola_run: 2LPT ICs + {cfg.n_steps} COLA steps z=9->0 + final kick, {desc}, "
                               f"Philox white noise seed {seed}, BBKS LCDM",
                   "np": np_side, "nm": nm, "box_mpc_h": box, "n_steps": cfg.n_steps},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom_bytes, "ms_per_launch": dom_ms_launch,
                     "rocprofv3": profile},
        "pm_step": {"ms": pm_step_ms, "particle_steps_per_s": np_side**3 / (pm_step_ms * 1e-3),
                    "b_alg_bytes": b_alg, "hbm_frac": b_alg / (pm_step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                    "b_alg_three_chains_bytes": b_alg_three_chains(np_side, nm),
                    "hbm_frac_three_chains": b_alg_three_chains(np_side, nm) / (pm_step_ms * 1e-3)
                    / (HBM_PEAK_GBS * 1e9),
                    "timed": f"each COLA step inside cola_run, HIP events around the step only, "
                             f"mean of {steps_rec[1]} steps",
                    "cola_step_call": {
                        "ms": api_step_ms, "particle_steps_per_s": np_side**3 / (api_step_ms * 1e-3),
                        "hbm_frac": b_alg / (api_step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                        "hbm_frac_three_chains": b_alg_three_chains(np_side, nm) / (api_step_ms * 1e-3)
                        / (HBM_PEAK_GBS * 1e9),
                        "timed": "the public cola_step call on the caller's Lagrangian-order arrays (bins from "
                                 "scratch each call), HIP events around each call, median over steps 1.."
                                 f"{cfg.n_steps - 1} after cola_init_2lpt",
                        "stages_ms_per_call": api_stages},
                    "cola_step_call_resident": {
                        "ms": res_step_ms, "particle_steps_per_s": np_side**3 / (res_step_ms * 1e-3),
                        "hbm_frac": b_alg / (res_step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                        "timed": "the public cola_step call with resident steps on (each call continues from the "
                                 "tile-sorted state the previous call left in the workspace and writes s, v to the "
                                 "caller's arrays), HIP events around each call, median over steps 1.."
                                 f"{cfg.n_steps - 1} after cola_init_2lpt",
                        "stages_ms_per_call": res_stages}},
        "stages_per_run": per_run,
        "tuning": tuning,
    }
    # density statistics of Section 3.1 on the final state: the run against itself
    # through cola_cross_power (two deposits, two forward FFTs, shell sums)
    out_stats = torch.zeros((6, nm // 2), dtype=torch.float64, device="cuda")
    if not args.no_analysis:
        plan.cross_power(p.s, p.s, out_stats, ws)
        torch.cuda.synchronize()
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        for _ in range(args.steps):
            plan.cross_power(p.s, p.s, out_stats, ws)
        eb.record(stream)
        torch.cuda.synchronize()
        out["analysis"] = {"call": "cola_cross_power (P_aa, P_bb, P_ab, rho, n_max per shell)",
                           "ms": ea.elapsed_time(eb) / args.steps,
                           "rho_min_shells_1_to_nm/2-1": float(out_stats[4, 1:].min().item())}
    if not args.no_ensemble:
        del ws
        torch.cuda.empty_cache()
        out["ensemble"] = bench_ensemble(stream)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(stream)
        torch.cuda.empty_cache()
    if not args.no_paper_mesh and args.config == "c1":
        if "ensemble" not in out:
            del ws
        torch.cuda.empty_cache()
        out["paper_mesh"] = bench_paper_mesh(args.steps)
        torch.cuda.empty_cache()
        out["c2"] = bench_paper_mesh(args.steps, "c2")
        torch.cuda.empty_cache()
    out["copy_bandwidth"] = copy_bandwidth(stream)
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(np_side, nm, box, seed)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
