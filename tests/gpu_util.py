"""Helpers for the GPU parity tests: device transfer and error metrics."""
import sys

import numpy as np
import torch


def dev(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda")


def host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy()


def _as_f64(a) -> np.ndarray:
    """float64 view of real data; complex data as (real, imaginary) pairs, so both
    parts take part in every error norm."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.stack([a.real, a.imag]).astype(np.float64)
    return a.astype(np.float64)


def rel_l2(got, ref) -> float:
    got, ref = _as_f64(got), _as_f64(ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def max_rel_to_rms(got, ref) -> float:
    """max |got - ref| / rms(ref) (complex: over real and imaginary parts)."""
    got, ref = _as_f64(got), _as_f64(ref)
    return float(np.abs(got - ref).max() / max(np.sqrt((ref * ref).mean()), 1e-300))


def periodic_max_err(x_got, x_ref, box) -> float:
    d = np.asarray(x_got, dtype=np.float64) - np.asarray(x_ref, dtype=np.float64)
    d = d - box * np.round(d / box)
    return float(np.abs(d).max())


def announce(msg: str):
    """Print (and flush) what the next GPU step is, so a fault names its case."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()
