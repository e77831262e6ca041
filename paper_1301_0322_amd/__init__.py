"""Python binding of the MI355X COLA particle-mesh library (``include/cola.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libcola_mi355x.so``.  Device buffers are torch tensors on the current HIP device;
work is enqueued on ``torch.cuda.current_stream()``.  There is no CPU fallback:
if the library is missing every call raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcola_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cola.h")

COLA_OK = 0
COLA_FLAG_KDK_STD = 0x1
COLA_FLAG_NO_LPT_FRAME = 0x2
COLA_FLAG_LOG_A_STEPS = 0x4
COLA_FLAG_U1_DRIFT = 0x8

SUPPORTED_SIZES = (16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
STEP_TABLE_COLUMNS = ("a", "D1", "D2", "TD1", "TD2", "T2D1", "T2D2", "alpha", "beta",
                      "dD1", "dD2", "a_mid", "force")


class ColaConfig(ctypes.Structure):
    _fields_ = [
        ("np", ctypes.c_int32), ("nm", ctypes.c_int32), ("box", ctypes.c_double),
        ("omega_m", ctypes.c_double), ("omega_l", ctypes.c_double), ("h", ctypes.c_double),
        ("n_s", ctypes.c_double), ("sigma8", ctypes.c_double), ("a_init", ctypes.c_double),
        ("a_final", ctypes.c_double), ("n_steps", ctypes.c_int32), ("n_lpt", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


class ColaParticles(ctypes.Structure):
    _fields_ = [("s", ctypes.c_void_p), ("v", ctypes.c_void_p), ("s1", ctypes.c_void_p),
                ("s2", ctypes.c_void_p)]


_VP = ctypes.c_void_p
_PROTOS = {
    "cola_plan_create": (ctypes.c_int, [ctypes.POINTER(ColaConfig), ctypes.POINTER(_VP)]),
    "cola_plan_destroy": (ctypes.c_int, [_VP]),
    "cola_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "cola_step_table": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    "cola_noise": (ctypes.c_int, [_VP, ctypes.c_uint64, _VP, _VP]),
    "cola_init_2lpt": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ColaParticles), _VP, _VP]),
    "cola_density": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "cola_density_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "cola_cross_power": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "cola_pm_force": (ctypes.c_int, [_VP, _VP, ctypes.c_double, _VP, _VP, _VP]),
    "cola_step": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ColaParticles), _VP, _VP]),
    "cola_finish": (ctypes.c_int, [_VP, ctypes.POINTER(ColaParticles), _VP, _VP, _VP, _VP]),
    "cola_run": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ColaParticles), _VP, _VP, _VP, _VP]),
    "cola_run_checkpointed": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ColaParticles), _VP, _VP, _VP, _VP, _VP]),
    "cola_adjoint_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "cola_run_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "cola_fft_r2c": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    "cola_fft_c2r": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    "cola_plan_set_fft_tile": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "cola_plan_set_bin_depth": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "cola_plan_set_fft_rotation": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "cola_plan_set_resident_steps": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "cola_plan_get_fft_rotation": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "cola_plan_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "cola_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(ColaParticles), _VP, ctypes.c_size_t, _VP,
                                     ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "cola_tuning_workspace_bytes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "cola_ensemble_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                            ctypes.POINTER(ColaParticles), ctypes.POINTER(_VP),
                                            ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP)]),
    "cola_run_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                        ctypes.POINTER(ColaParticles), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                        ctypes.POINTER(_VP), _VP]),
    "cola_ensemble_launch": (ctypes.c_int, [_VP, _VP]),
    "cola_ensemble_destroy": (ctypes.c_int, [_VP]),
    "cola_trace_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "cola_trace_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_int32]),
    "cola_trace_stage_count": (ctypes.c_int32, []),
    "cola_trace_stage_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "cola_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cola_last_hip_error": (ctypes.c_int, []),
}

_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1301_0322_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback path")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class ColaError(RuntimeError):
    def __init__(self, name: str, status: int):
        msg = lib().cola_strerror(status).decode()
        if status == -4:
            msg += f" (hipError_t {lib().cola_last_hip_error()})"
        super().__init__(f"{name} failed with status {status}: {msg}")
        self.status = status


def _check(name: str, status: int):
    if status != COLA_OK:
        raise ColaError(name, status)


def _ptr(t) -> int:
    if t is None:
        return 0
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        return t.data_ptr()
    return int(t)


def _stream(stream=None) -> int:
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _need(t, nbytes: int, name: str, dtype_size: int = 4):
    """Checks a device buffer before its pointer crosses the C-ABI: a CUDA tensor,
    contiguous, of the element size the entry point reads, at least nbytes long.
    The library cannot check sizes itself (it receives bare pointers).  None passes
    through as a null pointer, which every entry point rejects with an error status."""
    import torch
    if t is None:
        return t
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if t.element_size() != dtype_size:
        raise ValueError(f"{name}: expected {dtype_size}-byte elements, got {t.dtype}")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, needs at least {nbytes}")
    return t


@dataclass
class Config:
    """Mirror of ``cola_config`` with the defaults of the paper's run (Section 2)."""
    np: int = 32
    nm: int = 64
    box: float = 100.0
    omega_m: float = 0.3
    omega_l: float = 0.7
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    a_init: float = 0.1
    a_final: float = 1.0
    n_steps: int = 10
    n_lpt: float = -2.5
    flags: int = 0

    def to_c(self) -> ColaConfig:
        return ColaConfig(self.np, self.nm, self.box, self.omega_m, self.omega_l, self.h, self.n_s,
                          self.sigma8, self.a_init, self.a_final, self.n_steps, self.n_lpt, self.flags)


@dataclass
class Particles:
    """Device particle arrays, each a contiguous float32 tensor of shape (3, np^3)."""
    s: object
    v: object
    s1: object
    s2: object

    @staticmethod
    def empty(np_side: int, device="cuda"):
        import torch
        n = np_side**3
        mk = lambda: torch.empty((3, n), dtype=torch.float32, device=device)
        return Particles(mk(), mk(), mk(), mk())

    def to_c(self) -> ColaParticles:
        return ColaParticles(_ptr(self.s), _ptr(self.v), _ptr(self.s1), _ptr(self.s2))

    def checked(self, np_side: int) -> "Particles":
        for name in ("s", "v", "s1", "s2"):
            _need(getattr(self, name), 12 * np_side**3, f"particles.{name}")
        return self


class Plan:
    """Owns a ``cola_plan``; methods are the C entry points of the same names."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self._c = _VP()
        _check("cola_plan_create", lib().cola_plan_create(ctypes.byref(cfg.to_c()), ctypes.byref(self._c)))

    def close(self):
        if self._c:
            lib().cola_plan_destroy(self._c)
            self._c = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- host-only -------------------------------------------------------------------
    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check("cola_workspace_bytes", lib().cola_workspace_bytes(self._c, ctypes.byref(b)))
        return b.value

    def step_table(self):
        """Per-step FP64 scalars as a dict of lists (columns of cola_step_table)."""
        n = self.cfg.n_steps + 1
        buf = (ctypes.c_double * (13 * n))()
        _check("cola_step_table", lib().cola_step_table(self._c, buf, 13 * n))
        vals = list(buf)
        return {c: [vals[13 * i + j] for i in range(n)] for j, c in enumerate(STEP_TABLE_COLUMNS)}

    # -- device ----------------------------------------------------------------------
    def _p3(self, bytes_per_particle: int) -> int:
        return bytes_per_particle * self.cfg.np**3

    def _ws(self, ws):
        return _need(ws, self.workspace_bytes(), "ws")

    def _fft_buffers(self, n: int, inp, out):
        # n^3 floats in, n * n * (n/2) complex (also n^3 floats) out; sizes other than
        # np and nm are left to the library, which rejects them
        if n in (self.cfg.np, self.cfg.nm):
            _need(inp, 4 * n**3, "in")
            _need(out, 4 * n**3, "out")

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes() // 4, dtype=torch.float32, device=device)

    def noise(self, seed: int, w, stream=None):
        _need(w, self._p3(4), "w")
        _check("cola_noise", lib().cola_noise(self._c, seed, _ptr(w), _stream(stream)))

    def init_2lpt(self, w, p: Particles, ws, stream=None):
        _need(w, self._p3(4), "w")
        self._ws(ws)
        cp = p.checked(self.cfg.np).to_c()
        _check("cola_init_2lpt", lib().cola_init_2lpt(self._c, _ptr(w), ctypes.byref(cp), _ptr(ws),
                                                      _stream(stream)))

    def density(self, s, rho, ws, stream=None):
        _need(s, self._p3(12), "s")
        _need(rho, 4 * self.cfg.nm**3, "rho")
        self._ws(ws)
        _check("cola_density", lib().cola_density(self._c, _ptr(s), _ptr(rho), _ptr(ws), _stream(stream)))

    def density_noalloc(self, s, rho, stream=None):
        """cola_density without a workspace: the binning buffers live in the library's
        static per-GPU scratch (256 MiB); raises ColaError (status -6) beyond it.  Calls
        that overlap in time on one GPU race."""
        _need(s, self._p3(12), "s")
        _need(rho, 4 * self.cfg.nm**3, "rho")
        _check("cola_density_noalloc", lib().cola_density_noalloc(self._c, _ptr(s), _ptr(rho), _stream(stream)))

    def cross_power(self, s_a, s_b, out, ws, stream=None):
        """cola_cross_power: out (float64, 6 x nm/2 on the device) receives the mode
        count, P_aa, P_bb, P_ab, rho and n_max per shell; s_b may be None."""
        _need(s_a, self._p3(12), "s_a")
        if s_b is not None:
            _need(s_b, self._p3(12), "s_b")
        _need(out, 8 * 6 * (self.cfg.nm // 2), "out", dtype_size=8)
        self._ws(ws)
        _check("cola_cross_power", lib().cola_cross_power(self._c, _ptr(s_a), _ptr(s_b),
                                                          _ptr(out), _ptr(ws), _stream(stream)))

    def pm_force(self, s, a: float, acc, ws, stream=None):
        _need(s, self._p3(12), "s")
        _need(acc, self._p3(12), "acc")
        self._ws(ws)
        _check("cola_pm_force", lib().cola_pm_force(self._c, _ptr(s), a, _ptr(acc), _ptr(ws),
                                                    _stream(stream)))

    def step(self, i: int, p: Particles, ws, stream=None):
        self._ws(ws)
        cp = p.checked(self.cfg.np).to_c()
        _check("cola_step", lib().cola_step(self._c, i, ctypes.byref(cp), _ptr(ws), _stream(stream)))

    def finish(self, p: Particles, x_out, v_out, ws, stream=None):
        _need(x_out, self._p3(12), "x_out")
        _need(v_out, self._p3(12), "v_out")
        self._ws(ws)
        cp = p.checked(self.cfg.np).to_c()
        _check("cola_finish", lib().cola_finish(self._c, ctypes.byref(cp), _ptr(x_out), _ptr(v_out),
                                                _ptr(ws), _stream(stream)))

    def run(self, w, p: Particles, x_out, v_out, ws, stream=None):
        _need(w, self._p3(4), "w")
        _need(x_out, self._p3(12), "x_out")
        _need(v_out, self._p3(12), "v_out")
        self._ws(ws)
        cp = p.checked(self.cfg.np).to_c()
        _check("cola_run", lib().cola_run(self._c, _ptr(w), ctypes.byref(cp), _ptr(x_out), _ptr(v_out),
                                          _ptr(ws), _stream(stream)))

    def set_fft_tile(self, pass_: int, width: int):
        _check("cola_plan_set_fft_tile", lib().cola_plan_set_fft_tile(self._c, pass_, width))

    def set_bin_depth(self, depth: int):
        _check("cola_plan_set_bin_depth", lib().cola_plan_set_bin_depth(self._c, depth))

    def set_resident_steps(self, on: int):
        """Resident steps: consecutive step() calls on the same particles and workspace keep
        the tile-sorted state in the workspace (the arrays must not be changed between
        them).  0 off (default), 1 on."""
        _check("cola_plan_set_resident_steps", lib().cola_plan_set_resident_steps(self._c, on))

    def set_fft_rotation(self, on: int):
        """Rotated planes between the y and x passes of the mesh transforms: 1 on, 0 off,
        -1 the default."""
        _check("cola_plan_set_fft_rotation", lib().cola_plan_set_fft_rotation(self._c, on))

    def get_fft_rotation(self) -> int:
        """Rows per plane of the rotation in use (0: plain planes)."""
        r = ctypes.c_int32()
        _check("cola_plan_get_fft_rotation", lib().cola_plan_get_fft_rotation(self._c, ctypes.byref(r)))
        return r.value

    def get_tuning(self):
        y, x, tz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("cola_plan_get_tuning", lib().cola_plan_get_tuning(self._c, ctypes.byref(y), ctypes.byref(x),
                                                                  ctypes.byref(tz)))
        return y.value, x.value, tz.value

    def autotune(self, p: Particles, ws, cache_path=None, stream=None) -> bool:
        """Times the tile shapes on the PM force of p and keeps the fastest; True if
        the choice came from cache_path."""
        import torch
        need = ctypes.c_size_t()
        _check("cola_tuning_workspace_bytes", lib().cola_tuning_workspace_bytes(self._c, ctypes.byref(need)))
        if ws is None or ws.numel() * 4 < need.value:
            ws = torch.empty(need.value // 4 + 1, dtype=torch.float32, device=p.s.device)
        cp = p.checked(self.cfg.np).to_c()
        used = ctypes.c_int32()
        path = cache_path.encode() if cache_path else None
        _check("cola_autotune", lib().cola_autotune(self._c, ctypes.byref(cp), _ptr(ws), ws.numel() * 4,
                                                    _stream(stream), path, ctypes.byref(used)))
        return bool(used.value)

    def trace_enable(self, enable: int = 1):
        """1: events around every kernel; 2: around each cola_run step only; 0: off."""
        _check("cola_trace_enable", lib().cola_trace_enable(self._c, int(enable)))

    def trace_read(self):
        """{stage name: (milliseconds, launches)} since the last read (waits for the events)."""
        n = lib().cola_trace_stage_count()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        _check("cola_trace_read", lib().cola_trace_read(self._c, ms, cnt, n))
        return {lib().cola_trace_stage_name(k).decode(): (ms[k], cnt[k]) for k in range(n) if cnt[k]}

    def run_checkpointed(self, w, p: Particles, x_out, v_out, ckpt, ws, stream=None):
        _need(w, self._p3(4), "w")
        _need(x_out, self._p3(12), "x_out")
        _need(v_out, self._p3(12), "v_out")
        _need(ckpt, (self.cfg.n_steps + 1) * self._p3(12), "ckpt")
        self._ws(ws)
        cp = p.checked(self.cfg.np).to_c()
        _check("cola_run_checkpointed", lib().cola_run_checkpointed(
            self._c, _ptr(w), ctypes.byref(cp), _ptr(x_out), _ptr(v_out), _ptr(ckpt), _ptr(ws), _stream(stream)))

    def adjoint_workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check("cola_adjoint_workspace_bytes", lib().cola_adjoint_workspace_bytes(self._c, ctypes.byref(b)))
        return b.value

    def adjoint_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.adjoint_workspace_bytes() // 4, dtype=torch.float32, device=device)

    def run_adjoint(self, w, ckpt, dL_drho, dL_dw, ws, stream=None):
        _need(w, self._p3(4), "w")
        _need(ckpt, (self.cfg.n_steps + 1) * self._p3(12), "ckpt")
        _need(dL_drho, 4 * self.cfg.nm**3, "dL_drho")
        _need(dL_dw, self._p3(4), "dL_dw")
        _need(ws, self.adjoint_workspace_bytes(), "ws")
        _check("cola_run_adjoint", lib().cola_run_adjoint(self._c, _ptr(w), _ptr(ckpt), _ptr(dL_drho),
                                                          _ptr(dL_dw), _ptr(ws), _stream(stream)))

    def fft_r2c(self, n: int, inp, out, stream=None):
        self._fft_buffers(n, inp, out)
        _check("cola_fft_r2c", lib().cola_fft_r2c(self._c, n, _ptr(inp), _ptr(out), _stream(stream)))

    def fft_c2r(self, n: int, inp, out, stream=None):
        self._fft_buffers(n, inp, out)
        _check("cola_fft_c2r", lib().cola_fft_c2r(self._c, n, _ptr(inp), _ptr(out), _stream(stream)))


class Ensemble:
    """Whole runs of several plans captured once into one hipGraph (one branch per
    member) and replayed with ``launch()``.  Buffers are allocated here and kept
    alive with the graph: ``x[k]``, ``v[k]``, ``particles[k]``."""

    def __init__(self, plans, noises, device="cuda"):
        import torch
        self.plans = list(plans)
        noises = list(noises)
        if not self.plans or len(noises) != len(self.plans):
            raise ValueError(f"{len(self.plans)} plans and {len(noises)} noise arrays: need one per member")
        # the graph bakes in bare pointers, so every member's noise is checked before
        # anything is allocated or captured (a short buffer would be read past on
        # every replay)
        self._c = _VP()
        self.noises = []
        for k, (pl, w) in enumerate(zip(self.plans, noises)):
            if isinstance(w, torch.Tensor):
                w = w.contiguous()
            self.noises.append(_need(w, 4 * pl.cfg.np**3, f"noises[{k}]"))
        self.particles = [Particles.empty(pl.cfg.np, device) for pl in self.plans]
        self.ws = [pl.workspace(device) for pl in self.plans]
        self.x = [torch.empty((3, pl.cfg.np**3), dtype=torch.float32, device=device) for pl in self.plans]
        self.v = [torch.empty_like(x) for x in self.x]
        n = len(self.plans)
        arr = lambda vals: (_VP * n)(*vals)
        parts = (ColaParticles * n)(*[p.to_c() for p in self.particles])
        _check("cola_ensemble_create", lib().cola_ensemble_create(
            n, arr([pl._c for pl in self.plans]), arr([_ptr(w) for w in self.noises]), parts,
            arr([_ptr(x) for x in self.x]), arr([_ptr(v) for v in self.v]), arr([_ptr(w) for w in self.ws]),
            ctypes.byref(self._c)))

    def launch(self, stream=None):
        _check("cola_ensemble_launch", lib().cola_ensemble_launch(self._c, _stream(stream)))

    def close(self):
        if self._c:
            import torch
            torch.cuda.synchronize()
            lib().cola_ensemble_destroy(self._c)
            self._c = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batched(plans, noises, particles, xs, vs, workspaces, stream=None):
    """cola_run_batched: whole runs of several plans as one graph launch, waited for.
    Every buffer is the caller's and is checked against its plan's sizes first."""
    plans = list(plans)
    n = len(plans)
    lists = [list(noises), list(particles), list(xs), list(vs), list(workspaces)]
    if n == 0 or any(len(l) != n for l in lists):
        raise ValueError("run_batched needs one noise, particle set, x, v and workspace per plan")
    noises, particles, xs, vs, workspaces = lists
    for k, pl in enumerate(plans):
        _need(noises[k], 4 * pl.cfg.np**3, f"noises[{k}]")
        particles[k].checked(pl.cfg.np)
        _need(xs[k], 12 * pl.cfg.np**3, f"xs[{k}]")
        _need(vs[k], 12 * pl.cfg.np**3, f"vs[{k}]")
        _need(workspaces[k], pl.workspace_bytes(), f"workspaces[{k}]")
    arr = lambda vals: (_VP * n)(*vals)
    parts = (ColaParticles * n)(*[p.to_c() for p in particles])
    _check("cola_run_batched", lib().cola_run_batched(
        n, arr([pl._c for pl in plans]), arr([_ptr(w) for w in noises]), parts, arr([_ptr(x) for x in xs]),
        arr([_ptr(v) for v in vs]), arr([_ptr(w) for w in workspaces]), _stream(stream)))


def run(cfg: Config, w, device="cuda"):
    """Allocate, run the whole COLA evolution from white noise w; returns (x, v, particles)."""
    import torch
    plan = Plan(cfg)
    p = Particles.empty(cfg.np, device)
    ws = plan.workspace(device)
    x = torch.empty((3, cfg.np**3), dtype=torch.float32, device=device)
    v = torch.empty_like(x)
    plan.run(w, p, x, v, ws)
    return x, v, p


def _autograd_function():
    import torch

    class ColaDensity(torch.autograd.Function):
        """Final mean-1 CIC density (nm^3) of a whole COLA run as a function of the
        white noise w (np^3).  Forward: cola_run_checkpointed + cola_density;
        backward: cola_run_adjoint (the hand-written adjoint of the whole run)."""

        @staticmethod
        def forward(ctx, w, plan):
            cfg = plan.cfg
            n = cfg.np**3
            w = w.contiguous()
            p = Particles.empty(cfg.np, w.device)
            ws = plan.workspace(w.device)
            ckpt = torch.empty((cfg.n_steps + 1, 3, n), dtype=torch.float32, device=w.device)
            x = torch.empty((3, n), dtype=torch.float32, device=w.device)
            v = torch.empty_like(x)
            plan.run_checkpointed(w, p, x, v, ckpt, ws)
            rho = torch.empty(cfg.nm**3, dtype=torch.float32, device=w.device)
            plan.density(ckpt[cfg.n_steps], rho, ws)
            ctx.save_for_backward(w, ckpt)
            ctx.plan = plan
            return rho

        @staticmethod
        def backward(ctx, grad_rho):
            w, ckpt = ctx.saved_tensors
            plan = ctx.plan
            aws = plan.adjoint_workspace(w.device)
            dw = torch.empty_like(w)
            plan.run_adjoint(w, ckpt, grad_rho.contiguous().float(), dw, aws)
            return dw, None

    return ColaDensity


def cola_density(w, plan: Plan):
    """Differentiable final density: ColaDensity.apply(w, plan)."""
    global _COLA_DENSITY
    try:
        fn = _COLA_DENSITY
    except NameError:
        fn = _COLA_DENSITY = _autograd_function()
    return fn.apply(w, plan)
