"""MI355X-native batched RK4 integrator of Kerr geodesics (Python binding).

Thin ctypes binding over ``libmalbec.so`` (the C ABI in ``include/malbec.h``).
Each function marshals torch tensors (device memory, current HIP stream) into
the C call of the same name; every step of the computation runs in the HIP
kernels of the library.  There is no CPU fallback: importing this module on a
machine without the built library raises, and calling it without a GPU fails
in the HIP runtime.

Method: G. D. Quiroga, "MALBEC: a new CUDA-C ray-tracer in General
Relativity" (arXiv:1803.08320): Kerr metric in Boyer-Lindquist coordinates
(Section 2), classic RK4 (Section 5), per-lane horizon stop (Section 5).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch  # noqa: F401  (loads the HIP runtime before libmalbec)

__all__ = [
    "ICSpec", "Camera", "init_particles", "integrate", "invariants", "trace_camera",
    "workspace_bytes", "last_error", "version", "lib", "MalbecError", "STATUS", "adjoint",
    "IntegrateFromParams", "convert_state", "integrate_record", "integrate_adaptive",
    "adaptive_order", "Grid", "grid_kerr", "integrate_grid", "integrate_adaptive_noalloc",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmalbec.so")

STATUS = {"ACTIVE": 0, "HORIZON": 1, "ESCAPE": 2, "DISK": 3, "NONFINITE": 4, "BUDGET": 5}
F64, F32_KAHAN = 0, 1
FORM_CHRISTOFFEL, FORM_HAMILTONIAN = 0, 1
IC_CANONICAL, IC_CIRCULAR, IC_CONSTANTS, IC_PARAMS = 0, 1, 2, 3
OP_INTEGRATE, OP_CAMERA, OP_ADJOINT, OP_ADAPTIVE, OP_ADAPTIVE_ORDER = 1, 2, 3, 4, 5
OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP, ESAMPLE = 0, -1, -2, -3, -4, -5
SCHED_INDEX, SCHED_PERIAPSIS, SCHED_BUCKETS = 0, 1, 1024
NOALLOC_MAX_LANES = 1 << 21
GRID_F64, GRID_F32 = 0, 1
MAX_SPACETIMES = 64

# FP64 flops of one RK4 step of one lane (static counts by csrc/flopcount.cpp:
# add/sub/mul/div 1, fma 2, sincos 2).  Christoffel form: the work of a step is fixed
# by its direct evaluation (kerr_accel_direct in csrc/kerr_accel.hpp: coefficients, then
# the contraction), 514; the kernels evaluate the same acceleration regrouped, in 442
# (FLOPS_PER_STEP_F64_KERNEL).  Hamilton's equations: 336.
FLOPS_PER_STEP_F64 = 514
FLOPS_PER_STEP_F64_KERNEL = 442
FLOPS_PER_STEP_F64_HAM = 336
# FP32-compensated steps (FP32 flops): the stage increment plus d + lo and a two-sum per
# component (7 each); Christoffel form (direct evaluation, and as the kernel evaluates
# it) and Hamilton's equations
FLOPS_PER_STEP_F32K = 562
FLOPS_PER_STEP_F32K_KERNEL = 490
FLOPS_PER_STEP_F32K_HAM = 386
# one Dormand-Prince 5(4) attempt (six right-hand sides and the tableau; csrc/dp45.hpp),
# direct evaluation of the acceleration, and as the kernel evaluates it
FLOPS_PER_ATTEMPT_DP45 = 1024
FLOPS_PER_ATTEMPT_DP45_KERNEL = 916


class MalbecError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("malbec error %d: %s" % (code, msg))
        self.code = code


# ---- C structures (layout of include/malbec.h) ---------------------------------------
class c_spacetime(C.Structure):
    _fields_ = [("M", C.c_double), ("a", C.c_double)]


class c_batch(C.Structure):
    _fields_ = [("st", C.POINTER(c_spacetime)), ("n_st", C.c_int32), ("pad_", C.c_int32),
                ("st_of_lane", C.c_void_p)]


class c_ic_spec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("strict", C.c_int32), ("seed", C.c_uint64),
                ("lane0", C.c_int64), ("mu2", C.c_double), ("r_lo", C.c_double),
                ("r_hi", C.c_double), ("dL", C.c_double), ("prograde", C.c_int32),
                ("e_from_norm", C.c_int32), ("r_range", C.c_double * 2),
                ("th_range", C.c_double * 2), ("E_range", C.c_double * 2),
                ("Lz_range", C.c_double * 2), ("Q_range", C.c_double * 2),
                ("max_attempts", C.c_int64), ("rows", C.c_void_p)]


class c_run(C.Structure):
    _fields_ = [("h", C.c_double), ("n_steps", C.c_int64), ("precision", C.c_int32),
                ("block", C.c_int32), ("horizon_factor", C.c_double), ("r_escape", C.c_double),
                ("fp64_zone_factor", C.c_double), ("steps_per_chunk", C.c_int32),
                ("checkpoint_every", C.c_int32), ("persistent", C.c_int32),
                ("formulation", C.c_int32)]


class c_camera(C.Structure):
    _fields_ = [("M", C.c_double), ("a", C.c_double), ("r_obs", C.c_double),
                ("incl", C.c_double), ("half_width", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32), ("h0", C.c_double), ("h_r0", C.c_double),
                ("r_escape", C.c_double), ("horizon_factor", C.c_double),
                ("disk_r_in", C.c_double), ("disk_r_out", C.c_double), ("max_steps", C.c_int64),
                ("block", C.c_int32), ("steps_per_chunk", C.c_int32), ("persistent", C.c_int32),
                ("pad_", C.c_int32)]


class c_adaptive(C.Structure):
    _fields_ = [("tau_end", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("fac", C.c_double), ("facmin", C.c_double), ("facmax", C.c_double),
                ("max_attempts", C.c_int64), ("horizon_factor", C.c_double),
                ("r_escape", C.c_double), ("block", C.c_int32), ("persistent", C.c_int32),
                ("steps_per_chunk", C.c_int32), ("schedule", C.c_int32)]


class c_grid(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nth", C.c_int32), ("r0", C.c_double), ("dr", C.c_double),
                ("th0", C.c_double), ("dth", C.c_double), ("r_stop", C.c_double),
                ("nodes", C.c_void_p), ("node_precision", C.c_int32), ("pad_", C.c_int32)]


EXPORTS = {
    "malbec_last_error": (C.c_char_p, []),
    "malbec_version": (C.c_int, []),
    "malbec_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64, C.c_int32]),
    "malbec_init_particles": (C.c_int, [C.POINTER(c_ic_spec), C.POINTER(c_batch), C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "malbec_integrate": (C.c_int, [C.POINTER(c_run), C.POINTER(c_batch), C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "malbec_integrate_monitored": (C.c_int, [C.POINTER(c_run), C.POINTER(c_batch), C.c_int64,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                             C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                             C.c_void_p]),
    "malbec_trace_camera": (C.c_int, [C.POINTER(c_camera), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "malbec_invariants": (C.c_int, [C.POINTER(c_batch), C.c_int64, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "malbec_integrate_adaptive": (C.c_int, [C.POINTER(c_adaptive), C.POINTER(c_batch), C.c_int64,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                            C.c_void_p]),
    "malbec_integrate_adaptive_noalloc": (C.c_int, [C.POINTER(c_adaptive), C.POINTER(c_batch),
                                                    C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                                    C.c_void_p, C.c_void_p, C.c_void_p,
                                                    C.c_void_p]),
    "malbec_adaptive_order": (C.c_int, [C.POINTER(c_batch), C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_size_t, C.c_void_p]),
    "malbec_grid_fill_kerr": (C.c_int, [C.POINTER(c_grid), C.c_double, C.c_double, C.c_void_p,
                                        C.c_void_p]),
    "malbec_integrate_grid": (C.c_int, [C.POINTER(c_run), C.POINTER(c_grid), C.c_int64,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "malbec_integrate_record": (C.c_int, [C.POINTER(c_run), C.POINTER(c_batch), C.c_int64,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                          C.c_void_p, C.c_void_p]),
    "malbec_convert_state": (C.c_int, [C.POINTER(c_batch), C.c_int64, C.c_void_p, C.c_int32,
                                       C.c_void_p]),
    "malbec_adjoint": (C.c_int, [C.POINTER(c_run), C.POINTER(c_batch), C.c_int64, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
}

_lib = None


def lib():
    """Load libmalbec.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmalbec.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().malbec_last_error().decode()


def version() -> int:
    return lib().malbec_version()


def workspace_bytes(op: int, n: int, aux: int = 0) -> int:
    return lib().malbec_workspace_bytes(op, n, aux)


def _check(rc):
    if rc != 0:
        raise MalbecError(rc, last_error())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor], dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return C.c_void_p(t.data_ptr())


class _Batch:
    """Holds the ctypes batch descriptor and keeps its arrays alive."""

    def __init__(self, spacetimes, st_of_lane: Optional[torch.Tensor], n: int):
        sts = [tuple(map(float, s)) for s in spacetimes]
        if not 1 <= len(sts) <= MAX_SPACETIMES:
            raise ValueError("need 1..%d spacetimes" % MAX_SPACETIMES)
        self.arr = (c_spacetime * len(sts))(*[c_spacetime(M, a) for M, a in sts])
        self.c = c_batch(C.cast(self.arr, C.POINTER(c_spacetime)), len(sts), 0,
                         _ptr(st_of_lane, torch.int32, n, "st_of_lane"))


def _spacetimes(spacetimes):
    if isinstance(spacetimes, tuple) and len(spacetimes) == 2 and not hasattr(spacetimes[0], "__len__"):
        return [spacetimes]
    return list(spacetimes)


@dataclass
class ICSpec:
    """Initial-condition recipe, see malbec_ic_spec in include/malbec.h."""
    mode: int = IC_CONSTANTS
    seed: int = 0
    lane0: int = 0
    mu2: float = 1.0
    r_lo: float = 6.5
    r_hi: float = 20.0
    dL: float = 0.0
    prograde: bool = True
    e_from_norm: bool = True
    r_range: Tuple[float, float] = (5.0, 50.0)
    th_range: Tuple[float, float] = (0.7853981633974483, 2.356194490192345)
    E_range: Tuple[float, float] = (0.92, 0.98)
    Lz_range: Tuple[float, float] = (2.5, 4.5)
    Q_range: Tuple[float, float] = (0.0, 12.0)
    max_attempts: int = 100000
    rows: Optional[torch.Tensor] = field(default=None, repr=False)
    strict: bool = False  # CONSTANTS: raise (MALBEC_ESAMPLE) if a lane exhausts max_attempts

    def to_c(self, n):
        return c_ic_spec(self.mode, int(self.strict), self.seed & 0xFFFFFFFFFFFFFFFF, self.lane0, self.mu2,
                         self.r_lo, self.r_hi, self.dL, int(self.prograde), int(self.e_from_norm),
                         (C.c_double * 2)(*self.r_range), (C.c_double * 2)(*self.th_range),
                         (C.c_double * 2)(*self.E_range), (C.c_double * 2)(*self.Lz_range),
                         (C.c_double * 2)(*self.Q_range), self.max_attempts,
                         _ptr(self.rows, torch.float64,
                              None if self.rows is None else (6 if self.mode == IC_PARAMS else 8) * n,
                              "rows"))


def init_particles(spec: ICSpec, spacetimes, n: int, st_of_lane: Optional[torch.Tensor] = None,
                   device="cuda", want_consts=True, want_attempts=True):
    """Build n initial states on the device.  Returns (state[8, n], consts[4, n] or None,
    attempts[n] or None)."""
    dev = torch.device(device)
    state = torch.empty((8, n), dtype=torch.float64, device=dev)
    consts = torch.empty((4, n), dtype=torch.float64, device=dev) if want_consts else None
    attempts = torch.empty(n, dtype=torch.int64, device=dev) if want_attempts else None
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    cs = spec.to_c(n)
    _check(lib().malbec_init_particles(C.byref(cs), C.byref(b.c), n, _ptr(state),
                                       _ptr(consts), _ptr(attempts), _stream()))
    return state, consts, attempts


def integrate(state: torch.Tensor, status: torch.Tensor, steps: torch.Tensor, spacetimes,
              h: float, n_steps: int, horizon_factor: float = 1.01, r_escape: float = 1500.0,
              precision: str = "f64", fp64_zone_factor: float = 1.2, block: int = 0,
              steps_per_chunk: int = 0, st_of_lane: Optional[torch.Tensor] = None,
              checkpoints: Optional[torch.Tensor] = None, checkpoint_every: int = 0,
              persistent: bool = False, ws: Optional[torch.Tensor] = None,
              formulation: str = "christoffel"):
    """Advance state[8, n] in place (status, steps int32[n] in/out).  formulation
    "christoffel": state = (x^mu, u^mu); "hamiltonian": state = (x^mu, p_mu), see
    convert_state.  block = 0 (and, for a persistent launch, steps_per_chunk = 0) takes
    the autotuner's cached launch shape for this kind of batch when there is one
    (autotune.integrate_shape), else the library's defaults."""
    n = state.shape[-1]
    prec = {"f64": F64, "f32k": F32_KAHAN}[precision]
    form = {"christoffel": FORM_CHRISTOFFEL, "hamiltonian": FORM_HAMILTONIAN}[formulation]
    if block == 0 and checkpoint_every == 0 and state.is_cuda:
        from . import autotune
        shape = autotune.lookup_integrate(n, len(_spacetimes(spacetimes)), precision, formulation,
                                          persistent)
        if shape:
            block = shape[0]
            if persistent and steps_per_chunk == 0:
                steps_per_chunk = shape[1]
    run = c_run(h, n_steps, prec, block, horizon_factor, r_escape, fp64_zone_factor,
                steps_per_chunk, checkpoint_every, int(persistent), form)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    if checkpoint_every > 0:
        if checkpoints is None:
            raise ValueError("checkpoint_every > 0 needs a checkpoints tensor")
        slots = n_steps // checkpoint_every + 1
        if checkpoints.numel() < slots * 8 * n:
            raise ValueError("checkpoints must hold %d slots of 8 x %d doubles" % (slots, n))
    need = workspace_bytes(OP_INTEGRATE, n, int(persistent))
    if need and ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=state.device)
    _check(lib().malbec_integrate(C.byref(run), C.byref(b.c), n,
                                  _ptr(state, torch.float64, 8 * n, "state"),
                                  _ptr(status, torch.int32, n, "status"),
                                  _ptr(steps, torch.int32, n, "steps"),
                                  _ptr(checkpoints, torch.float64, None, "checkpoints"),
                                  _ptr(ws), ws.numel() if ws is not None else 0, _stream()))


def integrate_monitored(state: torch.Tensor, status: torch.Tensor, steps: torch.Tensor, spacetimes,
                        h: float, n_steps: int, monitor_every: int,
                        monitor: Optional[torch.Tensor] = None, reset: bool = True,
                        horizon_factor: float = 1.01, r_escape: float = 1500.0,
                        precision: str = "f64", fp64_zone_factor: float = 1.2, block: int = 0,
                        steps_per_chunk: int = 0, st_of_lane: Optional[torch.Tensor] = None,
                        persistent: bool = False, ws: Optional[torch.Tensor] = None,
                        formulation: str = "christoffel"):
    """integrate() with the invariant monitor every monitor_every steps of each lane's
    life.  monitor [8, n] float64: rows 0..3 the reference (E, L_z, Q, g(u,u)), rows
    4..7 the running maxima of |I - I_0| (written from the entry state when reset;
    carried over otherwise).  Returns monitor."""
    n = state.shape[-1]
    prec = {"f64": F64, "f32k": F32_KAHAN}[precision]
    form = {"christoffel": FORM_CHRISTOFFEL, "hamiltonian": FORM_HAMILTONIAN}[formulation]
    run = c_run(h, n_steps, prec, block, horizon_factor, r_escape, fp64_zone_factor,
                steps_per_chunk, 0, int(persistent), form)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    if monitor is None:
        if not reset:
            raise ValueError("reset=False needs the monitor tensor of the previous call")
        monitor = torch.full((8, n), float("nan"), dtype=torch.float64, device=state.device)
    need = workspace_bytes(OP_INTEGRATE, n, int(persistent))
    if need and ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=state.device)
    _check(lib().malbec_integrate_monitored(C.byref(run), C.byref(b.c), n,
                                            _ptr(state, torch.float64, 8 * n, "state"),
                                            _ptr(status, torch.int32, n, "status"),
                                            _ptr(steps, torch.int32, n, "steps"),
                                            int(monitor_every), int(bool(reset)),
                                            _ptr(monitor, torch.float64, 8 * n, "monitor"),
                                            _ptr(ws), ws.numel() if ws is not None else 0,
                                            _stream()))
    return monitor


def invariants(state: torch.Tensor, spacetimes, st_of_lane: Optional[torch.Tensor] = None,
               out: Optional[torch.Tensor] = None):
    """(E, L_z, Q, g(u,u)) of each lane as a [4, n] device tensor."""
    n = state.shape[-1]
    if out is None:
        out = torch.empty((4, n), dtype=torch.float64, device=state.device)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    _check(lib().malbec_invariants(C.byref(b.c), n, _ptr(state, torch.float64, 8 * n, "state"),
                                   _ptr(out, torch.float64, 4 * n, "out"), _stream()))
    return out


def integrate_adaptive(state: torch.Tensor, tau: torch.Tensor, h: torch.Tensor,
                       status: torch.Tensor, steps: torch.Tensor, rejects: torch.Tensor,
                       spacetimes, tau_end: float, rtol: float = 1e-10, atol: float = 1e-10,
                       fac: float = 0.9, facmin: float = 0.2, facmax: float = 5.0,
                       max_attempts: int = 1 << 20, horizon_factor: float = 1.01,
                       r_escape: float = 1500.0, block: int = 0, persistent: bool = True,
                       steps_per_chunk: int = 0, st_of_lane: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, schedule: Optional[str] = None):
    """Dormand-Prince 5(4) with per-lane step size up to tau_end; state[8, n], tau and h
    (float64[n]), status, steps and rejects (int32[n]) in/out.  schedule: "index" or
    "periapsis" (persistent only: lanes handed out smallest periapsis first; the results
    are the same); None = "periapsis" for a persistent launch, else "index"."""
    n = state.shape[-1]
    if schedule is None:
        schedule = "periapsis" if persistent else "index"
    sched = {"index": SCHED_INDEX, "periapsis": SCHED_PERIAPSIS}[schedule]
    ad = c_adaptive(tau_end, rtol, atol, fac, facmin, facmax, max_attempts, horizon_factor,
                    r_escape, block, int(persistent), steps_per_chunk, sched)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    need = workspace_bytes(OP_ADAPTIVE, n, 1 + sched if persistent else 0)
    if need and ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=state.device)
    _check(lib().malbec_integrate_adaptive(C.byref(ad), C.byref(b.c), n,
                                           _ptr(state, torch.float64, 8 * n, "state"),
                                           _ptr(tau, torch.float64, n, "tau"),
                                           _ptr(h, torch.float64, n, "h"),
                                           _ptr(status, torch.int32, n, "status"),
                                           _ptr(steps, torch.int32, n, "steps"),
                                           _ptr(rejects, torch.int32, n, "rejects"),
                                           _ptr(ws), ws.numel() if ws is not None else 0,
                                           _stream()))


def integrate_adaptive_noalloc(state: torch.Tensor, tau: torch.Tensor, h: torch.Tensor,
                               status: torch.Tensor, steps: torch.Tensor, rejects: torch.Tensor,
                               spacetimes, tau_end: float, rtol: float = 1e-10,
                               atol: float = 1e-10, fac: float = 0.9, facmin: float = 0.2,
                               facmax: float = 5.0, max_attempts: int = 1 << 20,
                               horizon_factor: float = 1.01, r_escape: float = 1500.0,
                               block: int = 0, persistent: bool = True, steps_per_chunk: int = 0,
                               st_of_lane: Optional[torch.Tensor] = None,
                               schedule: Optional[str] = None):
    """integrate_adaptive without a workspace: the library's static scratch serves the
    work queue and the work order (n <= NOALLOC_MAX_LANES; calls that overlap on one GPU
    race).  Allocates nothing."""
    n = state.shape[-1]
    if schedule is None:
        schedule = "periapsis" if persistent else "index"
    sched = {"index": SCHED_INDEX, "periapsis": SCHED_PERIAPSIS}[schedule]
    ad = c_adaptive(tau_end, rtol, atol, fac, facmin, facmax, max_attempts, horizon_factor,
                    r_escape, block, int(persistent), steps_per_chunk, sched)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    _check(lib().malbec_integrate_adaptive_noalloc(C.byref(ad), C.byref(b.c), n,
                                                   _ptr(state, torch.float64, 8 * n, "state"),
                                                   _ptr(tau, torch.float64, n, "tau"),
                                                   _ptr(h, torch.float64, n, "h"),
                                                   _ptr(status, torch.int32, n, "status"),
                                                   _ptr(steps, torch.int32, n, "steps"),
                                                   _ptr(rejects, torch.int32, n, "rejects"),
                                                   _stream()))


@dataclass
class Grid:
    """A 3+1 metric on a uniform (r, theta) grid (include/malbec.h, malbec_grid):
    nodes is a device tensor [nr, nth, 5] of (alpha, beta^phi, gamma_rr, gamma_thth,
    gamma_phph / sin^2 theta), float64 or float32 (MALBEC_GRID_F32: half the gathered
    bytes; the arithmetic stays FP64)."""
    nodes: torch.Tensor
    r0: float
    dr: float
    th0: float
    dth: float
    r_stop: float

    def to_c(self):
        nr, nth, k = self.nodes.shape
        if k != 5:
            raise ValueError("nodes must have shape [nr, nth, 5]")
        prec = {torch.float64: GRID_F64, torch.float32: GRID_F32}.get(self.nodes.dtype)
        if prec is None:
            raise ValueError("nodes must be float64 or float32")
        _ptr(self.nodes, self.nodes.dtype, nr * nth * 5, "nodes")
        return c_grid(nr, nth, self.r0, self.dr, self.th0, self.dth, self.r_stop,
                      self.nodes.data_ptr(), prec, 0)



def adaptive_order(state: torch.Tensor, tau: torch.Tensor, status: torch.Tensor, spacetimes,
                   tau_end: float, st_of_lane: Optional[torch.Tensor] = None):
    """The persistent adaptive kernel's periapsis work order: returns (order, keys), both
    int32[n] on the device holding uint32 values (see malbec_adaptive_order)."""
    n = state.shape[-1]
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    order = torch.empty(n, dtype=torch.int32, device=state.device)
    keys = torch.empty(n, dtype=torch.int32, device=state.device)
    need = workspace_bytes(OP_ADAPTIVE_ORDER, n, 0)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=state.device)
    _check(lib().malbec_adaptive_order(C.byref(b.c), n,
                                       _ptr(state, torch.float64, 8 * n, "state"),
                                       _ptr(tau, torch.float64, n, "tau"),
                                       _ptr(status, torch.int32, n, "status"), tau_end,
                                       _ptr(order), _ptr(keys), _ptr(ws), need, _stream()))
    return order, keys


def grid_kerr(M: float, a: float, nr: int, nth: int, r0: float, dr: float, th0: float, dth: float,
              r_stop: float, node_dtype=torch.float64) -> Grid:
    """A grid filled on the device with Kerr's 3+1 functions (Section 2), node values
    stored as node_dtype (float64 or float32)."""
    g = Grid(torch.empty((nr, nth, 5), dtype=node_dtype, device="cuda"), r0, dr, th0, dth,
             r_stop)
    cg = g.to_c()
    _check(lib().malbec_grid_fill_kerr(C.byref(cg), M, a, C.c_void_p(g.nodes.data_ptr()),
                                       _stream()))
    return g


def integrate_grid(state: torch.Tensor, status: torch.Tensor, steps: torch.Tensor, grid: Grid,
                   h: float, n_steps: int, r_escape: float, block: int = 0,
                   steps_per_chunk: int = 0):
    """Canonical RK4 of state[8, n] = (x, p) in the gridded 3+1 metric (in place)."""
    n = state.shape[-1]
    run = c_run(h, n_steps, F64, block, 1.0, r_escape, 1.0, steps_per_chunk, 0, 0,
                FORM_HAMILTONIAN)
    cg = grid.to_c()
    _check(lib().malbec_integrate_grid(C.byref(run), C.byref(cg), n,
                                       _ptr(state, torch.float64, 8 * n, "state"),
                                       _ptr(status, torch.int32, n, "status"),
                                       _ptr(steps, torch.int32, n, "steps"), _stream()))


def integrate_record(state: torch.Tensor, status: torch.Tensor, steps: torch.Tensor, spacetimes,
                     h: float, n_steps: int, record_every: int, traj: Optional[torch.Tensor] = None,
                     horizon_factor: float = 1.01, r_escape: float = 1500.0, block: int = 0,
                     st_of_lane: Optional[torch.Tensor] = None, formulation: str = "christoffel"):
    """integrate() that also records (tau, t, x, y, z) every record_every steps into
    traj[n_steps // record_every, 5, n] (allocated if None); returns traj."""
    n = state.shape[-1]
    if record_every < 1 or n_steps % record_every:
        raise ValueError("n_steps must be a positive multiple of record_every")
    n_rec = n_steps // record_every
    if traj is None:
        traj = torch.empty((n_rec, 5, n), dtype=torch.float64, device=state.device)
    form = {"christoffel": FORM_CHRISTOFFEL, "hamiltonian": FORM_HAMILTONIAN}[formulation]
    run = c_run(h, n_steps, F64, block, horizon_factor, r_escape, 1.0, 0, 0, 0, form)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    _check(lib().malbec_integrate_record(C.byref(run), C.byref(b.c), n,
                                         _ptr(state, torch.float64, 8 * n, "state"),
                                         _ptr(status, torch.int32, n, "status"),
                                         _ptr(steps, torch.int32, n, "steps"), record_every,
                                         _ptr(traj, torch.float64, n_rec * 5 * n, "traj"),
                                         _stream()))
    return traj


def convert_state(state: torch.Tensor, spacetimes, to_momenta: bool,
                  st_of_lane: Optional[torch.Tensor] = None):
    """In place: (x, u^mu) -> (x, p_mu) if to_momenta, else (x, p_mu) -> (x, u^mu)."""
    n = state.shape[-1]
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    _check(lib().malbec_convert_state(C.byref(b.c), n, _ptr(state, torch.float64, 8 * n, "state"),
                                      int(bool(to_momenta)), _stream()))
    return state


@dataclass
class Camera:
    """Camera of malbec_trace_camera (include/malbec.h)."""
    M: float = 1.0
    a: float = 0.998
    r_obs: float = 1000.0
    incl: float = 1.0471975511965976
    half_width: float = 25.0
    nx: int = 2048
    ny: int = 2048
    h0: float = 0.1
    h_r0: float = 10.0
    r_escape: float = 1500.0
    horizon_factor: float = 1.01
    disk_r_in: float = -1.0
    disk_r_out: float = 30.0
    max_steps: int = 100000
    block: int = 0
    steps_per_chunk: int = 0
    persistent: int = 1

    def to_c(self):
        return c_camera(self.M, self.a, self.r_obs, self.incl, self.half_width, self.nx, self.ny,
                        self.h0, self.h_r0, self.r_escape, self.horizon_factor, self.disk_r_in,
                        self.disk_r_out, self.max_steps, self.block, self.steps_per_chunk,
                        self.persistent, 0)


def trace_camera(cam: Camera, final_state: bool = False, device="cuda", out=None, ws=None):
    """Trace every pixel; returns dict(status[n], steps[n], hit[2, n], final_state[8, n]?).
    A persistent camera with block = 0 and steps_per_chunk = 0 takes the autotuner's
    cached shape when there is one (autotune.camera_shape)."""
    npix = cam.nx * cam.ny
    if cam.persistent and cam.block == 0 and cam.steps_per_chunk == 0 and \
            torch.device(device).type == "cuda":
        from . import autotune
        shape = autotune.lookup_camera(cam)
        if shape:
            cam = Camera(**{**cam.__dict__, "block": shape[0], "steps_per_chunk": shape[1]})
    dev = torch.device(device)
    if out is None:
        out = {"status": torch.empty(npix, dtype=torch.int32, device=dev),
               "steps": torch.empty(npix, dtype=torch.int32, device=dev),
               "hit": torch.empty((2, npix), dtype=torch.float64, device=dev)}
        if final_state:
            out["final_state"] = torch.empty((8, npix), dtype=torch.float64, device=dev)
    need = workspace_bytes(OP_CAMERA, npix, 0)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    cc = cam.to_c()
    _check(lib().malbec_trace_camera(C.byref(cc), _ptr(out["status"], torch.int32, npix),
                                     _ptr(out["steps"], torch.int32, npix),
                                     _ptr(out["hit"], torch.float64, 2 * npix),
                                     _ptr(out.get("final_state"), torch.float64, None),
                                     _ptr(ws), ws.numel(), _stream()))
    return out


def adjoint(checkpoints: torch.Tensor, status: torch.Tensor, steps: torch.Tensor,
            g_final: torch.Tensor, spacetimes, h: float, n_steps: int, checkpoint_every: int,
            horizon_factor: float = 1.01, r_escape: float = 1500.0,
            E_fixed: Optional[torch.Tensor] = None, named: bool = True, block: int = 0,
            st_of_lane: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Discrete adjoint of a checkpointed FP64 integrate call.  Returns (g_initial[8, n],
    g_named[5, n] or None)."""
    n = g_final.shape[-1]
    K = checkpoint_every
    slots = n_steps // K + 1
    if checkpoints.numel() < slots * 8 * n:
        raise ValueError("checkpoints must hold %d slots of 8 x %d doubles" % (slots, n))
    run = c_run(h, n_steps, F64, block, horizon_factor, r_escape, 1.0, 0, K, 0, 0)
    b = _Batch(_spacetimes(spacetimes), st_of_lane, n)
    g_initial = torch.empty((8, n), dtype=torch.float64, device=g_final.device)
    g_named = torch.empty((5, n), dtype=torch.float64, device=g_final.device) if named else None
    need = workspace_bytes(OP_ADJOINT, n, K)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=g_final.device)
    _check(lib().malbec_adjoint(C.byref(run), C.byref(b.c), n, _ptr(checkpoints, torch.float64),
                                _ptr(status, torch.int32, n, "status"),
                                _ptr(steps, torch.int32, n, "steps"),
                                _ptr(g_final, torch.float64, 8 * n, "g_final"),
                                _ptr(g_initial), _ptr(E_fixed, torch.float64, n, "E_fixed"),
                                _ptr(g_named), _ptr(ws), ws.numel(), _stream()))
    return g_initial, g_named


class IntegrateFromParams(torch.autograd.Function):
    """y_N = RK4^N(y_0(p)), p = (r0, theta0, u^r0, u^theta0, L_z) [5, n] with E [n] held
    fixed; backward runs the discrete adjoint (malbec_adjoint) from the checkpoints
    saved by the forward pass.  Returns (y_N [8, n], status [n], steps [n])."""

    @staticmethod
    def forward(ctx, p, E, spacetime, h, n_steps, checkpoint_every, horizon_factor=1.01,
                r_escape=1500.0):
        n = p.shape[1]
        rows = torch.cat([p.t(), E.reshape(n, 1)], dim=1).contiguous()
        spec = ICSpec(mode=IC_PARAMS, rows=rows)
        state, _, _ = init_particles(spec, [spacetime], n, device=p.device, want_consts=False,
                                     want_attempts=False)
        status, steps = new_lane_arrays(n, device=p.device)
        K = checkpoint_every
        ck = torch.empty((n_steps // K + 1, 8, n), dtype=torch.float64, device=p.device)
        integrate(state, status, steps, [spacetime], h=h, n_steps=n_steps,
                  horizon_factor=horizon_factor, r_escape=r_escape, checkpoints=ck,
                  checkpoint_every=K)
        ctx.save_for_backward(ck, status, steps, E)
        ctx.cfg = (spacetime, h, n_steps, K, horizon_factor, r_escape)
        ctx.mark_non_differentiable(status, steps)
        return state, status, steps

    @staticmethod
    def backward(ctx, g_state, g_status, g_steps):
        ck, status, steps, E = ctx.saved_tensors
        spacetime, h, n_steps, K, hf, resc = ctx.cfg
        _, g_named = adjoint(ck, status, steps, g_state.contiguous(), [spacetime], h, n_steps, K,
                             horizon_factor=hf, r_escape=resc, E_fixed=E.contiguous())
        return g_named, None, None, None, None, None, None, None


def new_lane_arrays(n: int, device="cuda"):
    """Zeroed (status, steps) int32 arrays for n ACTIVE lanes."""
    return (torch.zeros(n, dtype=torch.int32, device=device),
            torch.zeros(n, dtype=torch.int32, device=device))
