"""Plain FP64 CPU oracle (test infrastructure).

This package checks the GPU product path; it shares no code with it.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product (``paper_1803_08320_amd``) never does.

The numerics live in ``malbec_oracle.c`` / ``oracle_core.inc`` (plain C, FP64,
``-ffp-contract=off``); this module builds the shared library with gcc and
wraps it with ctypes and numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "malbec_oracle.c"), os.path.join(_HERE, "oracle_core.inc")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

LANE_STATUS = {"ACTIVE": 0, "HORIZON": 1, "ESCAPE": 2, "DISK": 3, "NONFINITE": 4, "BUDGET": 5}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC[0], "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def lib():
    """Load (building first if absent) the oracle library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRC):
        build()
    L = C.CDLL(_LIB_PATH)
    d, i64, i32, u64, vp = C.c_double, C.c_int64, C.c_int32, C.c_uint64, C.c_void_p
    P = C.POINTER
    sig = {
        "oracle_metric": (None, [d, d, d, d, P(d)]),
        "oracle_metric_partials": (None, [d, d, d, d, P(d)]),
        "oracle_metric_partials_complex_step": (None, [d, d, d, d, P(d)]),
        "oracle_inverse_metric": (C.c_int, [d, d, d, d, P(d)]),
        "oracle_christoffel": (None, [d, d, d, d, P(d)]),
        "oracle_rhs": (None, [d, d, P(d), P(d)]),
        "oracle_rhs_hamiltonian": (None, [d, d, P(d), P(d)]),
        "oracle_r_horizon": (d, [d, d]),
        "oracle_r_isco": (d, [d, d, C.c_int]),
        "oracle_circular_EL": (None, [d, d, d, C.c_int, P(d), P(d)]),
        "oracle_circular_EL_paper": (None, [d, d, d, C.c_int, P(d), P(d)]),
        "oracle_schwarzschild_circular": (None, [d, d, P(d), P(d)]),
        "oracle_draw_u64": (u64, [u64, u64, u64, u64]),
        "oracle_invariants_one": (None, [d, d, P(d), P(d)]),
        "oracle_potential_R": (d, [d, d, d, d, d, d, d]),
        "oracle_potential_Theta": (d, [d, d, d, d, d, d]),
        "oracle_velocity_from_constants": (None, [d, d, d, d, d, d, d, d, d, d, P(d)]),
        "oracle_ic_canonical": (C.c_int, [d, d, i64, P(d), P(d)]),
        "oracle_ic_circular": (C.c_int, [u64, d, d, i64, i64, d, d, d, C.c_int, C.c_int, P(d)]),
        "oracle_ic_constants": (C.c_int, [u64, P(d), vp, i64, i64, P(d), d, i64, P(d), vp, vp]),
        "oracle_integrate": (C.c_int, [P(d), vp, i64, P(d), P(i32), P(i32), d, i64, d, d,
                                       C.c_int, C.c_int]),
        "oracle_invariants": (C.c_int, [P(d), vp, i64, P(d), P(d)]),
        "oracle_invariants_hamiltonian_one": (None, [d, d, P(d), P(d)]),
        "oracle_integrate_monitored": (C.c_int, [P(d), vp, i64, P(d), P(i32), P(i32), d, i64, d,
                                                 d, C.c_int, i64, C.c_int, P(d), C.c_int]),
        "oracle_dp45_attempt": (None, [d, d, d, P(d), P(d), P(d)]),
        "oracle_kerr_3p1": (None, [d, d, d, d, P(d)]),
        "oracle_grid_fill_kerr": (None, [d, d, i64, i64, d, d, d, d, P(d)]),
        "oracle_grid_eval": (None, [i64, i64, d, d, d, d, P(d), d, d, P(d), P(d), P(d)]),
        "oracle_grid_rhs": (None, [i64, i64, d, d, d, d, P(d), P(d), P(d)]),
        "oracle_integrate_grid": (C.c_int, [i64, i64, d, d, d, d, P(d), i64, P(d), P(i32), P(i32),
                                            d, i64, d, d, C.c_int]),
        "oracle_integrate_adaptive": (C.c_int, [P(d), vp, i64, P(d), P(d), P(d), P(i32), P(i32),
                                                P(i32), d, d, d, d, d, d, i64, d, d, C.c_int]),
        "oracle_camera_ic": (None, [d, d, d, d, d, i64, i64, i64, i64, P(d)]),
        "oracle_trace_camera": (C.c_int, [d, d, d, d, d, i64, i64, d, d, d, d, d, d, i64, i64,
                                          P(i64), P(i32), P(i32), P(d), vp, C.c_int]),
        "oracle_ray_ic": (None, [d, d, d, d, d, d, P(d)]),
        "oracle_trace_rays": (C.c_int, [d, d, d, d, i64, P(d), P(d), d, d, d, d, d, d, i64,
                                        P(i32), P(i32), P(d), vp, C.c_int]),
        "oracle_tangent": (None, [d, d, d, i64, P(d), P(d), vp, P(d)]),
        "oracle_ic_map": (None, [d, d, d, P(d), P(d)]),
        "oracle_grad_ic": (C.c_int, [d, d, d, i64, i64, P(d), P(d), P(d), P(d), vp, C.c_int]),
        "oracle_loss_ic": (d, [d, d, d, i64, P(d), d, P(d)]),
        "oracle_max_threads": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _f64(x, n=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# ----------------------------------------------------------------------------- pointwise
def metric(M, a, r, th):
    g = np.zeros(16)
    lib().oracle_metric(M, a, r, th, _dp(g))
    return g.reshape(4, 4)


def metric_partials(M, a, r, th):
    dg = np.zeros(64)
    lib().oracle_metric_partials(M, a, r, th, _dp(dg))
    return dg.reshape(4, 4, 4)


def metric_partials_complex_step(M, a, r, th):
    dg = np.zeros(64)
    lib().oracle_metric_partials_complex_step(M, a, r, th, _dp(dg))
    return dg.reshape(4, 4, 4)


def inverse_metric(M, a, r, th):
    gi = np.zeros(16)
    rc = lib().oracle_inverse_metric(M, a, r, th, _dp(gi))
    assert rc == 0
    return gi.reshape(4, 4)


def christoffel(M, a, r, th):
    G = np.zeros(64)
    lib().oracle_christoffel(M, a, r, th, _dp(G))
    return G.reshape(4, 4, 4)


def rhs(M, a, y):
    y = _f64(y, 8)
    f = np.zeros(8)
    lib().oracle_rhs(M, a, _dp(y), _dp(f))
    return f


def rhs_hamiltonian(M, a, z):
    z = _f64(z, 8)
    f = np.zeros(8)
    lib().oracle_rhs_hamiltonian(M, a, _dp(z), _dp(f))
    return f


def invariants_one(M, a, y):
    y = _f64(y, 8)
    out = np.zeros(4)
    lib().oracle_invariants_one(M, a, _dp(y), _dp(out))
    return out


def r_horizon(M, a):
    return lib().oracle_r_horizon(M, a)


def r_isco(M, a, prograde=True):
    return lib().oracle_r_isco(M, a, int(prograde))


def circular_EL(M, a, r, prograde=True, paper_form=False):
    E, L = C.c_double(), C.c_double()
    fn = lib().oracle_circular_EL_paper if paper_form else lib().oracle_circular_EL
    fn(M, a, r, int(prograde), C.byref(E), C.byref(L))
    return E.value, L.value


def schwarzschild_circular(M, r):
    E, L = C.c_double(), C.c_double()
    lib().oracle_schwarzschild_circular(M, r, C.byref(E), C.byref(L))
    return E.value, L.value


def draw_u64(seed, lane, attempt, k):
    return lib().oracle_draw_u64(seed, lane, attempt, k)


def potential_R(M, a, E, Lz, Q, mu2, r):
    return lib().oracle_potential_R(M, a, E, Lz, Q, mu2, r)


def potential_Theta(a, E, Lz, Q, mu2, th):
    return lib().oracle_potential_Theta(a, E, Lz, Q, mu2, th)


def velocity_from_constants(M, a, E, Lz, Q, mu2, r, th, sr=1.0, sth=1.0):
    u = np.zeros(4)
    lib().oracle_velocity_from_constants(M, a, E, Lz, Q, mu2, r, th, sr, sth, _dp(u))
    return u


# ----------------------------------------------------------------------------- batches
def _Ma(spacetimes):
    return _f64(np.asarray(spacetimes, dtype=np.float64).reshape(-1))


def _st_ptr(st_of_lane, n):
    if st_of_lane is None:
        return None, None
    arr = np.ascontiguousarray(st_of_lane, dtype=np.int32)
    assert arr.size == n
    return arr, arr.ctypes.data_as(C.c_void_p)


def ic_canonical(M, a, rows):
    rows = _f64(rows).reshape(-1, 8)
    n = rows.shape[0]
    state = np.zeros(8 * n)
    rc = lib().oracle_ic_canonical(M, a, n, _dp(np.ascontiguousarray(rows.reshape(-1))), _dp(state))
    assert rc == 0
    return state.reshape(8, n)


def ic_circular(seed, M, a, n, r_lo, r_hi, dL, prograde=True, e_from_norm=True, lane0=0):
    state = np.zeros(8 * n)
    lib().oracle_ic_circular(seed, M, a, n, lane0, r_lo, r_hi, dL, int(prograde), int(e_from_norm),
                             _dp(state))
    return state.reshape(8, n)


def ic_constants(seed, spacetimes, n, ranges, mu2=1.0, max_attempts=100000, st_of_lane=None,
                 lane0=0):
    """ranges = ((r_lo, r_hi), (th_lo, th_hi), (E_lo, E_hi), (Lz_lo, Lz_hi), (Q_lo, Q_hi))."""
    Ma = _Ma(spacetimes)
    rng = _f64(np.asarray(ranges, dtype=np.float64).reshape(-1), 10)
    state = np.zeros(8 * n)
    consts = np.zeros(4 * n)
    attempts = np.zeros(n, dtype=np.int64)
    _keep, stp = _st_ptr(st_of_lane, n)
    rc = lib().oracle_ic_constants(seed, _dp(Ma), stp, n, lane0, _dp(rng), mu2, max_attempts,
                                   _dp(state), consts.ctypes.data_as(C.c_void_p),
                                   attempts.ctypes.data_as(C.c_void_p))
    return rc, state.reshape(8, n), consts.reshape(4, n), attempts


def integrate(spacetimes, state, h, n_steps, status=None, steps=None, horizon_factor=1.01,
              r_escape=1500.0, hamiltonian=False, st_of_lane=None, nthreads=0):
    """Integrate a SoA batch (8, n) in place-copy; returns (state, status, steps)."""
    state = np.array(state, dtype=np.float64, copy=True)
    n = state.shape[1]
    s = np.ascontiguousarray(state.reshape(-1))
    status = np.zeros(n, np.int32) if status is None else np.array(status, np.int32, copy=True)
    steps = np.zeros(n, np.int32) if steps is None else np.array(steps, np.int32, copy=True)
    Ma = _Ma(spacetimes)
    _keep, stp = _st_ptr(st_of_lane, n)
    lib().oracle_integrate(_dp(Ma), stp, n, _dp(s), _ip(status), _ip(steps), h, n_steps,
                           horizon_factor, r_escape, int(hamiltonian), nthreads)
    return s.reshape(8, n), status, steps


def integrate_monitored(spacetimes, state, h, n_steps, every, monitor=None, status=None,
                        steps=None, horizon_factor=1.01, r_escape=1500.0, hamiltonian=False,
                        st_of_lane=None, nthreads=0):
    """Fixed-step RK4 with the invariant monitor every `every` steps of each lane's
    life (copies).  monitor=None resets (I0 from the entry state, maxima 0); otherwise
    the given [8, n] monitor continues.  Returns (state, status, steps, monitor)."""
    state = np.array(state, dtype=np.float64, copy=True)
    n = state.shape[1]
    s = np.ascontiguousarray(state.reshape(-1))
    status = np.zeros(n, np.int32) if status is None else np.array(status, np.int32, copy=True)
    steps = np.zeros(n, np.int32) if steps is None else np.array(steps, np.int32, copy=True)
    reset = monitor is None
    mon = np.full(8 * n, np.nan) if reset else np.array(monitor, np.float64, copy=True).reshape(-1)
    Ma = _Ma(spacetimes)
    _keep, stp = _st_ptr(st_of_lane, n)
    rc = lib().oracle_integrate_monitored(_dp(Ma), stp, n, _dp(s), _ip(status), _ip(steps), h,
                                          n_steps, horizon_factor, r_escape, int(hamiltonian),
                                          every, int(reset), _dp(mon), nthreads)
    if rc:
        raise ValueError("every must be >= 1")
    return s.reshape(8, n), status, steps, mon.reshape(8, n)


def invariants_hamiltonian_one(M, a, z):
    z = _f64(z, 8)
    out = np.zeros(4)
    lib().oracle_invariants_hamiltonian_one(M, a, _dp(z), _dp(out))
    return out


def dp45_attempt(M, a, h, y):
    """One Dormand-Prince attempt: (y1 of 5th order, y1 - y1* of the 4th-order pair)."""
    y = _f64(y)
    y1, e = np.zeros(8), np.zeros(8)
    lib().oracle_dp45_attempt(M, a, h, _dp(y), _dp(y1), _dp(e))
    return y1, e


class Grid:
    """A uniform (r, theta) grid of the 3+1 functions (alpha, beta^phi, gamma_rr,
    gamma_thth, gamma_phph / sin^2 theta), nodes[i, j, k]."""

    def __init__(self, nodes, r0, dr, th0, dth):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.nr, self.nth = self.nodes.shape[:2]
        self.r0, self.dr, self.th0, self.dth = float(r0), float(dr), float(th0), float(dth)

    def args(self):
        return (self.nr, self.nth, self.r0, self.dr, self.th0, self.dth, _dp(self.nodes.reshape(-1)))


def kerr_3p1(M, a, r, th):
    F = np.zeros(5)
    lib().oracle_kerr_3p1(M, a, r, th, _dp(F))
    return F


def grid_kerr(M, a, nr, nth, r0, dr, th0, dth):
    nodes = np.zeros(nr * nth * 5)
    lib().oracle_grid_fill_kerr(M, a, nr, nth, r0, dr, th0, dth, _dp(nodes))
    return Grid(nodes.reshape(nr, nth, 5), r0, dr, th0, dth)


def grid_eval(grid, r, th):
    F, Fr, Ft = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().oracle_grid_eval(*grid.args(), r, th, _dp(F), _dp(Fr), _dp(Ft))
    return F, Fr, Ft


def grid_rhs(grid, z):
    z = _f64(z)
    f = np.zeros(8)
    lib().oracle_grid_rhs(*grid.args(), _dp(z), _dp(f))
    return f


def integrate_grid(grid, state, h, n_steps, r_stop, r_escape, status=None, steps=None, nthreads=0):
    """Canonical RK4 on the gridded metric (copies); returns (state, status, steps)."""
    state = np.array(state, dtype=np.float64, copy=True)
    n = state.shape[1]
    s = np.ascontiguousarray(state.reshape(-1))
    status = np.zeros(n, np.int32) if status is None else np.array(status, np.int32, copy=True)
    steps = np.zeros(n, np.int32) if steps is None else np.array(steps, np.int32, copy=True)
    lib().oracle_integrate_grid(*grid.args(), n, _dp(s), _ip(status), _ip(steps), h, n_steps,
                                r_stop, r_escape, nthreads)
    return s.reshape(8, n), status, steps


def integrate_adaptive(spacetimes, state, tau_end, h0, rtol=1e-10, atol=1e-10, fac=0.9,
                       facmin=0.2, facmax=5.0, max_attempts=1 << 20, tau=None, h=None,
                       status=None, steps=None, rejects=None, horizon_factor=1.01,
                       r_escape=1500.0, st_of_lane=None, nthreads=0):
    """Dormand-Prince 5(4) with per-lane step-size control up to tau_end (copies);
    returns (state, tau, h, status, steps, rejects)."""
    state = np.array(state, dtype=np.float64, copy=True)
    n = state.shape[1]
    s = np.ascontiguousarray(state.reshape(-1))
    tau = np.zeros(n) if tau is None else np.array(tau, np.float64, copy=True)
    h = np.full(n, float(h0)) if h is None else np.array(h, np.float64, copy=True)
    status = np.zeros(n, np.int32) if status is None else np.array(status, np.int32, copy=True)
    steps = np.zeros(n, np.int32) if steps is None else np.array(steps, np.int32, copy=True)
    rejects = np.zeros(n, np.int32) if rejects is None else np.array(rejects, np.int32, copy=True)
    Ma = _Ma(spacetimes)
    _keep, stp = _st_ptr(st_of_lane, n)
    lib().oracle_integrate_adaptive(_dp(Ma), stp, n, _dp(s), _dp(tau), _dp(h), _ip(status),
                                    _ip(steps), _ip(rejects), tau_end, rtol, atol, fac, facmin,
                                    facmax, max_attempts, horizon_factor, r_escape, nthreads)
    return s.reshape(8, n), tau, h, status, steps, rejects


def invariants(spacetimes, state, st_of_lane=None):
    state = _f64(state)
    n = state.size // 8
    out = np.zeros(4 * n)
    Ma = _Ma(spacetimes)
    _keep, stp = _st_ptr(st_of_lane, n)
    lib().oracle_invariants(_dp(Ma), stp, n, _dp(state.reshape(-1)), _dp(out))
    return out.reshape(4, n)


def camera_ic(M, a, r_obs, incl, half_width, nx, ny, i, j):
    y = np.zeros(8)
    lib().oracle_camera_ic(M, a, r_obs, incl, half_width, nx, ny, i, j, _dp(y))
    return y


def trace_camera(cam, pix, nthreads=0, final_state=False):
    """cam: dict with M, a, r_obs, incl, half_width, nx, ny, h0, h_r0, r_escape,
    horizon_factor, disk_r_in (<= 0: prograde ISCO), disk_r_out, max_steps."""
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    npx = pix.size
    status = np.zeros(npx, np.int32)
    steps = np.zeros(npx, np.int32)
    hit = np.zeros(2 * npx)
    fs = np.zeros(8 * npx) if final_state else None
    r_in = cam["disk_r_in"]
    if r_in <= 0:
        r_in = r_isco(cam["M"], cam["a"], True)
    lib().oracle_trace_camera(cam["M"], cam["a"], cam["r_obs"], cam["incl"], cam["half_width"],
                              cam["nx"], cam["ny"], cam["h0"], cam["h_r0"], cam["r_escape"],
                              cam["horizon_factor"], r_in, cam["disk_r_out"], cam["max_steps"], npx,
                              _lp(pix), _ip(status), _ip(steps), _dp(hit),
                              None if fs is None else fs.ctypes.data_as(C.c_void_p), nthreads)
    out = {"status": status, "steps": steps, "hit": hit.reshape(npx, 2).T.copy()}
    if fs is not None:
        out["final_state"] = fs.reshape(8, npx)
    return out


def ray_ic(M, a, r_obs, incl, alpha, beta):
    y = np.zeros(8)
    lib().oracle_ray_ic(M, a, r_obs, incl, alpha, beta, _dp(y))
    return y


def trace_rays(M, a, r_obs, incl, alpha, beta, h0=0.1, h_r0=10.0, r_escape=1500.0,
               horizon_factor=1.01, disk_r_in=1.0, disk_r_out=-1.0, max_steps=100000, nthreads=0,
               final_state=False):
    """Trace rays at explicit image-plane points; disk_r_in > disk_r_out disables the disk.
    Returns (status, steps, hit[2, n]) and, with final_state=True, the state [8, n] too."""
    alpha = _f64(alpha)
    beta = _f64(beta, alpha.size)
    n = alpha.size
    status = np.zeros(n, np.int32)
    steps = np.zeros(n, np.int32)
    hit = np.zeros(2 * n)
    fs = np.zeros(8 * n) if final_state else None
    lib().oracle_trace_rays(M, a, r_obs, incl, n, _dp(alpha), _dp(beta), h0, h_r0, r_escape,
                            horizon_factor, disk_r_in, disk_r_out, max_steps, _ip(status),
                            _ip(steps), _dp(hit), None if fs is None else fs.ctypes.data_as(C.c_void_p),
                            nthreads)
    if final_state:
        return status, steps, hit.reshape(n, 2).T.copy(), fs.reshape(8, n)
    return status, steps, hit.reshape(n, 2).T.copy()


def tangent(M, a, h, n_steps, y0, v):
    y0, v = _f64(y0, 8), _f64(v, 8)
    y = np.zeros(8)
    dy = np.zeros(8)
    lib().oracle_tangent(M, a, h, n_steps, _dp(y0), _dp(v), y.ctypes.data_as(C.c_void_p), _dp(dy))
    return y, dy


def ic_map(M, a, E, p):
    p = _f64(p, 5)
    y = np.zeros(8)
    lib().oracle_ic_map(M, a, E, _dp(p), _dp(y))
    return y


def grad_ic(M, a, h, n_steps, p_soa, E, target_soa, nthreads=0):
    p_soa = _f64(p_soa)
    n = p_soa.size // 5
    E = _f64(E, n)
    target_soa = _f64(target_soa, 3 * n)
    grad = np.zeros(5 * n)
    loss = np.zeros(n)
    lib().oracle_grad_ic(M, a, h, n_steps, n, _dp(p_soa), _dp(E), _dp(target_soa), _dp(grad),
                         loss.ctypes.data_as(C.c_void_p), nthreads)
    return grad.reshape(5, n), loss


def loss_ic(M, a, h, n_steps, p, E, target):
    return lib().oracle_loss_ic(M, a, h, n_steps, _dp(_f64(p, 5)), E, _dp(_f64(target, 3)))


def max_threads():
    return lib().oracle_max_threads()
