"""C ABI checks that need no GPU: the library loads, exports every symbol that
include/malbec.h declares, its structures have the header's layout, and argument
errors are reported without touching the device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "malbec.h")


@pytest.fixture(scope="module")
def m():
    import paper_1803_08320_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1803_08320_amd import _build_lib
        _build_lib.build()
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"MALBEC_API\s+[\w\s\*]*?\b(malbec_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(m):
    names = declared_functions()
    assert len(names) >= 8
    out = subprocess.run(["nm", "-D", "--defined-only", m.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (malbec_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    for name in names:
        assert hasattr(m.lib(), name)
    assert set(names) == set(m.EXPORTS)
    # internal C++ symbols stay hidden
    assert not re.search(r"\bT _ZN6malbec", out)


def test_struct_layout_matches_header(m, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "malbec.h"\n'
                   "#define P(T) printf(#T \" %zu\\n\", sizeof(T));\n"
                   "#define O(T, f) printf(#T \".\" #f \" %zu\\n\", offsetof(T, f));\n"
                   "int main(void){P(malbec_spacetime)P(malbec_batch)P(malbec_ic_spec)"
                   "P(malbec_run)P(malbec_camera)P(malbec_adaptive)O(malbec_adaptive, max_attempts)"
                   "P(malbec_grid)O(malbec_grid, r_stop)O(malbec_grid, nodes)O(malbec_grid, node_precision)"
                   "O(malbec_adaptive, steps_per_chunk)O(malbec_adaptive, schedule)O(malbec_ic_spec, rows)O(malbec_ic_spec, max_attempts)"
                   "O(malbec_ic_spec, strict)printf(\"ESAMPLE %d\\n\", MALBEC_ESAMPLE);"
                   "O(malbec_run, checkpoint_every)O(malbec_run, persistent)O(malbec_run, formulation)"
                   "O(malbec_camera, max_steps)O(malbec_camera, persistent)"
                   "O(malbec_batch, st_of_lane)return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in lines if l)
    assert int(got["malbec_spacetime"]) == C.sizeof(m.c_spacetime)
    assert int(got["malbec_batch"]) == C.sizeof(m.c_batch)
    assert int(got["malbec_ic_spec"]) == C.sizeof(m.c_ic_spec)
    assert int(got["malbec_run"]) == C.sizeof(m.c_run)
    assert int(got["malbec_camera"]) == C.sizeof(m.c_camera)
    assert int(got["malbec_adaptive"]) == C.sizeof(m.c_adaptive)
    assert int(got["malbec_grid"]) == C.sizeof(m.c_grid)
    assert int(got["malbec_grid.r_stop"]) == m.c_grid.r_stop.offset
    assert int(got["malbec_grid.nodes"]) == m.c_grid.nodes.offset
    assert int(got["malbec_grid.node_precision"]) == m.c_grid.node_precision.offset
    assert int(got["malbec_adaptive.max_attempts"]) == m.c_adaptive.max_attempts.offset
    assert int(got["malbec_adaptive.steps_per_chunk"]) == m.c_adaptive.steps_per_chunk.offset
    assert int(got["malbec_adaptive.schedule"]) == m.c_adaptive.schedule.offset
    assert int(got["malbec_ic_spec.rows"]) == m.c_ic_spec.rows.offset
    assert int(got["malbec_ic_spec.max_attempts"]) == m.c_ic_spec.max_attempts.offset
    assert int(got["malbec_ic_spec.strict"]) == m.c_ic_spec.strict.offset
    assert int(got["ESAMPLE"]) == m.ESAMPLE
    assert int(got["malbec_run.checkpoint_every"]) == m.c_run.checkpoint_every.offset
    assert int(got["malbec_run.persistent"]) == m.c_run.persistent.offset
    assert int(got["malbec_run.formulation"]) == m.c_run.formulation.offset
    assert int(got["malbec_camera.max_steps"]) == m.c_camera.max_steps.offset
    assert int(got["malbec_camera.persistent"]) == m.c_camera.persistent.offset
    assert int(got["malbec_batch.st_of_lane"]) == m.c_batch.st_of_lane.offset


def _batch(m, sts=((1.0, 0.9),)):
    arr = (m.c_spacetime * len(sts))(*[m.c_spacetime(M, a) for M, a in sts])
    return arr, m.c_batch(C.cast(arr, C.POINTER(m.c_spacetime)), len(sts), 0, None)


def _run(m, **kw):
    d = dict(h=0.02, n_steps=10, precision=0, block=0, horizon_factor=1.01, r_escape=1500.0,
             fp64_zone_factor=1.2, steps_per_chunk=0, checkpoint_every=0, persistent=0,
             formulation=0)
    d.update(kw)
    return m.c_run(**d)


FAKE = C.c_void_p(0x1000)  # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("kw,sts,n,expect", [
    (dict(h=0.0), ((1.0, 0.9),), 4, -1),
    (dict(h=float("nan")), ((1.0, 0.9),), 4, -1),
    (dict(n_steps=-1), ((1.0, 0.9),), 4, -1),
    (dict(), ((1.0, 1.2),), 4, -1),          # a > M
    (dict(), ((0.0, 0.0),), 4, -1),          # M <= 0
    (dict(), ((1.0, -0.1),), 4, -1),         # a < 0
    (dict(horizon_factor=0.5), ((1.0, 0.9),), 4, -1),
    (dict(precision=7), ((1.0, 0.9),), 4, -1),
    (dict(block=100), ((1.0, 0.9),), 4, -1),
    (dict(), ((1.0, 0.9),), -3, -1),         # n < 0
    (dict(checkpoint_every=4), ((1.0, 0.9),), 4, -1),  # no checkpoint buffer
    (dict(persistent=2), ((1.0, 0.9),), 4, -1),
    (dict(persistent=1), ((1.0, 0.9),), 4, -2),        # persistent needs a workspace
    (dict(formulation=2), ((1.0, 0.9),), 4, -1),
])
def test_integrate_argument_errors(m, kw, sts, n, expect):
    run = _run(m, **kw)
    arr, b = _batch(m, sts)
    rc = m.lib().malbec_integrate(C.byref(run), C.byref(b), n, FAKE, FAKE, FAKE, None, None, 0, None)
    assert rc == expect
    assert m.last_error() != ""


@pytest.mark.parametrize("kw,every,reset,mon,expect", [
    (dict(), 0, 1, FAKE, -1),                       # monitor_every < 1
    (dict(), 10, 2, FAKE, -1),                      # reset not 0 / 1
    (dict(), 10, 1, None, -1),                      # no monitor buffer
    (dict(h=-1.0), 10, 1, FAKE, -1),                # the run's own checks apply
    (dict(precision=1, fp64_zone_factor=0.5), 10, 1, FAKE, -1),
    (dict(checkpoint_every=4), 10, 1, FAKE, -4),    # no checkpoints here
    (dict(persistent=1), 10, 1, FAKE, -2),          # persistent needs a workspace
])
def test_monitored_argument_errors(m, kw, every, reset, mon, expect):
    run = _run(m, **kw)
    arr, b = _batch(m)
    rc = m.lib().malbec_integrate_monitored(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, every,
                                            reset, mon, None, 0, None)
    assert rc == expect
    assert m.last_error() != ""


def test_hamiltonian_with_checkpoints_is_unsupported(m):
    run = _run(m, formulation=1, checkpoint_every=4)
    arr, b = _batch(m)
    rc = m.lib().malbec_integrate(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, None, 0, None)
    assert rc == -4 and "Christoffel" in m.last_error()


def test_null_pointer_and_table_errors(m):
    run = _run(m)
    arr, b = _batch(m)
    assert m.lib().malbec_integrate(C.byref(run), C.byref(b), 4, None, FAKE, FAKE, None, None, 0,
                                    None) == -1
    assert "non-NULL" in m.last_error()
    assert m.lib().malbec_integrate(None, C.byref(b), 4, FAKE, FAKE, FAKE, None, None, 0, None) == -1
    assert m.lib().malbec_integrate(C.byref(run), None, 4, FAKE, FAKE, FAKE, None, None, 0, None) == -1
    big = [(1.0, 0.1)] * 65
    arr, b = _batch(m, big)
    assert m.lib().malbec_integrate(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, None, None, 0,
                                    None) == -1
    assert "n_st" in m.last_error()
    # zero lanes or zero steps: a valid no-op that enqueues nothing
    arr, b = _batch(m)
    assert m.lib().malbec_integrate(C.byref(run), C.byref(b), 0, None, None, None, None, None, 0,
                                    None) == 0
    assert m.last_error() == ""
    run0 = _run(m, n_steps=0)
    assert m.lib().malbec_integrate(C.byref(run0), C.byref(b), 4, FAKE, FAKE, FAKE, None, None, 0,
                                    None) == 0


def test_init_and_camera_argument_errors(m):
    arr, b = _batch(m)
    spec = m.ICSpec(mode=9).to_c(4)
    assert m.lib().malbec_init_particles(C.byref(spec), C.byref(b), 4, FAKE, None, None, None) == -1
    spec = m.ICSpec(mode=m.IC_CONSTANTS, max_attempts=0).to_c(4)
    assert m.lib().malbec_init_particles(C.byref(spec), C.byref(b), 4, FAKE, None, None, None) == -1
    spec = m.ICSpec(mode=m.IC_CONSTANTS, E_range=(1.0, 0.5)).to_c(4)
    assert m.lib().malbec_init_particles(C.byref(spec), C.byref(b), 4, FAKE, None, None, None) == -1
    spec = m.ICSpec(mode=m.IC_CANONICAL).to_c(4)
    assert m.lib().malbec_init_particles(C.byref(spec), C.byref(b), 4, FAKE, None, None, None) == -1
    cam = m.Camera(nx=4, ny=4).to_c()
    ws_need = m.workspace_bytes(m.OP_CAMERA, 16)
    assert m.workspace_bytes(m.OP_ADJOINT, 100, 256) == 256 * 8 * 100 * 8
    assert ws_need == 256 + 64 * 16  # work counter, then the rays' initial states
    # workspace too small
    assert m.lib().malbec_trace_camera(C.byref(cam), FAKE, FAKE, FAKE, None, FAKE, 4, None) == -2
    for bad in (dict(a=1.5), dict(incl=0.0), dict(nx=0), dict(h0=-1.0), dict(r_escape=10.0),
                dict(max_steps=0), dict(block=96)):
        kw = dict(nx=4, ny=4)
        kw.update(bad)
        cam = m.Camera(**kw).to_c()
        assert m.lib().malbec_trace_camera(C.byref(cam), FAKE, FAKE, FAKE, None, FAKE, ws_need,
                                           None) == -1, bad
    assert m.lib().malbec_invariants(C.byref(b), -1, FAKE, FAKE, None) == -1
    # adjoint: no checkpoint interval, no workspace, wrong precision
    run = _run(m, checkpoint_every=0)
    assert m.lib().malbec_adjoint(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                  None, FAKE, 10 ** 9, None) == -1
    run = _run(m, checkpoint_every=4)
    assert m.lib().malbec_adjoint(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                  None, FAKE, 8, None) == -2
    run = _run(m, checkpoint_every=4, precision=1)
    assert m.lib().malbec_adjoint(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                  None, FAKE, 10 ** 9, None) == -4
    run = _run(m, checkpoint_every=4, formulation=1)
    assert m.lib().malbec_adjoint(C.byref(run), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, FAKE, None,
                                  None, FAKE, 10 ** 9, None) == -4
    assert m.lib().malbec_convert_state(C.byref(b), 4, FAKE, 2, None) == -1
    assert m.lib().malbec_convert_state(C.byref(b), 4, None, 1, None) == -1
    assert m.lib().malbec_convert_state(C.byref(b), 0, None, 1, None) == 0
    assert m.version() >= 300


def _adaptive(m, **kw):
    d = dict(tau_end=10.0, rtol=1e-9, atol=1e-9, fac=0.9, facmin=0.2, facmax=5.0,
             max_attempts=100, horizon_factor=1.01, r_escape=1500.0, block=0, persistent=0,
             steps_per_chunk=0, schedule=0)
    d.update(kw)
    return m.c_adaptive(**d)


@pytest.mark.parametrize("kw,expect", [
    (dict(rtol=0.0), -1), (dict(atol=-1.0), -1), (dict(fac=1.5), -1), (dict(facmin=0.0), -1),
    (dict(facmax=0.5), -1), (dict(max_attempts=0), -1), (dict(tau_end=float("inf")), -1),
    (dict(block=100), -1), (dict(persistent=3), -1), (dict(persistent=1), -2),
    (dict(horizon_factor=0.5), -1), (dict(schedule=2), -1), (dict(schedule=-1), -1),
    (dict(schedule=1), -1), (dict(persistent=1, schedule=1), -2),
])
def test_adaptive_argument_errors(m, kw, expect):
    ad = _adaptive(m, **kw)
    arr, b = _batch(m)
    rc = m.lib().malbec_integrate_adaptive(C.byref(ad), C.byref(b), 4, FAKE, FAKE, FAKE, FAKE,
                                           FAKE, FAKE, None, 0, None)
    assert rc == expect, m.last_error()
    assert m.workspace_bytes(m.OP_ADAPTIVE, 10, 1) >= 8


def test_adaptive_noalloc_limits(m):
    """The no-allocation adaptive entry point refuses batches beyond its static scratch
    and a NULL control block before touching the device."""
    ad = _adaptive(m, persistent=1, schedule=1)
    arr, b = _batch(m)
    fn = m.lib().malbec_integrate_adaptive_noalloc
    big = m.NOALLOC_MAX_LANES + 1
    assert fn(C.byref(ad), C.byref(b), big, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert "no-allocation scratch" in m.last_error()
    assert fn(None, C.byref(b), 4, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1
    # the scratch holds the workspace of the largest batch it accepts
    assert m.workspace_bytes(m.OP_ADAPTIVE, m.NOALLOC_MAX_LANES, 2) == (
        256 + 2 * 4 * m.SCHED_BUCKETS + 8 * m.NOALLOC_MAX_LANES)


def test_adaptive_order_workspace_and_argument_errors(m):
    """Workspace of the periapsis schedule (bucket counts and offsets, keys, order) and the
    argument checks of malbec_adaptive_order, none of which touches the device."""
    rnd = lambda x: (x + 255) // 256 * 256
    for n in (1, 255, 1000, 1 << 20):
        assert m.workspace_bytes(m.OP_ADAPTIVE_ORDER, n, 0) == 2 * 4 * m.SCHED_BUCKETS + rnd(4 * n)
        assert m.workspace_bytes(m.OP_ADAPTIVE, n, 2) == (256 + 2 * 4 * m.SCHED_BUCKETS + rnd(4 * n)
                                                           + 4 * n)
        assert m.workspace_bytes(m.OP_ADAPTIVE, n, 1) == 256
    assert m.workspace_bytes(m.OP_ADAPTIVE_ORDER, 0, 0) == 0
    arr, b = _batch(m)
    order = m.lib().malbec_adaptive_order
    big = 1 << 30
    assert order(C.byref(b), -1, FAKE, FAKE, FAKE, 10.0, FAKE, None, FAKE, big, None) == -1
    assert order(C.byref(b), 1 << 32, FAKE, FAKE, FAKE, 10.0, FAKE, None, FAKE, big, None) == -1
    assert order(C.byref(b), 4, FAKE, FAKE, FAKE, 10.0, None, None, FAKE, big, None) == -1
    assert order(C.byref(b), 4, None, FAKE, FAKE, 10.0, FAKE, None, FAKE, big, None) == -1
    assert order(C.byref(b), 4, FAKE, FAKE, FAKE, float("nan"), FAKE, None, FAKE, big, None) == -1
    assert order(C.byref(b), 4, FAKE, FAKE, FAKE, 10.0, FAKE, None, FAKE, 100, None) == -2
    assert order(C.byref(b), 4, FAKE, FAKE, FAKE, 10.0, FAKE, None, None, big, None) == -2
    assert order(C.byref(b), 0, None, None, None, 10.0, None, None, None, 0, None) == 0


@pytest.mark.parametrize("kw,run_kw,expect", [
    (dict(nr=3), {}, -1), (dict(dr=0.0), {}, -1), (dict(th0=0.0), {}, -1),
    (dict(dth=1.0), {}, -1), (dict(r_stop=1.0), {}, -1), (dict(nodes=None), {}, -1),
    ({}, dict(formulation=0), -1), ({}, dict(precision=1), -4), ({}, dict(persistent=1), -4),
    ({}, dict(r_escape=100.0), -1), ({}, dict(h=-1.0), -1), (dict(node_precision=2), {}, -1),
    (dict(node_precision=-1), {}, -1),
])
def test_grid_argument_errors(m, kw, run_kw, expect):
    d = dict(nr=16, nth=8, r0=2.5, dr=0.5, th0=0.5, dth=0.2, r_stop=3.2, nodes=0x1000)
    d.update(kw)
    g = m.c_grid(**d)
    r = dict(formulation=1, r_escape=8.0)
    r.update(run_kw)
    run = _run(m, **r)
    rc = m.lib().malbec_integrate_grid(C.byref(run), C.byref(g), 4, FAKE, FAKE, FAKE, None)
    assert rc == expect, m.last_error()
    d = dict(nr=16, nth=8, r0=2.5, dr=0.5, th0=0.5, dth=0.2, r_stop=3.2, nodes=0x1000)
    g = m.c_grid(**d)
    assert m.lib().malbec_grid_fill_kerr(C.byref(g), 1.0, 0.5, C.c_void_p(0x2000), None) == -1
    assert m.lib().malbec_grid_fill_kerr(C.byref(g), 1.0, 1.5, C.c_void_p(0x1000), None) == -1


def test_flop_count_constant(m, tmp_path):
    """The roofline's flops per lane-step equal the static count of the templates: the
    direct evaluation of the acceleration (the work of a step) and the regrouped one the
    kernels instantiate."""
    exe = tmp_path / "flopcount"
    src = os.path.join(ROOT, "paper_1803_08320_amd", "csrc", "flopcount.cpp")
    subprocess.run(["g++", "-O0", "-std=c++17", src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    vals = dict(l.split() for l in out.strip().split("\n"))
    assert int(vals["step_flops"]) == m.FLOPS_PER_STEP_F64
    assert int(vals["step_flops_kernel"]) == m.FLOPS_PER_STEP_F64_KERNEL
    assert int(vals["ham_step_flops"]) == m.FLOPS_PER_STEP_F64_HAM
    assert int(vals["f32k_step_flops"]) == m.FLOPS_PER_STEP_F32K
    assert int(vals["f32k_step_flops_kernel"]) == m.FLOPS_PER_STEP_F32K_KERNEL
    assert int(vals["f32k_ham_step_flops"]) == m.FLOPS_PER_STEP_F32K_HAM
    assert int(vals["dp45_attempt_flops"]) == m.FLOPS_PER_ATTEMPT_DP45
    assert int(vals["dp45_attempt_flops_kernel"]) == m.FLOPS_PER_ATTEMPT_DP45_KERNEL
    # the regrouped evaluation needs fewer operations than the direct one
    assert int(vals["rhs_flops_kernel"]) < int(vals["rhs_flops"])


def test_missing_library_and_host_tensors_fail_loudly(m, monkeypatch):
    """No fallback: without the built library the binding raises, and host tensors are
    refused before any call (every step runs in the HIP kernels)."""
    import torch
    monkeypatch.setattr(m, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libmalbec.so"))
    monkeypatch.setattr(m, "_lib", None)
    with pytest.raises(ImportError):
        m.lib()
    monkeypatch.undo()
    m.lib()
    state = torch.zeros((8, 4), dtype=torch.float64)
    status = torch.zeros(4, dtype=torch.int32)
    steps = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(ValueError, match="device tensor"):
        m.integrate(state, status, steps, [(1.0, 0.9)], h=0.02, n_steps=10)
