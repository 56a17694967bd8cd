#!/usr/bin/env python3
"""Benchmark: geodesic RK4 lane-steps per second on one MI355X (Kerr, FP64).

Workload (one benchmark "step" = one pass of the hot path over the batch):
Kerr M = 1, a = 0.9, 1,048,576 timelike bound geodesics drawn on the device
(r0 in [5, 50], theta0 in [pi/4, 3pi/4], E in [0.92, 0.98], L_z in [2.5, 4.5],
Carter Q in [0, 12], accepted when the radial and polar potentials are >= 0,
random signs of u^r and u^theta, seed 2), then: reset the state, invariant
monitor, 20,000 fixed RK4 steps of h = 0.02 M in FP64 with horizon/escape
termination, invariant monitor.  Inputs are resident in HBM before timing.

value = sum over lanes of the RK4 steps each lane took / wall time of the timed
steps.  roofline: FP64 vector ALU bound; achieved = algorithmic flops per
lane-step (FLOPS_PER_STEP_F64 = 514, the static count of the step with the direct
evaluation of the acceleration) x lane-steps of one integrate launch / that
launch's average duration (HIP events on its stream); the kernel evaluates the same
step in fewer operations (FLOPS_PER_STEP_F64_KERNEL), reported beside it.
cpu_baseline: the oracle (plain C, FP64) on a strided sample of the same
workload, on the host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
# 256 CU x 2.4 GHz x 256 FP32 flop/clk/CU: the published vector FP32 figure, reached
# here without packed instructions (a wave64 FP32 VALU instruction issues in about half
# the clocks of an FP64 one, counters of the FP32-compensated kernel)
PEAK_FP32_VECTOR_TFLOPS = 157.3

# HBM traffic of one rk4_f64_kernel launch of this workload, from rocprofv3 counter
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the ratio of a
# plain 1 GiB device copy's known bytes to what the same counter reads for it.  The
# figures hold for the sources that define the kernel's body, whose SHA-256 is given;
# after any change to them the traffic is reported as null until the counters are
# taken again.
KERNEL_SOURCES = ("integrate.hip", "kerr_device.hpp", "kerr_accel.hpp", "ham_accel.hpp",
                  "persistent.hpp", "sincos_table.hpp")
TRAFFIC = {"sources_sha256": "5a6ab0341c68de51e9c473087ee15a8d581b8cf3b3e74fcb06994aca22ca6b95",
           "fetch_kib": 36960.0625, "fetch_scale": 1048576 / 524307.5625,
           "write_kib": 73728.0, "write_scale": 1048576 / 1048576.0}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1803_08320_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic_bytes():
    t = TRAFFIC
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--lanes", type=int, default=1 << 20)
    p.add_argument("--rk-steps", type=int, default=20000)
    p.add_argument("--block", type=int, default=0)
    p.add_argument("--cpu-lanes", type=int, default=12288,
                   help="oracle sample: this many strided lanes x the full step count")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-f32k", action="store_true", help="skip the FP32-compensated leg")
    p.add_argument("--no-ham", action="store_true", help="skip the Hamiltonian-form leg")
    p.add_argument("--no-traj", action="store_true", help="skip the trajectory-output leg")
    p.add_argument("--no-adaptive", action="store_true", help="skip the adaptive (DP45) leg")
    p.add_argument("--no-grid", action="store_true", help="skip the gridded 3+1 metric leg")
    p.add_argument("--no-e2e", action="store_true",
                   help="skip the transfer-inclusive leg and the 1/8-shard leg")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the camera, mixed-spin batch and adjoint legs")
    p.add_argument("--probe-copy-bytes", type=int, default=0,
                   help="first run one device-to-device copy of this many bytes (a plain copy "
                        "kernel of known size, used to calibrate HBM byte counters)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU (--gpus 1): lanes are independent, so a batch split "
              "over G GPUs runs its 1/G share per GPU (see the shard_1_of_8 leg); runs on "
              "several GPUs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1803_08320_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    import paper_1803_08320_amd as m

    torch.cuda.set_device(0)
    if args.probe_copy_bytes:
        src = torch.ones(args.probe_copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    st = [(1.0, 0.9)]
    n, n_rk, h = args.lanes, args.rk_steps, 0.02
    spec = m.ICSpec(mode=m.IC_CONSTANTS, seed=2)
    s0, consts, attempts = m.init_particles(spec, st, n)
    state = torch.empty_like(s0)
    status, steps = m.new_lane_arrays(n)
    inv0 = torch.empty((4, n), dtype=torch.float64, device="cuda")
    inv1 = torch.empty_like(inv0)
    torch.cuda.synchronize()
    # launch shape: the autotuner's choice for this batch (timed on a sample before the
    # timed region, cached), which the integrate calls below take through block = 0
    if args.block == 0:
        from paper_1803_08320_amd import autotune
        shape_block = autotune.integrate_shape(s0, st, h)[0]
    else:
        shape_block = args.block

    def one_step(ev=None):
        state.copy_(s0)
        status.zero_()
        steps.zero_()
        m.invariants(state, st, out=inv0)
        if ev:
            ev[0].record()
        m.integrate(state, status, steps, st, h=h, n_steps=n_rk, block=args.block)
        if ev:
            ev[1].record()
        m.invariants(state, st, out=inv1)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    lane_steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_step_lane_steps = int(steps.sum().item())
    lane_steps = per_step_lane_steps * args.steps
    wall = t1 - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    achieved = m.FLOPS_PER_STEP_F64 * per_step_lane_steps / avg_kern_s / 1e12

    # physics of the last step: conserved-quantity drift on lanes still active
    i0, i1 = inv0.cpu().numpy(), inv1.cpu().numpy()
    act = status.cpu().numpy() == 0
    dE = np.abs(i1[0] / i0[0] - 1)[act]
    Qok = act & (i0[2] >= 0.1)
    dQ = np.abs(i1[2] / i0[2] - 1)[Qok]

    result = {
        "metric": "geodesic RK4 steps/sec on 1 GPU (Kerr), FP64 vs FP32-comp at stated dQ/Q",
        "value": lane_steps / wall,
        "unit": "lane-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "kerr_a0.9_bound_timelike_1M_lanes_20000_steps_h0.02_fp64",
                   "lanes": n, "rk4_steps": n_rk, "h": h, "spin": 0.9, "seed": 2,
                   "block": shape_block,
                   "launch_shape": "autotuned" if args.block == 0 else "fixed by --block"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": measured_traffic_bytes(), "kernel": "rk4_f64_kernel",
                     "algorithmic_bytes": 144.0 * n,
                     "flops_per_lane_step": m.FLOPS_PER_STEP_F64,
                     "kernel_flops_per_lane_step": m.FLOPS_PER_STEP_F64_KERNEL,
                     "frac_at_kernel_flops": achieved * m.FLOPS_PER_STEP_F64_KERNEL
                     / m.FLOPS_PER_STEP_F64 / PEAK_FP64_VECTOR_TFLOPS,
                     "kernel_ms_avg": 1e3 * avg_kern_s,
                     "kernel_ms_median": float(np.median(kern_ms)),
                     "kernel_ms_each": [round(x, 3) for x in kern_ms]},
        "physics": {"active_frac": float(act.mean()),
                    "dE_over_E_p99": float(np.quantile(dE, 0.99)) if dE.size else None,
                    "dQ_over_Q_p99": float(np.quantile(dQ, 0.99)) if dQ.size else None,
                    "dQ_over_Q_max": float(dQ.max()) if dQ.size else None},
        "context": {"paper_gpu_lane_steps_per_s": 3.69e6,
                    "paper_hardware": "GTX 960M, Kerr a=0.5, h=0.1, FP64, no I/O"},
    }

    if not args.no_e2e:
        # the same workload with the state starting and ending in pinned host memory:
        # host-to-device copy of the initial state, the integration and the
        # device-to-host copy of state, status and steps, all inside the timed region
        # (the figure a caller that hands over host buffers sees; not the headline)
        res_final = state.clone()
        host_in = s0.cpu().pin_memory()
        host_out = torch.empty_like(host_in, device="cpu").pin_memory()
        st_out = torch.empty(n, dtype=torch.int32).pin_memory()
        sp_out = torch.empty(n, dtype=torch.int32).pin_memory()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

        def run_e2e():
            ev[0].record()
            state.copy_(host_in, non_blocking=True)
            status.zero_()
            steps.zero_()
            ev[1].record()
            m.integrate(state, status, steps, st, h=h, n_steps=n_rk, block=args.block)
            ev[2].record()
            host_out.copy_(state, non_blocking=True)
            st_out.copy_(status, non_blocking=True)
            sp_out.copy_(steps, non_blocking=True)
            ev[3].record()
        run_e2e()
        torch.cuda.synchronize()
        t = time.perf_counter()
        run_e2e()
        torch.cuda.synchronize()
        wall_e2e = time.perf_counter() - t
        e_steps = int(sp_out.to(torch.int64).sum().item())
        h2d_ms, d2h_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
        moved = 64.0 * n + 72.0 * n
        result["end_to_end"] = {
            "value": e_steps / wall_e2e, "unit": "lane-steps/s",
            "vs_resident": e_steps / wall_e2e / result["value"],
            "h2d_ms": h2d_ms, "d2h_ms": d2h_ms,
            "pcie_GB_per_s": moved / ((h2d_ms + d2h_ms) / 1e3) / 1e9,
            "bytes_moved": moved,
            "bitwise_equal_to_resident": bool(torch.equal(host_out, res_final.cpu()))}

        # one GPU's share of the same batch on eight GPUs (lane ranges of 131,072)
        ns = n // 8
        sh_state = s0[:, :ns].contiguous()
        sh0 = sh_state.clone()
        sh_status, sh_steps = m.new_lane_arrays(ns)
        evs8 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        for rec in (False, True):
            sh_state.copy_(sh0)
            sh_status.zero_()
            sh_steps.zero_()
            if rec:
                evs8[0].record()
            m.integrate(sh_state, sh_status, sh_steps, st, h=h, n_steps=n_rk, block=args.block)
            if rec:
                evs8[1].record()
        torch.cuda.synchronize()
        dt8 = evs8[0].elapsed_time(evs8[1]) / 1e3
        s8 = int(sh_steps.to(torch.int64).sum().item())
        result["shard_1_of_8"] = {
            "value": s8 / dt8, "unit": "lane-steps/s", "lanes": ns, "kernel_ms": 1e3 * dt8,
            "vs_full_batch": s8 / dt8 / (per_step_lane_steps / avg_kern_s),
            "bitwise_equal_to_full_batch_slice": bool(torch.equal(sh_state, res_final[:, :ns]))}
        del sh_state, sh0, sh_status, sh_steps, res_final

    if not args.no_f32k:
        # FP32 state with compensated update, FP64 within 1.2 r_+: same ICs, one timed run
        fin64 = state.clone()
        st64 = status.clone()
        state.copy_(s0)
        status.zero_()
        steps.zero_()
        m.integrate(state, status, steps, st, h=h, n_steps=n_rk, precision="f32k",
                    fp64_zone_factor=1.2, block=args.block)  # warm-up
        state.copy_(s0)
        status.zero_()
        steps.zero_()
        ev32 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        torch.cuda.synchronize()
        ev32[0].record()
        m.integrate(state, status, steps, st, h=h, n_steps=n_rk, precision="f32k",
                    fp64_zone_factor=1.2, block=args.block)
        ev32[1].record()
        torch.cuda.synchronize()
        dt = ev32[0].elapsed_time(ev32[1]) / 1e3
        k_steps = int(steps.sum().item())
        m.invariants(state, st, out=inv1)
        j1 = inv1.cpu().numpy()
        act32 = (status == 0).cpu().numpy() & act
        dE32 = np.abs(j1[0] / i0[0] - 1)[act32]
        q32 = act32 & (i0[2] >= 0.1)
        dQ32 = np.abs(j1[2] / i0[2] - 1)[q32]
        a64, a32 = fin64.cpu().numpy(), state.cpu().numpy()

        def cart(y):
            rr = np.sqrt(y[1] ** 2 + 0.81)
            return np.stack([rr * np.sin(y[2]) * np.cos(y[3]), rr * np.sin(y[2]) * np.sin(y[3]),
                             y[1] * np.cos(y[2])])
        pos = (np.linalg.norm(cart(a32) - cart(a64), axis=0) / a64[1])[act32]
        v32 = k_steps / dt
        ach32 = m.FLOPS_PER_STEP_F32K * v32 / 1e12
        result["f32k"] = {"value": v32, "unit": "lane-steps/s", "speedup_vs_f64": v32 / result["value"],
                          "kernel_ms": 1e3 * dt,
                          "roofline": {"bound": "alu", "achieved": ach32,
                                       "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                       "frac": ach32 / PEAK_FP32_VECTOR_TFLOPS,
                                       "flops_per_lane_step": m.FLOPS_PER_STEP_F32K,
                                       "kernel_flops_per_lane_step": m.FLOPS_PER_STEP_F32K_KERNEL,
                                       "dtype": "f32 stages, f32 pair state"},
                          "zone": "FP64 steps inside 1.2 r_+",
                          "dE_over_E_p99": float(np.quantile(dE32, 0.99)),
                          "dQ_over_Q_p99": float(np.quantile(dQ32, 0.99)),
                          "dQ_over_Q_max": float(dQ32.max()),
                          "pos_err_vs_f64_p50": float(np.quantile(pos, 0.5)),
                          "pos_err_vs_f64_p99": float(np.quantile(pos, 0.99)),
                          "status_agree_frac": float(((status == st64).float().mean()).item())}

    if not args.no_ham:
        # Hamilton's equations (Section 2, eq. Ham) on the same initial data: state
        # (x^mu, p_mu), converted once before timing
        z0 = s0.clone()
        m.convert_state(z0, st, True)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

        def run_ham(record):
            state.copy_(z0)
            status.zero_()
            steps.zero_()
            if record:
                ev[0].record()
            m.integrate(state, status, steps, st, h=h, n_steps=n_rk, block=args.block,
                        formulation="hamiltonian")
            if record:
                ev[1].record()
        run_ham(False)
        torch.cuda.synchronize()
        run_ham(True)
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) / 1e3
        h_steps = int(steps.sum().item())
        m.convert_state(state, st, False)
        m.invariants(state, st, out=inv1)
        j1 = inv1.cpu().numpy()
        acth = (status == 0).cpu().numpy() & act
        qh = acth & (i0[2] >= 0.1)
        dQh = np.abs(j1[2] / i0[2] - 1)[qh]
        vh = h_steps / dt
        ach = m.FLOPS_PER_STEP_F64_HAM * h_steps / dt / 1e12
        result["hamiltonian"] = {
            "value": vh, "unit": "lane-steps/s", "speedup_vs_christoffel": vh / result["value"],
            "kernel_ms": 1e3 * dt, "flops_per_lane_step": m.FLOPS_PER_STEP_F64_HAM,
            "achieved_tflops": ach, "frac": ach / PEAK_FP64_VECTOR_TFLOPS,
            "dE_over_E_max": float(np.abs(j1[0] / i0[0] - 1)[acth].max()),
            "dQ_over_Q_p99": float(np.quantile(dQh, 0.99)),
            "dQ_over_Q_max": float(dQh.max())}

    if not args.no_ham and not args.no_f32k:
        # Hamilton's equations on the FP32-compensated state, FP64 within 1.2 r_+
        state.copy_(z0)
        status.zero_()
        steps.zero_()
        m.integrate(state, status, steps, st, h=h, n_steps=n_rk, precision="f32k",
                    fp64_zone_factor=1.2, block=args.block, formulation="hamiltonian")
        state.copy_(z0)
        status.zero_()
        steps.zero_()
        ev[0].record()
        m.integrate(state, status, steps, st, h=h, n_steps=n_rk, precision="f32k",
                    fp64_zone_factor=1.2, block=args.block, formulation="hamiltonian")
        ev[1].record()
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) / 1e3
        hk_steps = int(steps.sum().item())
        m.convert_state(state, st, False)
        m.invariants(state, st, out=inv1)
        j1 = inv1.cpu().numpy()
        acth = (status == 0).cpu().numpy() & act
        qh = acth & (i0[2] >= 0.1)
        dQh = np.abs(j1[2] / i0[2] - 1)[qh]
        achh32 = m.FLOPS_PER_STEP_F32K_HAM * hk_steps / dt / 1e12
        result["f32k_hamiltonian"] = {
            "value": hk_steps / dt, "unit": "lane-steps/s",
            "speedup_vs_f64_christoffel": hk_steps / dt / result["value"],
            "kernel_ms": 1e3 * dt,
            "roofline": {"bound": "alu", "achieved": achh32, "peak": PEAK_FP32_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": achh32 / PEAK_FP32_VECTOR_TFLOPS,
                         "flops_per_lane_step": m.FLOPS_PER_STEP_F32K_HAM},
            "zone": "FP64 steps inside 1.2 r_+",
            "dE_over_E_max": float(np.abs(j1[0] / i0[0] - 1)[acth].max()),
            "dQ_over_Q_p99": float(np.quantile(dQh, 0.99)),
            "dQ_over_Q_max": float(dQh.max())}

    if not args.no_traj:
        # the paper's output stream: (tau, t, x, y, z) of every lane every 200 steps,
        # moved to pinned host memory on a second stream while the next chunk runs;
        # chunks of 2 records (400 steps, 84 MB): the first chunk's integration and the
        # last chunk's copy do not overlap anything, so short chunks keep that tail small
        from paper_1803_08320_amd.stream import stream_trajectories
        every, per_chunk = 200, 2
        seen = {"bytes": 0}

        def sink(recs, k):
            seen["bytes"] += recs.nbytes
            seen["tau_last"] = float(recs[-1, 0, 0])

        def run_stream():
            state.copy_(s0)
            status.zero_()
            steps.zero_()
            return stream_trajectories(state, status, steps, st, h, n_rk, every, per_chunk, sink,
                                       block=args.block)
        run_stream()  # warm-up (allocates the pinned buffers)
        seen["bytes"] = 0
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = run_stream()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        ls = int(steps.sum().item())
        result["trajectory_stream"] = {
            "value": ls / dt, "unit": "lane-steps/s", "vs_no_output": ls / dt / result["value"],
            "record_every": every, "records": info["records"], "chunks": info["chunks"],
            "bytes_to_host": seen["bytes"], "host_GB_per_s": seen["bytes"] / dt / 1e9,
            "wall_s": dt}

    if not args.no_adaptive:
        # Dormand-Prince 5(4) with a per-lane step size on the same initial data, to the
        # same affine parameter (tau_end = 20,000 x 0.02), persistent work queue; the
        # tolerance 1e-12 gives invariant drift of the order of the fixed-step run's
        tau_end = n_rk * h
        tau = torch.zeros(n, dtype=torch.float64, device="cuda")
        hstep = torch.empty(n, dtype=torch.float64, device="cuda")
        rej = torch.zeros(n, dtype=torch.int32, device="cuda")
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

        def run_dp(record, schedule):
            state.copy_(s0)
            tau.zero_()
            hstep.fill_(0.1)
            status.zero_()
            steps.zero_()
            rej.zero_()
            if record:
                ev[0].record()
            m.integrate_adaptive(state, tau, hstep, status, steps, rej, st, tau_end, rtol=1e-12,
                                 atol=1e-12, persistent=True, block=args.block,
                                 schedule=schedule)
            if record:
                ev[1].record()
        # lanes in index order, then in periapsis order (longest expected first; the
        # order's computation is inside the timed call); the results are identical
        run_dp(False, "index")
        run_dp(True, "index")
        torch.cuda.synchronize()
        dt_index = ev[0].elapsed_time(ev[1]) / 1e3
        run_dp(False, "periapsis")
        torch.cuda.synchronize()
        run_dp(True, "periapsis")
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) / 1e3
        m.invariants(state, st, out=inv1)
        j1 = inv1.cpu().numpy()
        actd = (status == 0).cpu().numpy() & act
        qd = actd & (i0[2] >= 0.1)
        acc_att, rej_att = int(steps.sum().item()), int(rej.sum().item())
        lane_tau = float(tau.sum().item())
        result["adaptive_dp45"] = {
            "lane_tau_per_s": lane_tau / dt, "rk4_lane_tau_per_s": result["value"] * h,
            "speedup_vs_rk4_h0.02": lane_tau / dt / (result["value"] * h),
            "rtol": 1e-12, "atol": 1e-12, "schedule": "periapsis", "kernel_ms": 1e3 * dt,
            "index_order_ms": 1e3 * dt_index, "speedup_vs_index_order": dt_index / dt,
            "accepted_per_lane": acc_att / n, "rejected_per_lane": rej_att / n,
            "accepted_per_lane_p99": float(torch.quantile(steps[:1 << 20].double(), 0.99).item()),
            "accepted_per_lane_max": int(steps.max().item()),
            "attempts_per_s": (acc_att + rej_att) / dt,
            "achieved_tflops": m.FLOPS_PER_ATTEMPT_DP45 * (acc_att + rej_att) / dt / 1e12,
            "frac": m.FLOPS_PER_ATTEMPT_DP45 * (acc_att + rej_att) / dt / 1e12
            / PEAK_FP64_VECTOR_TFLOPS,
            "dE_over_E_p99": float(np.quantile(np.abs(j1[0] / i0[0] - 1)[actd], 0.99)),
            "dQ_over_Q_p99": float(np.quantile(np.abs(j1[2] / i0[2] - 1)[qd], 0.99))}
        # Each lane is one work item of ~440 attempts (p99 ~1,200), so a batch of n lanes
        # fills the resident lane slots only n / slots times over; whatever tail the
        # order leaves (slots idle while the last lanes finish) is a visible part of the
        # launch.  The same lanes four times over (4 n) show the rate with it amortised.
        s4 = s0.repeat(1, 4)
        st4 = torch.empty_like(s4)
        tau4 = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
        h4 = torch.full((4 * n,), 0.1, dtype=torch.float64, device="cuda")
        status4, steps4 = m.new_lane_arrays(4 * n)
        rej4 = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
        for record in (False, True):
            st4.copy_(s4)
            tau4.zero_()
            h4.fill_(0.1)
            status4.zero_()
            steps4.zero_()
            rej4.zero_()
            ev[0].record()
            m.integrate_adaptive(st4, tau4, h4, status4, steps4, rej4, st, tau_end, rtol=1e-12,
                                 atol=1e-12, persistent=True, block=args.block,
                                 schedule="periapsis")
            ev[1].record()
        torch.cuda.synchronize()
        dt4 = ev[0].elapsed_time(ev[1]) / 1e3
        att4 = int(steps4.sum().item()) + int(rej4.sum().item())
        result["adaptive_dp45"]["batch_x4"] = {
            "lanes": 4 * n, "kernel_ms": 1e3 * dt4, "attempts_per_s": att4 / dt4,
            "frac": m.FLOPS_PER_ATTEMPT_DP45 * att4 / dt4 / 1e12 / PEAK_FP64_VECTOR_TFLOPS}
        del s4, st4, tau4, h4, status4, steps4, rej4

    if not args.no_grid:
        # the same orbits in Kerr sampled in 3+1 form on a 801 x 401 (r, theta) grid
        # (Section 2): Hamilton's equations with the interpolated metric, 2,000 steps
        n_g = 2000
        g = m.grid_kerr(1.0, 0.9, 801, 401, 1.5, 60.0 / 800, 0.1, (math.pi - 0.2) / 400,
                        1.2 * (1.0 + math.sqrt(1.0 - 0.81)))
        z0 = s0.clone()
        m.convert_state(z0, st, True)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

        def run_grid(record, grid):
            state.copy_(z0)
            status.zero_()
            steps.zero_()
            if record:
                ev[0].record()
            m.integrate_grid(state, status, steps, grid, h, n_g, 55.0, block=args.block)
            if record:
                ev[1].record()
        run_grid(False, g)
        torch.cuda.synchronize()
        run_grid(True, g)
        torch.cuda.synchronize()
        dt = ev[0].elapsed_time(ev[1]) / 1e3
        ls = int(steps.sum().item())
        end64 = state.clone()
        st64 = status.clone()
        act64 = st64 == 0
        result["grid_3p1"] = {
            "value": ls / dt, "unit": "lane-steps/s", "grid": [801, 401],
            "rk4_steps": n_g, "kernel_ms": 1e3 * dt,
            "vs_analytic_hamiltonian": (ls / dt) / result["hamiltonian"]["value"]
            if "hamiltonian" in result else None,
            # stencil bytes the interpolation reads per lane-step (mostly from the
            # lanes' LDS stencil caches; the grid's rows only when a lane changes cell)
            "stencil_bytes_per_lane_step": 4 * 16 * 40,
            "stencil_GB_per_s": 4 * 16 * 40 * ls / dt / 1e9,
            "active_frac": float((status == 0).float().mean().item())}
        # the same grid with its node values stored in single precision (half the
        # gathered bytes; arithmetic in FP64), and how far its orbits end from the
        # double-precision grid's
        g32 = m.grid_kerr(1.0, 0.9, 801, 401, 1.5, 60.0 / 800, 0.1, (math.pi - 0.2) / 400,
                          1.2 * (1.0 + math.sqrt(1.0 - 0.81)), node_dtype=torch.float32)
        run_grid(False, g32)
        torch.cuda.synchronize()
        run_grid(True, g32)
        torch.cuda.synchronize()
        dt32 = ev[0].elapsed_time(ev[1]) / 1e3
        ls32 = int(steps.sum().item())
        both = act64 & (status == 0)
        dpos = ((state[1:4] - end64[1:4]).abs() / end64[1:4].abs().clamp(min=1.0)).amax(dim=0)
        dpos = dpos[both].cpu().numpy()
        result["grid_3p1"]["node_f32"] = {
            "value": ls32 / dt32, "unit": "lane-steps/s", "kernel_ms": 1e3 * dt32,
            "speedup_vs_f64_nodes": (ls32 / dt32) / (ls / dt),
            "stencil_bytes_per_lane_step": 4 * 16 * 20,
            "stencil_GB_per_s": 4 * 16 * 20 * ls32 / dt32 / 1e9,
            "pos_diff_vs_f64_nodes_p50": float(np.quantile(dpos, 0.5)),
            "pos_diff_vs_f64_nodes_p99": float(np.quantile(dpos, 0.99)),
            "status_agree_frac": float((status == st64).float().mean().item())}
        del g32, end64, st64

    if not args.no_extra:
        result["extra"] = extra_legs(m, torch, np)
        result["schwarzschild"] = schwarzschild_leg(m, torch, np)

    if not args.no_cpu_baseline:
        import oracle
        k = max(1, n // args.cpu_lanes)
        idx = list(range(0, n, k))[: args.cpu_lanes]
        ranges = (spec.r_range, spec.th_range, spec.E_range, spec.Lz_range, spec.Q_range)
        cols = [oracle.ic_constants(2, st, 1, ranges, lane0=i)[1] for i in idx]
        sc = np.concatenate(cols, axis=1)
        nthreads = oracle.max_threads()
        t = time.perf_counter()
        _, _, ref_steps = oracle.integrate(st, sc, h, n_rk, nthreads=nthreads)
        dt = time.perf_counter() - t
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh
                                  if ln.startswith("model name")), None)
        except OSError:
            pass
        result["cpu_baseline"] = {"value": float(ref_steps.sum()) / dt, "unit": "lane-steps/s",
                                  "cores": nthreads, "kind": "oracle", "cpu_model": cpu_model,
                                  "sample": "%d strided lanes of the workload x %d RK4 steps "
                                            "(%.1f s wall)" % (len(idx), n_rk, dt)}
        if not args.no_extra:
            result["cpu_baseline_by_config"] = oracle_configs(oracle, np, nthreads, result)
    print(json.dumps(result))


def _timed(torch, fn):
    fn()  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def schwarzschild_leg(m, torch, np):
    """Schwarzschild M = 1: 1,024 equatorial timelike lanes on circular orbits with
    r0 in [6.5, 20] and L perturbed by up to 1e-3 relative (seed 1), h = 0.01, 10,000
    steps, FP64; with the drift of E, L and of the norm from -1.  Too few lanes to fill
    the chip (16 waves): the rate shown is latency-bound."""
    st = [(1.0, 0.0)]
    n = 1024
    spec = m.ICSpec(mode=m.IC_CIRCULAR, seed=1, r_lo=6.5, r_hi=20.0, dL=1e-3)
    s0, c0, _ = m.init_particles(spec, st, n)
    state = torch.empty_like(s0)
    status, steps = m.new_lane_arrays(n)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def run():
        state.copy_(s0)
        status.zero_()
        steps.zero_()
        ev[0].record()
        m.integrate(state, status, steps, st, h=0.01, n_steps=10000)
        ev[1].record()
    run()
    run()
    torch.cuda.synchronize()
    dt = ev[0].elapsed_time(ev[1]) / 1e3
    inv = m.invariants(state, st)
    i0 = m.invariants(s0, st)
    torch.cuda.synchronize()
    i0, i1 = i0.cpu().numpy(), inv.cpu().numpy()
    return {"value": float(steps.sum().item()) / dt, "unit": "lane-steps/s", "kernel_ms": 1e3 * dt,
            "lanes": n, "rk4_steps": 10000, "h": 0.01,
            "dE_over_E_max": float(np.abs(i1[0] / i0[0] - 1).max()),
            "dL_over_L_max": float(np.abs(i1[1] / i0[1] - 1).max()),
            "norm_drift_max": float(np.abs(i1[3] + 1).max()),
            "active_frac": float((status == 0).float().mean().item())}


def oracle_configs(oracle, np, nthreads, result):
    """The oracle timed on a bounded sample of each of the other workloads, on the host's
    cores, beside the GPU's rate on the full workload."""
    out = {}
    kr = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))

    def gpu_ratio(entry, gpu_value):
        if gpu_value is not None:
            entry["gpu_value"] = gpu_value
            entry["gpu_over_oracle"] = gpu_value / entry["value"]
        return entry
    # Schwarzschild: all 1,024 lanes x 10,000 steps
    s1 = oracle.ic_circular(1, 1.0, 0.0, 1024, 6.5, 20.0, 1e-3)
    t = time.perf_counter()
    _, _, sp = oracle.integrate([(1.0, 0.0)], s1, 0.01, 10000, nthreads=nthreads)
    dt = time.perf_counter() - t
    out["schwarzschild"] = gpu_ratio(
        {"value": float(sp.sum()) / dt, "unit": "lane-steps/s", "cores": nthreads, "kind": "oracle",
         "sample": "all 1,024 lanes x 10,000 steps (%.1f s wall)" % dt},
        result.get("schwarzschild", {}).get("value"))
    # camera: the 256 x 256 sub-grid of every 8th pixel per axis, full rays
    cam = {"M": 1.0, "a": 0.998, "r_obs": 1000.0, "incl": math.pi / 3, "half_width": 25.0,
           "nx": 2048, "ny": 2048, "h0": 0.1, "h_r0": 10.0, "r_escape": 1500.0,
           "horizon_factor": 1.01, "disk_r_in": -1.0, "disk_r_out": 30.0, "max_steps": 100000}
    ii, jj = np.meshgrid(np.arange(4, 2048, 8), np.arange(4, 2048, 8))
    pix = (jj * 2048 + ii).ravel().astype(np.int64)
    t = time.perf_counter()
    r3 = oracle.trace_camera(cam, pix, nthreads=nthreads)
    dt = time.perf_counter() - t
    cp = result.get("extra", {}).get("camera_persistent", {})
    out["camera"] = gpu_ratio(
        {"value": float(r3["steps"].sum()) / dt, "unit": "lane-steps/s", "cores": nthreads,
         "kind": "oracle", "rays_per_s": pix.size / dt,
         "sample": "256 x 256 pixels (every 8th per axis) of 2048 x 2048, full rays (%.1f s wall)" % dt},
        cp.get("lane_steps_per_s"))
    # 16 spins: 256 lanes per spin (contiguous from the start of each spin's block), FP64
    spins = [(1.0, 0.99 * k / 15) for k in range(16)]
    sol = np.repeat(np.arange(16), 256).astype(np.int32)
    s4 = np.concatenate([oracle.ic_constants(4, spins, 256, kr, st_of_lane=sol[k * 256:(k + 1) * 256],
                                             lane0=k * 262144)[1] for k in range(16)], axis=1)
    t = time.perf_counter()
    _, _, sp = oracle.integrate(spins, s4, 0.02, 20000, st_of_lane=sol, nthreads=nthreads)
    dt = time.perf_counter() - t
    mx = result.get("extra", {})
    out["mixed_16_spins"] = gpu_ratio(
        {"value": float(sp.sum()) / dt, "unit": "lane-steps/s", "cores": nthreads, "kind": "oracle",
         "sample": "16 spins x 256 lanes x 20,000 steps, FP64 (%.1f s wall)" % dt},
        mx.get("mixed_f64_persistent", {}).get("lane_steps_per_s"))
    if "mixed_f32k_persistent" in mx:
        out["mixed_16_spins"]["gpu_f32k_over_oracle"] = (
            mx["mixed_f32k_persistent"]["lane_steps_per_s"] / out["mixed_16_spins"]["value"])
    # adjoint: the oracle's complex-step gradient (five directions) of 256 lanes,
    # a = 0.7, 8,192 steps
    rc, s5, c5, _ = oracle.ic_constants(5, [(1.0, 0.7)], 256, kr)
    p5 = np.ascontiguousarray(np.stack([s5[1], s5[2], s5[5], s5[6], c5[1]]))
    tg = np.ascontiguousarray(np.stack([s5[1], s5[2], np.zeros(256)]) + 0.5)
    t = time.perf_counter()
    oracle.grad_ic(1.0, 0.7, 0.02, 8192, p5.reshape(-1), np.ascontiguousarray(c5[0]),
                   tg.reshape(-1), nthreads=nthreads)
    dt = time.perf_counter() - t
    out["adjoint"] = gpu_ratio(
        {"value": 256 * 8192 / dt, "unit": "gradient lane-steps/s", "cores": nthreads,
         "kind": "oracle (complex-step gradient, 5 directions)",
         "sample": "256 lanes x 8,192 steps (%.1f s wall)" % dt},
        mx.get("adjoint", {}).get("gradient_lane_steps_per_s"))
    return out


def extra_legs(m, torch, np):
    """One timed run (after a warm-up) of each remaining hot-path configuration."""
    out = {}
    # camera: a = 0.998, r_obs = 1000 M, i = 60 deg, 2048 x 2048 pixels over +-25 M
    from paper_1803_08320_amd import autotune
    cam_shape = autotune.camera_shape(m.Camera(nx=2048, ny=2048))
    for persistent in (1, 0):
        cam = m.Camera(nx=2048, ny=2048, persistent=persistent)
        res = {}

        def run_cam():
            res["o"] = m.trace_camera(cam)
        dt = _timed(torch, run_cam)
        st = res["o"]["status"]
        ls = int(res["o"]["steps"].sum().item())
        key = "camera_persistent" if persistent else "camera_plain"
        out[key] = {"lane_steps_per_s": ls / dt, "rays_per_s": st.numel() / dt, "ms": 1e3 * dt,
                    "status_counts": [int(x) for x in torch.bincount(st, minlength=6).cpu()]}
    out["camera_persistent"]["speedup_vs_plain"] = (out["camera_persistent"]["lane_steps_per_s"] /
                                                    out["camera_plain"]["lane_steps_per_s"])
    out["camera_persistent"]["launch_shape"] = {"block": cam_shape[0], "steps_per_chunk": cam_shape[1],
                                                "source": "autotuned"}

    # mixed-spin batch: 16 spins a_k = 0.99 k / 15 x 262,144 lanes, FP32 compensated state,
    # FP64 within 1.2 r_+, 20,000 steps; persistent refill vs one thread per lane, and FP64
    spins = [(1.0, 0.99 * k / 15) for k in range(16)]
    n = 16 * 262144
    sol = torch.arange(16, device="cuda", dtype=torch.int32).repeat_interleave(262144)
    s0, c0, _ = m.init_particles(m.ICSpec(mode=m.IC_CONSTANTS, seed=4), spins, n, st_of_lane=sol)
    state = torch.empty_like(s0)
    status, steps = m.new_lane_arrays(n)
    inv = torch.empty((4, n), dtype=torch.float64, device="cuda")
    for name, kw in (("mixed_f32k_persistent", dict(precision="f32k", persistent=True)),
                     ("mixed_f32k_plain", dict(precision="f32k", persistent=False)),
                     ("mixed_f64_persistent", dict(precision="f64", persistent=True)),
                     ("mixed_f64_plain", dict(precision="f64", persistent=False))):
        def run_mix():
            state.copy_(s0)
            status.zero_()
            steps.zero_()
            m.integrate(state, status, steps, spins, h=0.02, n_steps=20000, st_of_lane=sol,
                        fp64_zone_factor=1.2, **kw)
        dt = _timed(torch, run_mix)
        ls = int(steps.sum().item())
        out[name] = {"lane_steps_per_s": ls / dt, "ms": 1e3 * dt,
                     "plunged_frac": float((status == 1).float().mean().item())}
        if name == "mixed_f32k_persistent":
            # the same launch with the FP64 invariant monitor folded into the step loop
            # every 1,000 steps
            mon = torch.empty((8, n), dtype=torch.float64, device="cuda")

            def run_mon():
                state.copy_(s0)
                status.zero_()
                steps.zero_()
                m.integrate_monitored(state, status, steps, spins, 0.02, 20000, 1000, monitor=mon,
                                      st_of_lane=sol, precision="f32k", fp64_zone_factor=1.2,
                                      persistent=True)
            dtm = _timed(torch, run_mon)
            lsm = int(steps.sum().item())
            act_m = status == 0
            rel = (mon[4:] / mon[:4].abs().clamp_min(1e-300))
            q_ok_m = act_m & (mon[2] >= 0.1)
            out["mixed_f32k_persistent_monitored"] = {
                "lane_steps_per_s": lsm / dtm, "ms": 1e3 * dtm, "monitor_every": 1000,
                "max_dE_over_E_p99": float(torch.quantile(rel[0][act_m][:1 << 20], 0.99).item()),
                "max_dQ_over_Q_p99": float(torch.quantile(rel[2][q_ok_m][:1 << 20], 0.99).item())}
            # the monitored run leaves state, status and steps bitwise as the plain one
            m.invariants(state, spins, st_of_lane=sol, out=inv)
            act = (status == 0)
            q_ok = act & (c0[2] >= 0.1)
            dQ = ((inv[2] / c0[2] - 1).abs())[q_ok]
            dE = ((inv[0] / c0[0] - 1).abs())[act]
            out[name]["dQ_over_Q_p99"] = float(torch.quantile(dQ[:1 << 20], 0.99).item())
            out[name]["dE_over_E_p99"] = float(torch.quantile(dE[:1 << 20], 0.99).item())
    for prec in ("f32k", "f64"):
        out["mixed_%s_persistent" % prec]["speedup_vs_plain"] = (
            out["mixed_%s_persistent" % prec]["lane_steps_per_s"]
            / out["mixed_%s_plain" % prec]["lane_steps_per_s"])
    out["mixed_f32k_persistent"]["speedup_vs_f64_persistent"] = (
        out["mixed_f32k_persistent"]["lane_steps_per_s"] / out["mixed_f64_persistent"]["lane_steps_per_s"])
    # adjoint: a = 0.7, 65,536 lanes, 8,192 steps, checkpoints every 256
    st7 = (1.0, 0.7)
    n, N, K = 65536, 8192, 256
    y0, c7, _ = m.init_particles(m.ICSpec(mode=m.IC_CONSTANTS, seed=5), [st7], n)
    p = torch.stack([y0[1], y0[2], y0[5], y0[6], c7[1]]).contiguous().requires_grad_(True)
    E = c7[0].contiguous()
    tgt = torch.stack([y0[1], y0[2], torch.zeros_like(y0[1])]) + 0.5
    times = {}

    def fwd_bwd():
        p.grad = None
        a = time.perf_counter()
        yN, st_, sp_ = m.IntegrateFromParams.apply(p, E, st7, 0.02, N, K)
        loss = ((yN[1:4] - tgt) ** 2).sum()
        torch.cuda.synchronize()
        b = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        times["fwd"], times["bwd"] = b - a, time.perf_counter() - b
        times["ls"] = int(sp_.sum().item())
    fwd_bwd()
    fwd_bwd()
    out["adjoint"] = {"forward_ms": 1e3 * times["fwd"], "backward_ms": 1e3 * times["bwd"],
                      "backward_over_forward": times["bwd"] / times["fwd"],
                      "gradient_lane_steps_per_s": times["ls"] / (times["fwd"] + times["bwd"])}
    return out


if __name__ == "__main__":
    main()
