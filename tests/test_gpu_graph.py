"""HIP graph capture of the launch sequences (torch.cuda.CUDAGraph is hipGraph on
ROCm).  Every replay, with eager work and synchronisation in between, must equal
the eager result bit for bit; the camera's work counter is cleared by a kernel,
not a memset node, so replays after the first see a fresh queue."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_08320_amd as m
    m.lib()
    return m


def test_integrate_graph_replays(m):
    import torch
    st = [(1.0, 0.9)]
    n = 5000
    s0, _, _ = m.init_particles(m.ICSpec(mode=m.IC_CONSTANTS, seed=2), st, n)
    state = torch.empty_like(s0)
    status, steps = m.new_lane_arrays(n)

    def run():
        state.copy_(s0)
        status.zero_()
        steps.zero_()
        m.integrate(state, status, steps, st, h=0.02, n_steps=300)

    run()
    torch.cuda.synchronize()
    want = (state.clone(), status.clone(), steps.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        state.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(state, want[0]), rep
        assert torch.equal(status, want[1]) and torch.equal(steps, want[2]), rep
        # eager work between replays
        run()
        torch.cuda.synchronize()
        assert torch.equal(state, want[0])


def test_camera_graph_replays(m):
    import torch
    cam = m.Camera(nx=96, ny=64)
    ref = m.trace_camera(cam, final_state=True)
    torch.cuda.synchronize()
    want = {k: v.clone() for k, v in ref.items()}
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    ws = torch.empty(m.workspace_bytes(m.OP_CAMERA, cam.nx * cam.ny), dtype=torch.uint8,
                     device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        m.trace_camera(cam, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.trace_camera(cam, out=out, ws=ws)
    for rep in range(3):
        for v in out.values():
            v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in want:
            assert torch.equal(torch.nan_to_num(out[k]), torch.nan_to_num(want[k])), (rep, k)
        m.trace_camera(cam, out=out, ws=ws)  # eager between replays
        torch.cuda.synchronize()


def test_autotuner_picks_a_candidate_and_shape_does_not_change_results(m, tmp_path, monkeypatch):
    import torch
    from paper_1803_08320_amd import autotune
    monkeypatch.setenv("MALBEC_TUNE_CACHE", str(tmp_path / "tune.json"))
    st = [(1.0, 0.9)]
    s0, _, _ = m.init_particles(m.ICSpec(mode=m.IC_CONSTANTS, seed=2), st, 20000)
    blk = autotune.integrate_block(s0, st, 0.02, probe_steps=50)
    assert blk in autotune.BLOCKS
    assert autotune.integrate_block(s0, st, 0.02) == blk  # cached
    outs = []
    for b in (64, blk):
        state = s0.clone()
        status, steps = m.new_lane_arrays(20000)
        m.integrate(state, status, steps, st, h=0.02, n_steps=100, block=b)
        outs.append(state)
    assert torch.equal(outs[0], outs[1])
    cam = m.Camera(nx=128, ny=128)
    shape = autotune.camera_shape(cam, sample=64)
    assert shape[0] in autotune.BLOCKS and shape[1] in autotune.CHUNKS
