"""HIP graph capture of the launch sequences (torch.cuda.CUDAGraph is hipGraph on
ROCm).  Every replay, with eager work and synchronisation in between, must equal
the eager result bit for bit, and the replayed results are compared with the oracle;
the camera's work counter is cleared by a kernel, not a memset node, so replays after
the first see a fresh queue."""
import math

import numpy as np
import pytest

from parity import compare

pytestmark = pytest.mark.gpu

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_08320_amd as m
    m.lib()
    return m


def test_integrate_graph_replays(m, orc):
    import torch
    st = [(1.0, 0.9)]
    n = 5000
    rc, s0h, _, _ = orc.ic_constants(2, st, n, KERR_RANGES)
    s0 = torch.as_tensor(s0h).cuda()
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
    # the replayed result against the oracle
    g.replay()
    torch.cuda.synchronize()
    ref = orc.integrate(st, s0h, 0.02, 300)
    compare(orc, st, s0h, state.cpu().numpy(), status.cpu().numpy(), steps.cpu().numpy(), *ref,
            lambda p0: orc.integrate(st, p0, 0.02, 300), label="hipGraph replay of integrate")


def test_camera_graph_replays(m, orc):
    import torch
    from test_gpu_camera import check_against_oracle
    cam = m.Camera(nx=96, ny=64, block=256, steps_per_chunk=32)
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
    g.replay()
    torch.cuda.synchronize()
    check_against_oracle(orc, cam, {k: v.cpu().numpy() for k, v in out.items()},
                         np.arange(cam.nx * cam.ny), "hipGraph replay of the camera, 96 x 64")


def test_autotuner_shapes_are_cached_and_used_by_block_zero(m, tmp_path, monkeypatch):
    """The tuner picks a candidate shape per kind of launch (plain: block; persistent:
    block and refill interval), caches it under a key that holds the precision,
    formulation, persistence and spacetime count, and the binding's block = 0 takes the
    cached shape; no launch shape changes the results."""
    import torch
    from paper_1803_08320_amd import autotune
    monkeypatch.setenv("MALBEC_TUNE_CACHE", str(tmp_path / "tune.json"))
    st = [(1.0, 0.9)]
    n = 20000
    s0, _, _ = m.init_particles(m.ICSpec(mode=m.IC_CONSTANTS, seed=2), st, n)
    assert autotune.lookup_integrate(n, 1) is None
    blk, ch = autotune.integrate_shape(s0, st, 0.02, probe_steps=50)
    assert blk in autotune.BLOCKS and ch == 0
    assert autotune.lookup_integrate(n, 1) == (blk, 0)
    pb, pc = autotune.integrate_shape(s0, st, 0.02, persistent=True, probe_steps=50)
    assert pb in autotune.BLOCKS and pc in autotune.CHUNKS
    assert autotune.lookup_integrate(n, 1, persistent=True) == (pb, pc)
    assert autotune.lookup_integrate(n, 1, precision="f32k") is None
    assert autotune.lookup_integrate(n, 1, formulation="hamiltonian") is None
    # a mixed-spin batch: its own entry, tuned with the sample's own spacetime indices
    sts = [(1.0, 0.0), (1.0, 0.5), (1.0, 0.99)]
    sol = torch.as_tensor(np.arange(n) % 3, dtype=torch.int32).cuda()
    mb = autotune.integrate_shape(s0, sts, 0.02, st_of_lane=sol, probe_steps=50)
    assert autotune.lookup_integrate(n, 3) == mb
    outs = []
    for kw in (dict(block=64), dict(block=0), dict(block=0, persistent=True),
               dict(block=128, persistent=True, steps_per_chunk=8)):
        state = s0.clone()
        status, steps = m.new_lane_arrays(n)
        m.integrate(state, status, steps, st, h=0.02, n_steps=100, **kw)
        outs.append((state, status, steps))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert torch.equal(x, y)
    cam = m.Camera(nx=128, ny=128)
    shape = autotune.camera_shape(cam, sample=64)
    assert shape[0] in autotune.BLOCKS and shape[1] in autotune.CHUNKS
    assert autotune.lookup_camera(cam) == shape
    a = m.trace_camera(cam, final_state=True)
    b = m.trace_camera(m.Camera(nx=128, ny=128, block=64, steps_per_chunk=128), final_state=True)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(torch.nan_to_num(a[k]), torch.nan_to_num(b[k])), k
