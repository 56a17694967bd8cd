"""GPU parity of the gridded 3+1 metric path (Section 2, eq. ADM; Hamilton's
equations, eq. Ham) against the oracle's own grid, interpolant and RK4."""
import math

import numpy as np
import pytest

from parity import compare, mixed_rel

pytestmark = pytest.mark.gpu

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))
GRID = dict(nr=401, nth=201, dr=60.0 / 400, th0=0.1, dth=(math.pi - 0.2) / 200)


def r_plus(a):
    return 1.0 + math.sqrt(1.0 - a * a)


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_08320_amd as m
    m.lib()
    return m


def to_dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def lower(orc, sts, s):
    z = s.copy()
    for i in range(s.shape[1]):
        z[4:, i] = orc.metric(*sts[0], s[1, i], s[2, i]) @ s[4:, i]
    return z


def gpu_grid_from(m, G, r_stop):
    import torch
    return m.Grid(to_dev(G.nodes, torch.float64), G.r0, G.dr, G.th0, G.dth, r_stop)


def f32_grids(orc, m, G, r_stop):
    """The oracle's grid with its node values rounded to single precision (the values a
    float-node grid stores): widened back to FP64 for the oracle, as float32 for the
    device."""
    import torch
    n32 = G.nodes.astype(np.float32)
    G32 = orc.Grid(n32.astype(np.float64), G.r0, G.dr, G.th0, G.dth)
    return G32, m.Grid(to_dev(n32, torch.float32), G.r0, G.dr, G.th0, G.dth, r_stop)


def assert_float_nodes(got, want64):
    """Float node values from the device fill: the oracle's FP64 values rounded to
    nearest, to within one unit in the float's last place (the device's and the
    oracle's FP64 values may lie on either side of a rounding boundary)."""
    assert got.dtype == np.float32
    want = want64.astype(np.float32)
    diff = np.abs(got.astype(np.float64) - want.astype(np.float64))
    assert np.all(diff <= np.spacing(np.abs(want)).astype(np.float64))
    assert (diff == 0).mean() > 0.999


def run_gpu(m, grid, z0, h, n_steps, r_escape, **kw):
    import torch
    n = z0.shape[1]
    state = to_dev(z0, torch.float64)
    status, steps = m.new_lane_arrays(n)
    m.integrate_grid(state, status, steps, grid, h, n_steps, r_escape, **kw)
    torch.cuda.synchronize()
    return state.cpu().numpy(), status.cpu().numpy(), steps.cpu().numpy()


def test_grid_fill_matches_oracle(m, orc):
    for a in (0.0, 0.9, 0.998):
        G = orc.grid_kerr(1.0, a, GRID["nr"], GRID["nth"], 2.1, GRID["dr"], GRID["th0"], GRID["dth"])
        g = m.grid_kerr(1.0, a, GRID["nr"], GRID["nth"], 2.1, GRID["dr"], GRID["th0"], GRID["dth"],
                        r_stop=2.5)
        got = g.nodes.cpu().numpy()
        assert np.max(np.abs(got - G.nodes) / (np.abs(G.nodes) + 1.0)) < 1e-14


def test_grid_fill_f32_matches_oracle(m, orc):
    import torch
    for a in (0.0, 0.9, 0.998):
        G = orc.grid_kerr(1.0, a, GRID["nr"], GRID["nth"], 2.1, GRID["dr"], GRID["th0"], GRID["dth"])
        g = m.grid_kerr(1.0, a, GRID["nr"], GRID["nth"], 2.1, GRID["dr"], GRID["th0"], GRID["dth"],
                        r_stop=2.5, node_dtype=torch.float32)
        assert_float_nodes(g.nodes.cpu().numpy(), G.nodes)


@pytest.mark.parametrize("a,n", [(0.9, 600), (0.0, 300)])
def test_grid_integration_parity_f32_nodes(m, orc, a, n):
    """Float node values: the kernel widens them on load, the oracle integrates on the
    same rounded values in FP64; several blocks and a ragged tail, 3,000 steps."""
    st = [(1.0, a)]
    r_stop = 1.2 * r_plus(a)
    G = orc.grid_kerr(1.0, a, r0=1.05 * r_plus(a), **GRID)
    G32, g32 = f32_grids(orc, m, G, r_stop)
    rc, s0, _, _ = orc.ic_constants(95, st, n, KERR_RANGES)
    z0 = lower(orc, st, s0)
    got = run_gpu(m, g32, z0, 0.02, 3000, 55.0)
    ref = orc.integrate_grid(G32, z0, 0.02, 3000, r_stop=r_stop, r_escape=55.0)
    compare(orc, st, z0, *got, *ref,
            lambda p0: orc.integrate_grid(G32, p0, 0.02, 3000, r_stop=r_stop, r_escape=55.0))
    assert np.array_equal(got[0][4], z0[4]) and np.array_equal(got[0][7], z0[7])


@pytest.mark.parametrize("a,n", [(0.9, 600), (0.0, 300)])
def test_grid_integration_parity(m, orc, a, n):
    """Several blocks and a ragged tail, 3,000 steps; the Schwarzschild draws plunge."""
    st = [(1.0, a)]
    # the grid starts just outside r_+ and the stencil of the stop radius stays on it
    r_stop = 1.2 * r_plus(a)
    G = orc.grid_kerr(1.0, a, r0=1.05 * r_plus(a), **GRID)
    rc, s0, _, _ = orc.ic_constants(91, st, n, KERR_RANGES)
    z0 = lower(orc, st, s0)
    got = run_gpu(m, gpu_grid_from(m, G, r_stop), z0, 0.02, 3000, 55.0)
    ref = orc.integrate_grid(G, z0, 0.02, 3000, r_stop=r_stop, r_escape=55.0)
    compare(orc, st, z0, *got, *ref,
            lambda p0: orc.integrate_grid(G, p0, 0.02, 3000, r_stop=r_stop, r_escape=55.0))
    if a == 0.0:
        assert (ref[1] == 1).sum() > 20
    assert np.array_equal(got[0][4], z0[4]) and np.array_equal(got[0][7], z0[7])


def test_off_grid_stops_and_chunking(m, orc):
    """A grid that covers only theta in [0.9, pi - 0.9] and r <= 30: lanes leaving it
    stop (NONFINITE, or ESCAPE at r_escape = 28) exactly where the oracle's do, and
    chunked launches give the same bits."""
    st = [(1.0, 0.7)]
    nth = 81
    G = orc.grid_kerr(1.0, 0.7, 301, nth, 1.5, 0.1, 0.9, (math.pi - 1.8) / (nth - 1))
    rc, s0, _, _ = orc.ic_constants(92, st, 500, ((5.0, 20.0),) + KERR_RANGES[1:])
    z0 = lower(orc, st, s0)
    ok = (z0[2] > 1.0) & (z0[2] < math.pi - 1.0)  # start inside the grid's interior
    z0 = np.ascontiguousarray(z0[:, ok])
    g = gpu_grid_from(m, G, 1.01 * r_plus(0.7))
    got = run_gpu(m, g, z0, 0.02, 4000, 28.0)
    ref = orc.integrate_grid(G, z0, 0.02, 4000, r_stop=g.r_stop, r_escape=28.0)
    assert (ref[1] == 4).sum() > 10
    compare(orc, st, z0, *got, *ref,
            lambda p0: orc.integrate_grid(G, p0, 0.02, 4000, r_stop=g.r_stop, r_escape=28.0))
    chunked = run_gpu(m, g, z0, 0.02, 4000, 28.0, steps_per_chunk=333)
    for x, y in zip(got, chunked):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("node_dtype", ["float64", "float32"])
def test_gridded_kerr_tracks_analytic_kerr(m, orc, node_dtype):
    """The same orbits in the gridded and in the analytic metric (Hamiltonian form):
    differences at the interpolation-error level, with node values stored in double
    or in single precision."""
    import torch
    st = [(1.0, 0.9)]
    rc, s0, _, _ = orc.ic_constants(93, st, 256, ((6.0, 20.0),) + KERR_RANGES[1:])
    z0 = lower(orc, st, s0)
    g = m.grid_kerr(1.0, 0.9, 801, 401, 1.5, 60.0 / 800, 0.1, (math.pi - 0.2) / 400,
                    1.2 * r_plus(0.9), node_dtype=getattr(torch, node_dtype))
    got = run_gpu(m, g, z0, 0.02, 2000, 55.0)
    x = to_dev(z0, torch.float64)
    status, steps = m.new_lane_arrays(256)
    m.integrate(x, status, steps, st, h=0.02, n_steps=2000, formulation="hamiltonian")
    ana = x.cpu().numpy()
    both = (got[1] == 0) & (status.cpu().numpy() == 0)
    assert both.mean() > 0.95
    assert mixed_rel(got[0][:, both], ana[:, both]).max() < 1e-4


@pytest.mark.parametrize("node_dtype", ["float64", "float32"])
def test_grid_full_size_sampled(m, orc, node_dtype):
    """The benchmark's gridded launches: 1,048,576 Kerr a = 0.9 lanes x 2,000 steps on
    an 801 x 401 grid filled on the device (all nodes checked against the oracle's
    fill), node values in double or in single precision; 256 strided lanes hold the
    oracle's initial data and are compared with the oracle's integration on its own
    grid (for float nodes: its values rounded to float, which the device grid then
    holds too)."""
    import torch
    from parity import mixed_rel
    st = [(1.0, 0.9)]
    n = 1 << 20
    geo = (1.0, 0.9, 801, 401, 1.5, 60.0 / 800, 0.1, (math.pi - 0.2) / 400)
    r_stop = 1.2 * r_plus(0.9)
    g = m.grid_kerr(*geo, r_stop, node_dtype=getattr(torch, node_dtype))
    G = orc.grid_kerr(*geo)
    got_nodes = g.nodes.cpu().numpy()
    if node_dtype == "float64":
        assert np.max(np.abs(got_nodes - G.nodes) / (np.abs(G.nodes) + 1.0)) < 1e-14
    else:
        assert_float_nodes(got_nodes, G.nodes)
        G, g = f32_grids(orc, m, G, r_stop)
    del got_nodes
    spec = m.ICSpec(mode=m.IC_CONSTANTS, seed=2, r_range=KERR_RANGES[0], th_range=KERR_RANGES[1],
                    E_range=KERR_RANGES[2], Lz_range=KERR_RANGES[3], Q_range=KERR_RANGES[4])
    state, _, _ = m.init_particles(spec, st, n)
    m.convert_state(state, st, True)
    idx = np.arange(0, n, n // 256)
    s0 = np.concatenate([orc.ic_constants(2, st, 1, KERR_RANGES, lane0=int(i))[1] for i in idx], axis=1)
    z0 = lower(orc, st, s0)
    assert mixed_rel(state.cpu().numpy()[:, idx], z0).max() < 5e-13
    state[:, torch.as_tensor(idx, device="cuda")] = to_dev(z0, torch.float64)
    status, steps = m.new_lane_arrays(n)
    m.integrate_grid(state, status, steps, g, 0.02, 2000, 55.0)
    torch.cuda.synchronize()
    got = (state.cpu().numpy()[:, idx], status.cpu().numpy()[idx], steps.cpu().numpy()[idx])
    ref = orc.integrate_grid(G, z0, 0.02, 2000, r_stop=r_stop, r_escape=55.0)
    compare(orc, st, z0, *got, *ref,
            lambda p0: orc.integrate_grid(G, p0, 0.02, 2000, r_stop=r_stop, r_escape=55.0))
    assert (status == 0).float().mean().item() > 0.99


@pytest.mark.parametrize("node_dtype", ["float64", "float32"])
def test_stencil_cache_block_sizes_and_chunks_same_bits(m, orc, node_dtype):
    """Each lane's LDS stencil cache is indexed by its thread in the block and starts
    empty in every launch: blocks of 64, 128 and 256 lanes and launch-chunked runs give
    the same bits (a ragged batch of 1,000 lanes that cross many cells in 3,000 steps)."""
    import torch
    st = [(1.0, 0.9)]
    rc, s0, _, _ = orc.ic_constants(96, st, 1000, KERR_RANGES)
    z0 = lower(orc, st, s0)
    g = m.grid_kerr(1.0, 0.9, 401, 201, 1.5, 60.0 / 400, 0.1, (math.pi - 0.2) / 200,
                    1.2 * r_plus(0.9), node_dtype=getattr(torch, node_dtype))
    ref = run_gpu(m, g, z0, 0.02, 3000, 55.0)
    assert (ref[1] == 0).mean() > 0.9
    for kw in (dict(block=64), dict(block=128), dict(steps_per_chunk=701)):
        got = run_gpu(m, g, z0, 0.02, 3000, 55.0, **kw)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), kw
