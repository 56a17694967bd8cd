"""The adaptive integrator's no-allocation entry point (malbec_integrate_adaptive_noalloc,
static scratch) against the entry point with a caller workspace: identical results on
two calls in a row, the second with a smaller batch, other initial conditions and mixed
spins, so that stale scratch contents from the first call would show."""
import math

import numpy as np
import pytest

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


def initial(m, sts, n, seed, st_of_lane=None):
    spec = m.ICSpec(mode=m.IC_CONSTANTS, seed=seed, r_range=KERR_RANGES[0],
                    th_range=KERR_RANGES[1], E_range=KERR_RANGES[2], Lz_range=KERR_RANGES[3],
                    Q_range=KERR_RANGES[4])
    state, _, _ = m.init_particles(spec, sts, n, st_of_lane=st_of_lane)
    return state


def run(m, fn, state0, sts, tau_end, st_of_lane, persistent, schedule):
    import torch
    n = state0.shape[1]
    state = state0.clone()
    tau = torch.zeros(n, dtype=torch.float64, device="cuda")
    h = torch.full((n,), 0.05, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    steps = torch.zeros(n, dtype=torch.int32, device="cuda")
    rej = torch.zeros(n, dtype=torch.int32, device="cuda")
    fn(state, tau, h, status, steps, rej, sts, tau_end, rtol=1e-10, atol=1e-10,
       st_of_lane=st_of_lane, persistent=persistent, schedule=schedule)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (state, tau, h, status, steps, rej)]


@pytest.mark.parametrize("persistent,schedule", [(True, "periapsis"), (True, "index"),
                                                 (False, "index")])
def test_noalloc_equals_workspace_call_on_two_calls(m, persistent, schedule):
    import torch
    cases = [
        # first call: one spin, the larger batch
        ([(1.0, 0.9)], 150_000, 21, False),
        # second call: smaller batch, three spins mixed lane by lane, other draws
        ([(1.0, 0.0), (1.0, 0.7), (1.0, 0.99)], 40_003, 22, True),
    ]
    for sts, n, seed, mix in cases:
        sol = None
        if mix:
            sol = torch.as_tensor(np.arange(n) % len(sts), dtype=torch.int32).cuda()
        print("noalloc persistent=%d schedule=%s n=%d seed=%d" % (persistent, schedule, n, seed),
              flush=True)
        s0 = initial(m, sts, n, seed, sol)
        ref = run(m, m.integrate_adaptive, s0, sts, 60.0, sol, persistent, schedule)
        got = run(m, m.integrate_adaptive_noalloc, s0, sts, 60.0, sol, persistent, schedule)
        print("  %d lanes still active, %d accepted attempts" %
              (int((got[3] == 0).sum()), int(got[4].sum())), flush=True)
        for name, a, b in zip(("state", "tau", "h", "status", "steps", "rejects"), got, ref):
            assert np.array_equal(a, b, equal_nan=True), "%s differs (n=%d)" % (name, n)
        assert got[4].sum() > 10 * n  # the lanes did integrate


def test_noalloc_rejects_batches_above_its_scratch(m):
    import torch
    n = m.NOALLOC_MAX_LANES + 1
    z = torch.zeros(8 * n, dtype=torch.float64, device="cuda")
    zi = torch.zeros(n, dtype=torch.int32, device="cuda")
    zd = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(m.MalbecError) as e:
        m.integrate_adaptive_noalloc(z.view(8, n), zd, zd.clone(), zi, zi.clone(), zi.clone(),
                                     [(1.0, 0.9)], 1.0)
    assert e.value.code == -1 and "no-allocation scratch" in str(e.value)
