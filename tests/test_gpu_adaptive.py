"""GPU parity of the adaptive Dormand-Prince 5(4) integrator against the oracle's
(same pair, same controller, same stop rules)."""
import math

import numpy as np
import pytest

from parity import compare

pytestmark = pytest.mark.gpu

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))
CTL = dict(rtol=1e-9, atol=1e-9, fac=0.9, facmin=0.2, facmax=5.0)


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


def run_gpu(m, sts, s0, tau_end, h0, st_of_lane=None, **kw):
    import torch
    n = s0.shape[1]
    state = to_dev(s0, torch.float64)
    tau = torch.zeros(n, dtype=torch.float64, device="cuda")
    h = torch.full((n,), h0, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    steps = torch.zeros(n, dtype=torch.int32, device="cuda")
    rej = torch.zeros(n, dtype=torch.int32, device="cuda")
    sol = None if st_of_lane is None else to_dev(st_of_lane, torch.int32)
    args = dict(CTL)
    args.update(kw)
    m.integrate_adaptive(state, tau, h, status, steps, rej, sts, tau_end, st_of_lane=sol, **args)
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in (state, tau, h, status, steps, rej))


def key(steps, rej):
    """Accepted and rejected attempt counts as one integer (both must match)."""
    return steps.astype(np.int64) * 65536 + rej


def oracle(orc, sts, s0, tau_end, h0, **kw):
    args = dict(CTL)
    args.update(kw)
    return orc.integrate_adaptive(sts, s0, tau_end, h0, **args)


def check(orc, sts, s0, got, ref, tau_end, h0, **kw):
    """State, status and attempt counts per lane against the oracle, with the
    conditioning guard of parity.compare (an accept/reject decision taken at
    err ~ 1 can go either way under a change of rounding).  A lane that both sides
    stop as HORIZON ends next to the coordinate singularity at r_+ (u^t ~ 1/Delta;
    a 1-ulp change of r0 moves its final state by ~1e-8 in the oracle itself), so
    for those the status and the attempt counts are the comparison."""
    def rerun(p0):
        y, tau, h, st, sp, rj = oracle(orc, sts, p0, tau_end, h0, **kw)
        return y, st, key(sp, rj)
    both_hz = (got[3] == 1) & (ref[3] == 1)
    g0 = np.where(both_hz[None, :], ref[0], got[0])
    stats = compare(orc, sts, s0, g0, got[3], key(got[4], got[5]), ref[0], ref[3],
                    key(ref[4], ref[5]), rerun)
    same = (got[3] == ref[3]) & (got[4] == ref[4]) & (got[5] == ref[5])
    # the affine parameter lands exactly on tau_end for lanes still active
    act = same & (ref[3] == 0)
    assert np.array_equal(got[1][act], ref[1][act]) and np.all(ref[1][act] == tau_end)
    # h on return is the step suggested after the last accepted step, and that step is
    # clipped to tau_end - tau_prev.  Every step size follows err^(-1/5) of an
    # embedded difference whose rounding floor is ~1e-4 of its tolerance at rtol =
    # 1e-12, so the two sides' steps differ by up to a few 1e-5 relative and their sums
    # tau_prev by up to ~1.5e-5 tau_prev (both measured without clipping in
    # test_adaptive_full_size_sampled); the clipped step carries that difference
    # absolute, and the suggestion is at most facmax times the clipped step.  The
    # state, tau and the attempt counts above already fix every accept/reject decision
    # exactly.
    facmax = kw.get("facmax", CTL["facmax"])
    dh = np.abs(got[2][same] - ref[2][same])
    print("final h: max |dh| %.3e, max |dh|/h %.3e, median |dh|/h %.3e"
          % (dh.max(), (dh / np.abs(ref[2][same])).max(), np.median(dh / np.abs(ref[2][same]))))
    assert np.all(dh <= 1e-3 * np.abs(ref[2][same]) + facmax * 3e-5 * tau_end)
    assert np.median(dh / np.abs(ref[2][same])) <= 1e-4
    return stats


@pytest.mark.parametrize("persistent", [False, True])
def test_adaptive_parity_kerr(m, orc, persistent):
    st = [(1.0, 0.9)]
    rc, s0, _, _ = orc.ic_constants(71, st, 600, KERR_RANGES)
    got = run_gpu(m, st, s0, 300.0, 0.1, persistent=persistent)
    ref = oracle(orc, st, s0, 300.0, 0.1)
    assert ref[5].sum() > 0  # the controller rejects some attempts
    check(orc, st, s0, got, ref, 300.0, 0.1)


def test_adaptive_plunging_and_mixed_spins(m, orc):
    sts = [(1.0, 0.0), (1.0, 0.5), (1.0, 0.998)]
    n = 900
    st_of_lane = (np.arange(n) % 3).astype(np.int32)
    rc, s0, _, _ = orc.ic_constants(72, sts, n, KERR_RANGES, st_of_lane=st_of_lane)
    got = run_gpu(m, sts, s0, 2000.0, 0.05, st_of_lane=st_of_lane)
    for k in range(3):
        sel = np.flatnonzero(st_of_lane == k)
        ref = oracle(orc, [sts[k]], s0[:, sel], 2000.0, 0.05)
        sub = tuple(x[..., sel] for x in got)
        check(orc, [sts[k]], s0[:, sel], sub, ref, 2000.0, 0.05)
        if k == 0:
            assert (ref[3] == 1).sum() > 30  # Schwarzschild draws plunge


def test_persistent_equals_plain_bitwise_and_budget(m, orc):
    st = [(1.0, 0.7)]
    rc, s0, _, _ = orc.ic_constants(73, st, 1000, KERR_RANGES)
    a = run_gpu(m, st, s0, 500.0, 0.1, persistent=False)
    b = run_gpu(m, st, s0, 500.0, 0.1, persistent=True, steps_per_chunk=3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    c = run_gpu(m, st, s0, 1e6, 0.1, max_attempts=7)
    assert np.all(c[3] == 5) and np.all(c[4] + c[5] == 7)
    ref = oracle(orc, st, s0, 1e6, 0.1, max_attempts=7)
    assert np.array_equal(ref[3], c[3])


def test_adaptive_full_size_sampled(m, orc):
    """The benchmark's adaptive launch: Kerr a = 0.9, 1,048,576 lanes to tau = 400 at
    rtol = atol = 1e-12 under the persistent queue.  256 strided lanes hold the
    oracle's own initial data (the device builder's agree with it to the rounding of
    sqrt(R)) and are compared with the oracle; over all lanes, active ones end on
    tau_end."""
    import torch
    from parity import mixed_rel
    st = [(1.0, 0.9)]
    n = 1 << 20
    spec = m.ICSpec(mode=m.IC_CONSTANTS, seed=2, r_range=KERR_RANGES[0], th_range=KERR_RANGES[1],
                    E_range=KERR_RANGES[2], Lz_range=KERR_RANGES[3], Q_range=KERR_RANGES[4])
    state, consts, _ = m.init_particles(spec, st, n)
    idx = np.arange(0, n, n // 256)
    s0 = np.concatenate([orc.ic_constants(2, st, 1, KERR_RANGES, lane0=int(i))[1] for i in idx], axis=1)
    assert mixed_rel(state.cpu().numpy()[:, idx], s0).max() < 5e-13
    state[:, torch.as_tensor(idx, device="cuda")] = to_dev(s0, torch.float64)
    tau = torch.zeros(n, dtype=torch.float64, device="cuda")
    h = torch.full((n,), 0.1, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    steps = torch.zeros(n, dtype=torch.int32, device="cuda")
    rej = torch.zeros(n, dtype=torch.int32, device="cuda")
    m.integrate_adaptive(state, tau, h, status, steps, rej, st, 400.0, rtol=1e-12, atol=1e-12,
                         persistent=True)
    torch.cuda.synchronize()
    all_out = tuple(x.cpu().numpy() for x in (state, tau, h, status, steps, rej))
    got = tuple(x[..., idx] for x in all_out)
    kw = dict(rtol=1e-12, atol=1e-12)
    ref = oracle(orc, st, s0, 400.0, 0.1, **kw)
    check(orc, st, s0, got, ref, 400.0, 0.1, **kw)
    act = all_out[3] == 0
    assert act.mean() > 0.99 and np.all(all_out[1][act] == 400.0)
    # the same lanes without the clipped last step: a fixed budget of attempts towards a
    # distant tau_end (every lane ends as BUDGET); the step sizes and their sum tau
    # agree to the rounding floor of the error estimate
    x = to_dev(s0, torch.float64)
    k = s0.shape[1]
    tau = torch.zeros(k, dtype=torch.float64, device="cuda")
    h = torch.full((k,), 0.1, dtype=torch.float64, device="cuda")
    z = [torch.zeros(k, dtype=torch.int32, device="cuda") for _ in range(3)]
    m.integrate_adaptive(x, tau, h, z[0], z[1], z[2], st, 1e6, max_attempts=400, **kw)
    torch.cuda.synchronize()
    g = [t.cpu().numpy() for t in (tau, h, z[0], z[1], z[2])]
    ref = oracle(orc, st, s0, 1e6, 0.1, max_attempts=400, **kw)
    assert np.array_equal(g[2], ref[3])
    assert np.array_equal(g[3], ref[4]) and np.array_equal(g[4], ref[5])
    bud = ref[3] == 5
    assert bud.mean() > 0.95
    assert np.all(np.abs(g[0] - ref[1])[bud] <= 3e-5 * ref[1][bud])
    assert np.all(np.abs(g[1] - ref[2])[bud] <= 1e-3 * ref[2][bud])
    assert np.median(np.abs(g[0] - ref[1])[bud] / ref[1][bud]) <= 1e-6
