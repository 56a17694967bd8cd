"""Discrete adjoint on the GPU against the oracle's complex-step gradient (parity
unpinned by the paper, which prints no gradient; the oracle's gradient is itself
pinned by central differences in test_oracle_grad.py)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))
ST = (1.0, 0.7)


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_08320_amd as m
    m.lib()
    return m


def params(orc, seed, n, lane0=0):
    rc, s, c, _ = orc.ic_constants(seed, [ST], n, KERR_RANGES, lane0=lane0)
    assert rc == 0
    p = np.stack([s[1], s[2], s[5], s[6], c[1]])
    return np.ascontiguousarray(p), np.ascontiguousarray(c[0])


def targets_for(orc, p, E, h, N, seed):
    rng = np.random.default_rng(seed)
    n = p.shape[1]
    y0 = np.stack([orc.ic_map(ST[0], ST[1], E[i], p[:, i]) for i in range(n)], axis=1)
    yN, _, _ = orc.integrate([ST], y0, h, N)
    return np.ascontiguousarray(yN[1:4] + rng.uniform(-1, 1, size=(3, n)))


def gpu_grad(m, p, E, tgt, h, N, K):
    import torch
    pt = torch.tensor(p, device="cuda", requires_grad=True)
    Et = torch.tensor(E, device="cuda")
    tg = torch.tensor(tgt, device="cuda")
    yN, status, steps = m.IntegrateFromParams.apply(pt, Et, ST, h, N, K)
    loss = ((yN[1:4] - tg) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return pt.grad.cpu().numpy(), status.cpu().numpy(), yN.detach().cpu().numpy()


def test_gradient_matches_oracle_complex_step(m, orc):
    n, h, N, K = 257, 0.02, 512, 64
    p, E = params(orc, 5, n)
    tgt = targets_for(orc, p, E, h, N, 1)
    g, status, _ = gpu_grad(m, p, E, tgt, h, N, K)
    ref, _ = orc.grad_ic(ST[0], ST[1], h, N, p.reshape(-1), E, tgt.reshape(-1))
    act = status == 0
    assert act.mean() > 0.95
    err = np.abs(g - ref) / (np.abs(ref) + 1e-3 * np.abs(ref).max(axis=0))
    assert np.median(err[:, act]) < 1e-12
    assert err[:, act].max() < 1e-9, err[:, act].max()


def test_checkpoint_interval_does_not_change_the_gradient(m, orc):
    n, h, N = 100, 0.02, 300
    p, E = params(orc, 6, n)
    tgt = targets_for(orc, p, E, h, N, 2)
    g1, _, y1 = gpu_grad(m, p, E, tgt, h, N, 32)
    g2, _, y2 = gpu_grad(m, p, E, tgt, h, N, 128)
    g3, _, y3 = gpu_grad(m, p, E, tgt, h, N, 300)
    assert np.array_equal(y1, y2) and np.array_equal(y1, y3)
    assert np.array_equal(g1, g2) and np.array_equal(g1, g3)


def test_transposed_tangent_identity(m, orc):
    """<g_initial, v> = <g_final, J v> with J v from the oracle's complex-step tangent."""
    import torch
    n, h, N, K = 16, 0.02, 400, 50
    rc, s0, _, _ = orc.ic_constants(7, [ST], n, KERR_RANGES)
    rng = np.random.default_rng(3)
    gf = rng.normal(size=(8, n))
    v = rng.normal(size=(8, n))
    state = torch.tensor(s0, device="cuda")
    status, steps = m.new_lane_arrays(n)
    ck = torch.empty((N // K + 1, 8, n), dtype=torch.float64, device="cuda")
    m.integrate(state, status, steps, [ST], h=h, n_steps=N, checkpoints=ck, checkpoint_every=K)
    gi, _ = m.adjoint(ck, status, steps, torch.tensor(gf, device="cuda"), [ST], h, N, K, named=False)
    gi = gi.cpu().numpy()
    assert np.all(status.cpu().numpy() == 0)
    for i in range(n):
        _, jv = orc.tangent(ST[0], ST[1], h, N, s0[:, i], v[:, i])
        lhs = float(gi[:, i] @ v[:, i])
        rhs = float(gf[:, i] @ jv)
        # both sides are the same discrete map's transpose and tangent: they agree to
        # rounding (3e-15 of the sum of the terms' magnitudes measured)
        assert abs(lhs - rhs) <= 1e-12 * np.abs(gf[:, i] * jv).sum()


def test_gradient_matches_gpu_central_differences(m, orc):
    import torch
    n, h, N, K = 8, 0.02, 256, 64
    p, E = params(orc, 8, n)
    tgt = targets_for(orc, p, E, h, N, 4)
    g, status, _ = gpu_grad(m, p, E, tgt, h, N, K)

    def loss(pp):
        with torch.no_grad():
            yN, st, _ = m.IntegrateFromParams.apply(torch.tensor(pp, device="cuda"),
                                                    torch.tensor(E, device="cuda"), ST, h, N, K)
            return (((yN[1:4] - torch.tensor(tgt, device="cuda")) ** 2).sum(dim=0)).cpu().numpy()

    for j in range(5):
        e = np.zeros_like(p)
        e[j] = 1e-6
        fd = (loss(p + e) - loss(p - e)) / 2e-6
        assert np.allclose(g[j], fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max()), (j, g[j], fd)


def test_stopped_lanes_give_finite_gradients(m, orc):
    import torch
    n, h, N, K = 64, 0.02, 400, 64
    p, E = params(orc, 9, n)
    p[0, :8] = 1.6   # start inside the stop radius of a = 0.7 (1.01 r_+ = 1.7297)
    tgt = np.zeros((3, n))
    g, status, _ = gpu_grad(m, p, E, tgt, h, N, K)
    assert np.all(status[:8] == 1)
    assert np.all(np.isfinite(g))
    # a lane that stopped at its first step keeps only the identity: dL/dr0 = 2 (r0 - 0)
    assert np.allclose(g[0, :8], 2 * p[0, :8], rtol=1e-12)


def test_full_size_adjoint_sampled(m, orc):
    """Kerr a = 0.7, 65,536 lanes, 8,192 steps, checkpoints every 256 steps: gradients
    of 256 strided lanes against the oracle's complex-step gradient (measured: median
    error 3e-14, largest 1.1e-11)."""
    n, h, N, K = 65536, 0.02, 8192, 256
    p, E = params(orc, 5, n)
    idx = np.arange(0, n, n // 256)
    rng = np.random.default_rng(11)
    tgt = np.ascontiguousarray(p[:3] * 0 + rng.uniform(-1, 1, size=(3, n)) + np.array([[20.0], [1.5], [0.0]]))
    g, status, _ = gpu_grad(m, p, E, tgt, h, N, K)
    ref, _ = orc.grad_ic(ST[0], ST[1], h, N, np.ascontiguousarray(p[:, idx]).reshape(-1),
                         np.ascontiguousarray(E[idx]), np.ascontiguousarray(tgt[:, idx]).reshape(-1))
    act = status[idx] == 0
    err = np.abs(g[:, idx] - ref) / (np.abs(ref) + 1e-3 * np.abs(ref).max(axis=0))
    assert act.mean() > 0.9
    print("adjoint full size: %d lanes, median error %.2e, largest %.2e" % (
        act.sum(), np.median(err[:, act]), err[:, act].max()))
    assert np.median(err[:, act]) < 1e-12
    assert err[:, act].max() < 1e-9
