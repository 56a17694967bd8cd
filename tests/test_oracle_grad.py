"""Pins of the oracle's gradient of the discrete RK4 map (complex-step tangents).

The paper prints no gradient: gradient parity is unpinned by the paper.  The
complex-step derivative is pinned here by central finite differences
(eps = 1e-6), by linearity of the tangent map, and by the RK4-of-the-variational
equation identity for the t and phi shift symmetries.
"""
import math

import numpy as np
import pytest

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))


@pytest.fixture(scope="module")
def lanes(orc):
    rc, s, c, _ = orc.ic_constants(5, [(1.0, 0.7)], 6, KERR_RANGES)
    assert rc == 0
    p = np.stack([s[1], s[2], s[5], s[6], c[1]])  # r0, th0, u^r0, u^th0, L_z
    return p, c[0].copy()


def test_ic_map_reproduces_state(orc, lanes):
    p, E = lanes
    rc, s, c, _ = orc.ic_constants(5, [(1.0, 0.7)], 6, KERR_RANGES)
    for i in range(p.shape[1]):
        y = orc.ic_map(1.0, 0.7, E[i], p[:, i])
        assert np.allclose(y, s[:, i], rtol=1e-12, atol=1e-14)


def test_complex_step_gradient_matches_central_differences(orc, lanes):
    p, E = lanes
    n_steps, h = 512, 0.02
    rng = np.random.default_rng(7)
    targets = np.zeros((3, p.shape[1]))
    for i in range(p.shape[1]):
        y = orc.ic_map(1.0, 0.7, E[i], p[:, i])
        ys, _, _ = orc.integrate([(1.0, 0.7)], y.reshape(8, 1), h, n_steps)
        targets[:, i] = ys[1:4, 0] + rng.uniform(-1, 1, 3)
    grad, loss = orc.grad_ic(1.0, 0.7, h, n_steps, p.reshape(-1), E, targets.reshape(-1))
    for i in range(p.shape[1]):
        L0 = orc.loss_ic(1.0, 0.7, h, n_steps, p[:, i], E[i], targets[:, i])
        assert L0 == pytest.approx(loss[i], rel=1e-14)
        for j in range(5):
            e = np.zeros(5)
            e[j] = 1e-6
            fd = (orc.loss_ic(1.0, 0.7, h, n_steps, p[:, i] + e, E[i], targets[:, i])
                  - orc.loss_ic(1.0, 0.7, h, n_steps, p[:, i] - e, E[i], targets[:, i])) / 2e-6
            assert grad[j, i] == pytest.approx(fd, rel=1e-5, abs=1e-7 * max(1.0, loss[i])), (i, j)


def test_tangent_is_linear(orc, lanes):
    p, E = lanes
    y0 = orc.ic_map(1.0, 0.7, E[0], p[:, 0])
    rng = np.random.default_rng(3)
    v1, v2 = rng.normal(size=8), rng.normal(size=8)
    _, d1 = orc.tangent(1.0, 0.7, 0.02, 300, y0, v1)
    _, d2 = orc.tangent(1.0, 0.7, 0.02, 300, y0, v2)
    _, d12 = orc.tangent(1.0, 0.7, 0.02, 300, y0, 2.0 * v1 - 3.0 * v2)
    assert np.allclose(d12, 2.0 * d1 - 3.0 * d2, rtol=1e-12, atol=1e-12 * np.abs(d12).max())


def test_tangent_on_circular_orbit(orc):
    """f does not depend on t or phi, so a shift of t_0 or phi_0 is carried through
    every RK4 step unchanged: those tangents are exact unit vectors."""
    a, r0 = 0.5, 8.0
    E, L = orc.circular_EL(1.0, a, r0, True)
    gi = orc.inverse_metric(1.0, a, r0, math.pi / 2)
    y0 = np.array([0, r0, math.pi / 2, 0, gi[0, 0] * -E + gi[0, 3] * L, 0, 0,
                   gi[3, 0] * -E + gi[3, 3] * L])
    v = np.zeros(8)
    v[0] = 1.0  # shift of t: f does not depend on t
    _, d = orc.tangent(1.0, a, 0.01, 1000, y0, v)
    assert np.allclose(d, np.eye(8)[0], atol=1e-15)
    v = np.zeros(8)
    v[3] = 1.0  # shift of phi
    _, d = orc.tangent(1.0, a, 0.01, 1000, y0, v)
    assert np.allclose(d, np.eye(8)[3], atol=1e-15)
