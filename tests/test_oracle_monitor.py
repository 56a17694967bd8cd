"""The oracle's invariant monitor (E, L_z, Carter Q, g(u,u) every K steps; Sections
3-4: p_t and p_phi conserved; Section 2, eq. geo: the norm) pinned by the
mathematics: exact conservation in the canonical form, the RK4 truncation order of
the drift, circular orbits as exact fixed points, and the running maximum's own
definition."""
import math

import numpy as np
import pytest

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))


def lower(orc, st, s):
    z = s.copy()
    for i in range(s.shape[1]):
        z[4:, i] = orc.metric(*st[0], s[1, i], s[2, i]) @ s[4:, i]
    return z


def test_hamiltonian_invariants_agree_with_the_velocity_form(orc):
    """The same geodesic state as (x, u) and as (x, p = g u): the two invariant
    formulas (metric on u; p_t, p_phi directly and the inverse metric on p) agree."""
    st = [(1.0, 0.9)]
    rc, s0, c0, _ = orc.ic_constants(61, st, 200, KERR_RANGES)
    z0 = lower(orc, st, s0)
    for i in range(200):
        a = orc.invariants_one(1.0, 0.9, s0[:, i])
        b = orc.invariants_hamiltonian_one(1.0, 0.9, z0[:, i])
        assert np.all(np.abs(a - b) <= 1e-12 * (np.abs(a) + 1.0))
        # and both reproduce the constants the lane was drawn with (E, L_z, Q, -1)
        assert np.all(np.abs(b[:3] - c0[:3, i]) <= 1e-11 * (np.abs(c0[:3, i]) + 1.0))
        assert abs(b[3] + 1.0) <= 1e-12


def test_canonical_form_conserves_E_and_Lz_exactly(orc):
    st = [(1.0, 0.9)]
    rc, s0, _, _ = orc.ic_constants(62, st, 64, KERR_RANGES)
    z0 = lower(orc, st, s0)
    z, status, steps, mon = orc.integrate_monitored(st, z0, 0.05, 4000, 50, hamiltonian=True)
    act = status == 0
    assert act.mean() > 0.9
    assert np.all(mon[4][act] == 0.0) and np.all(mon[5][act] == 0.0)
    # Q and the norm are conserved only to the truncation error
    assert np.all(mon[6][act] > 0.0) and np.all(mon[7][act] > 0.0)
    assert np.all(mon[6][act] < 1e-6 * (np.abs(mon[2][act]) + 1.0)) and np.all(mon[7][act] < 1e-6)


def test_drift_maxima_follow_the_rk4_order(orc):
    """Over the same affine interval and the same monitored instants, halving h
    divides the maximum drift of every invariant by ~2^4 (the global error of RK4)."""
    st = [(1.0, 0.5)]
    ranges = ((8.0, 20.0),) + KERR_RANGES[1:]
    rc, s0, _, _ = orc.ic_constants(63, st, 48, ranges)
    D, act = [], np.ones(48, bool)
    for h, n, every in ((0.2, 1000, 25), (0.1, 2000, 50)):
        y, status, steps, mon = orc.integrate_monitored(st, s0, h, n, every)
        act &= status == 0  # lanes that plunge are left out
        D.append(mon[4:])
    assert act.sum() >= 40
    for k in range(4):
        ratio = D[0][k][act] / D[1][k][act]
        assert 12.0 <= np.median(ratio) <= 20.0, (k, np.median(ratio))


def test_circular_orbits_are_fixed_points(orc):
    """Equatorial circular orbits (Sections 3-4) at r0 > r_isco: every RK4 stage has
    u^r = u^theta = 0 and zero radial and polar accelerations, so r, theta and u stay
    put and the invariants do not drift beyond rounding."""
    M, a = 1.0, 0.9
    st = [(M, a)]
    s0 = orc.ic_circular(64, M, a, 32, 4.0, 30.0, 0.0)
    y, status, steps, mon = orc.integrate_monitored(st, s0, 0.05, 4000, 100)
    assert np.all(status == 0)
    for k in range(4):
        assert np.all(mon[4 + k] <= 1e-13 * (np.abs(mon[k]) + 1.0)), k


def test_running_maximum_definition(orc):
    st = [(1.0, 0.7)]
    rc, s0, _, _ = orc.ic_constants(65, st, 40, KERR_RANGES)
    one = orc.integrate_monitored(st, s0, 0.1, 3000, 60)
    half = orc.integrate_monitored(st, s0, 0.1, 1500, 60)
    two = orc.integrate_monitored(st, half[0], 0.1, 1500, 60, monitor=half[3], status=half[1],
                                  steps=half[2])
    for x, y in zip(one, two):
        assert np.array_equal(x, y)
    # the last step is a monitored one, and the plain integrator reaches the same state
    y, status, steps = orc.integrate(st, s0, 0.1, 3000)
    assert np.array_equal(y, one[0])
    I0 = orc.invariants(st, s0)
    I1 = orc.invariants(st, y)
    act = status == 0
    assert np.array_equal(one[3][:4], I0)
    assert np.all(one[3][4:][:, act] >= np.abs(I1 - I0)[:, act])
    # monotone in time
    assert np.all(one[3][4:] >= half[3][4:])


def test_untouched_lanes_and_empty_calls(orc):
    st = [(1.0, 0.7)]
    rc, s0, _, _ = orc.ic_constants(66, st, 6, KERR_RANGES)
    status = np.array([0, 2, 0, 1, 0, 0], np.int32)
    y, st1, sp, mon = orc.integrate_monitored(st, s0, 0.1, 10, 5, status=status)
    for i in (1, 3):
        assert np.all(np.isnan(mon[:, i])) and np.array_equal(y[:, i], s0[:, i]) and sp[i] == 0
    assert np.all(np.isfinite(mon[:, [0, 2, 4, 5]]))
    y, st1, sp, mon = orc.integrate_monitored(st, s0, 0.1, 0, 5)
    assert np.all(np.isnan(mon)) and np.array_equal(y, s0) and np.all(sp == 0)
    with pytest.raises(ValueError):
        orc.integrate_monitored(st, s0, 0.1, 10, 0)
