"""Pins of the oracle's adaptive integrator (Dormand-Prince 5(4) with the standard
step-size control; the paper announces other Runge-Kutta members in Section 5):
order 5 of the solution and order 5 of the embedded error estimate (which pin the
tableau), exactness on circular orbits, the tolerance scaling of the global error,
agreement with a fine fixed-step RK4 reference, the landing on tau_end and the stop
rules."""
import math

import numpy as np
import pytest

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))
ST = [(1.0, 0.9)]


def fixed(orc, s0, h, tau_end):
    """The adaptive driver with the controller switched off: every attempt accepted,
    h never changes (facmin = facmax = 1)."""
    return orc.integrate_adaptive(ST, s0, tau_end, h, rtol=1e300, atol=1e300, facmin=1.0,
                                  facmax=1.0)


def test_fixed_step_solution_is_fifth_order(orc):
    rc, s0, _, _ = orc.ic_constants(61, ST, 48, ((6.0, 12.0),) + KERR_RANGES[1:])
    ys = [fixed(orc, s0, h, 256.0)[0] for h in (0.4, 0.2, 0.1)]
    d1 = np.abs(ys[0] - ys[1]).max(axis=0)
    d2 = np.abs(ys[1] - ys[2]).max(axis=0)
    ok = d2 > 3e-11  # truncation-dominated lanes
    assert ok.sum() > 15
    ratio = np.median(d1[ok] / d2[ok])
    assert 26.0 < ratio < 40.0, ratio  # 2^5 (classic RK4 gives 2^4)


def test_embedded_estimate_is_fifth_order(orc):
    """y1 - y1* of the pair is O(h^5): halving h divides it by ~32; and the
    5th-order step itself agrees with two half steps to O(h^6)."""
    rc, s0, _, _ = orc.ic_constants(62, ST, 16, ((6.0, 12.0),) + KERR_RANGES[1:])
    ratios, r6 = [], []
    for i in range(s0.shape[1]):
        y = s0[:, i]
        e = [np.abs(orc.dp45_attempt(1.0, 0.9, h, y)[1]).max() for h in (0.8, 0.4)]
        ratios.append(e[0] / e[1])
        one = orc.dp45_attempt(1.0, 0.9, 0.8, y)[0]
        half = orc.dp45_attempt(1.0, 0.9, 0.4, orc.dp45_attempt(1.0, 0.9, 0.4, y)[0])[0]
        one2 = orc.dp45_attempt(1.0, 0.9, 0.4, y)[0]
        half2 = orc.dp45_attempt(1.0, 0.9, 0.2, orc.dp45_attempt(1.0, 0.9, 0.2, y)[0])[0]
        r6.append(np.abs(one - half).max() / np.abs(one2 - half2).max())
    assert 28.0 < np.median(ratios) < 36.0, np.median(ratios)
    assert 56.0 < np.median(r6) < 72.0, np.median(r6)  # local error O(h^6): 2^6


def test_circular_orbit_is_exact_and_lands_on_tau_end(orc):
    """On an exact circular equatorial orbit the right-hand side is the same at every
    stage point, so each step moves only t and phi, linearly in tau."""
    s0 = orc.ic_circular(5, 1.0, 0.9, 8, 6.5, 20.0, 0.0)
    y, tau, h, st, steps, rej = orc.integrate_adaptive(ST, s0, 777.7, 0.1, rtol=1e-12, atol=1e-12)
    assert np.all(st == 0) and np.all(tau == 777.7)
    # (the controller grows the step to ~100 M here; the residual radial acceleration
    # of the rounded circular initial data, ~1e-17, moves r by ~1e-10 over tau_end)
    assert np.abs(y[1] - s0[1]).max() <= 1e-9 * s0[1].max()
    assert np.abs(y[3] - s0[7] * 777.7).max() <= 1e-11 * np.abs(y[3]).max()
    assert np.abs(y[0] - s0[4] * 777.7).max() <= 1e-11 * np.abs(y[0]).max()


def test_global_error_follows_the_tolerance(orc):
    rc, s0, _, _ = orc.ic_constants(63, ST, 24, KERR_RANGES)
    ref, rst, _ = orc.integrate(ST, s0, 0.005, 40000)  # fixed-step RK4, tau = 200
    errs, steps = [], []
    for tol in (1e-7, 1e-9, 1e-11):
        y, tau, h, st, sp, rj = orc.integrate_adaptive(ST, s0, 200.0, 0.1, rtol=tol, atol=tol)
        assert np.all(st == rst) and np.all(tau[st == 0] == 200.0)
        ok = st == 0
        errs.append((np.abs(y - ref) / (np.abs(ref) + 1)).max(axis=0)[ok].max())
        steps.append(sp.mean())
    assert errs[2] < 1e-8
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10, errs
    # steps grow like tol^(-1/5): x 2.5 per factor 100
    assert 1.8 < steps[1] / steps[0] < 3.5 and 1.8 < steps[2] / steps[1] < 3.5, steps


def test_stop_rules_and_budget(orc):
    st = [(1.0, 0.0)]
    rc, s0, _, _ = orc.ic_constants(64, st, 400, KERR_RANGES)
    y, tau, h, status, steps, rej = orc.integrate_adaptive(st, s0, 2000.0, 0.1, rtol=1e-9, atol=1e-9)
    ref, rstatus, _ = orc.integrate(st, s0, 0.02, 100000)
    assert (status == 1).sum() > 50
    assert np.array_equal(status == 1, rstatus == 1)  # the same orbits plunge
    r_stop = 1.01 * 2.0
    hz = status == 1
    assert np.all(y[1][hz] > r_stop * 0.5) and np.all(tau[hz] < 2000.0)
    # budget: 3 attempts per call
    rc, s1, _, _ = orc.ic_constants(65, ST, 20, KERR_RANGES)
    y, tau, h, status, steps, rej = orc.integrate_adaptive(ST, s1, 1e6, 0.1, rtol=1e-9, atol=1e-9,
                                                           max_attempts=3)
    assert np.all(status == 5) and np.all(steps + rej == 3)
