"""Pins of the oracle's RK4 integration, termination and initial-condition builders.

- the paper's worked example (Section 5 output table, h = 0.1);
- self-convergence ratio ~ 2^4 (Section 5.3, eq. Qt);
- circular orbits are RK4 fixed points (Sections 3-4, 5.1-5.2 stable orbits);
- unstable vs stable circular orbits (Section 4 ranges, Section 5.1);
- invariant drift falls ~16x per halving of h;
- 40-digit brute-force RK4 (sympy Christoffels + mpmath) on tiny inputs;
- SplitMix64 published outputs; IC round trips.
"""
import math

import numpy as np
import pytest

from conftest import load_golden

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))


def paper_rows(k_values):
    rows = []
    for k in k_values:
        rows.append([0.0, k, math.pi / 2, 0.0, math.sqrt((k * k - 4 * k + 4) / (k * (k - 3))), 0.0,
                     0.0, k / math.sqrt(k - 3)])
    return np.array(rows)


def cartesian(a, r, th, ph):
    """Section 2, eq. coord."""
    rr = np.sqrt(r * r + a * a)
    return rr * np.sin(th) * np.cos(ph), rr * np.sin(th) * np.sin(ph), r * np.cos(th)


@pytest.mark.parametrize("hamiltonian", [False, True])
def test_worked_example(orc, hamiltonian):
    gold = load_golden("worked_example.txt")
    rows = paper_rows([6.0, 3.5])
    for particle, tau, t, x, y, z in gold:
        n = int(round(tau / 0.1))
        p = int(particle)
        if hamiltonian:
            z0 = rows[p].copy()
            z0[4] = -z0[4]  # paper p_t = +E -> covariant p_t = -E
            s, _, _ = orc.integrate([(1.0, 0.0)], z0.reshape(8, 1), 0.1, n, hamiltonian=True)
        else:
            s0 = orc.ic_canonical(1.0, 0.0, rows[p:p + 1])
            s, _, _ = orc.integrate([(1.0, 0.0)], s0, 0.1, n)
        X, Y, Z = cartesian(0.0, s[1, 0], s[2, 0], s[3, 0])
        assert abs(s[0, 0] - t) <= 5.01e-5
        assert abs(X - x) <= 5.01e-5 and abs(Y - y) <= 5.01e-5 and abs(Z - z) <= 5.01e-5


def test_canonical_ic_map(orc):
    """Section 4: dt/dtau = p_t / (1 - 2M/r), dphi/dtau = p_phi / (r^2 sin^2)."""
    rows = paper_rows([6.0, 3.5, 4.0])
    s = orc.ic_canonical(1.0, 0.0, rows)
    for i, row in enumerate(rows):
        r = row[1]
        assert s[4, i] == pytest.approx(row[4] / (1 - 2 / r), rel=1e-15)
        assert s[7, i] == pytest.approx(row[7] / r ** 2, rel=1e-15)
        assert s[5, i] == 0 and s[6, i] == 0
        assert orc.invariants_one(1.0, 0.0, s[:, i])[3] == pytest.approx(-1.0, abs=1e-14)


def test_self_convergence_ratio(orc):
    """Section 5.3: Q = |y_h - y_{h/2}| / |y_{h/2} - y_{h/4}| (Euclidean over the 8
    components) fluctuates around 2^4 for 10 random Kerr a = 0.5 timelike geodesics."""
    ranges = ((5.0, 12.0),) + KERR_RANGES[1:]
    rc, s0, _, _ = orc.ic_constants(11, [(1.0, 0.5)], 48, ranges)
    assert rc == 0
    h, tau = 0.1, 200.0
    n = int(round(tau / h))
    yh, s1, _ = orc.integrate([(1.0, 0.5)], s0, h, n)
    yh2, s2, _ = orc.integrate([(1.0, 0.5)], s0, h / 2, 2 * n)
    yh4, s4, _ = orc.integrate([(1.0, 0.5)], s0, h / 4, 4 * n)
    d1 = np.linalg.norm(yh - yh2, axis=0)
    d2 = np.linalg.norm(yh2 - yh4, axis=0)
    # The ratio needs states at a common tau whose differences are truncation error:
    # keep the first 10 lanes that never reached the horizon (plunging lanes stop at
    # different steps for different h) and whose h/2-h/4 difference is far above the
    # roundoff floor (~1e-12 here; weak-field lanes sit on it and give Q ~ 1).
    keep = np.flatnonzero((s1 == 0) & (s2 == 0) & (s4 == 0) & (d2 > 5e-11))[:10]
    assert keep.size == 10
    Q = d1[keep] / d2[keep]
    assert np.all(Q > 13.0) and np.all(Q < 19.0), Q
    assert abs(np.median(Q) - 16.0) < 1.5


@pytest.mark.parametrize("a,prograde", [(0.0, True), (0.5, True), (0.5, False), (0.9, True)])
def test_circular_orbit_is_rk4_fixed_point(orc, a, prograde):
    """f(y0) has no r, theta, u components on a circular orbit, so RK4 keeps r = r0 and
    advances t, phi linearly (stable orbits outside the ISCO, Sections 5.1-5.2)."""
    r0 = orc.r_isco(1.0, a, prograde) + 1.5
    E, L = orc.circular_EL(1.0, a, r0, prograde)
    gi = orc.inverse_metric(1.0, a, r0, math.pi / 2)
    ut, uph = gi[0, 0] * -E + gi[0, 3] * L, gi[3, 0] * -E + gi[3, 3] * L
    y0 = np.array([0.0, r0, math.pi / 2, 0.0, ut, 0.0, 0.0, uph]).reshape(8, 1)
    h, n = 0.01, 10000
    s, st, steps = orc.integrate([(1.0, a)], y0, h, n)
    assert st[0] == 0 and steps[0] == n
    assert abs(s[1, 0] - r0) <= 1e-12 * r0
    assert s[2, 0] == pytest.approx(math.pi / 2, abs=1e-15)
    assert s[3, 0] == pytest.approx(uph * n * h, rel=1e-12)
    assert s[0, 0] == pytest.approx(ut * n * h, rel=1e-12)


def test_unstable_vs_stable_circular_orbits(orc):
    """Section 4: circular orbits with 3M < r < 6M are unstable, r > 6M stable.  A small
    fluctuation of the angular momentum (1e-8 relative) makes the unstable ones leave
    r0 within a few thousand M, while the stable ones stay put (Section 5.1)."""
    rows = paper_rows([4.0, 5.0, 7.0, 10.0])
    rows[:, 7] *= 1 + 1e-8
    s0 = orc.ic_canonical(1.0, 0.0, rows)
    s, st, _ = orc.integrate([(1.0, 0.0)], s0, 0.1, 30000, horizon_factor=1.0)
    dep = np.abs(s[1] - rows[:, 1])
    for i in (0, 1):  # unstable
        assert st[i] != 0 or dep[i] > 0.5, (i, st[i], dep[i])
    for i in (2, 3):  # stable: excursion of order the perturbation
        assert st[i] == 0 and dep[i] < 1e-5 * rows[i, 1]
    # the printed 4-decimal row r = 3.5 of the IC table is itself off the circular
    # orbit and leaves it
    gold = load_golden("ic_rows.txt")
    s0 = orc.ic_canonical(1.0, 0.0, gold[1:2])
    s, st, _ = orc.integrate([(1.0, 0.0)], s0, 0.1, 30000, horizon_factor=1.0)
    assert st[0] != 0 or abs(s[1, 0] - 3.5) > 0.5


def test_invariant_drift_scales_as_h4(orc):
    rc, s0, c0, _ = orc.ic_constants(12, [(1.0, 0.9)], 8, KERR_RANGES)
    drifts = []
    for h in (0.4, 0.2):
        n = int(round(200.0 / h))
        s, st, _ = orc.integrate([(1.0, 0.9)], s0, h, n)
        assert np.all(st == 0)
        inv = orc.invariants([(1.0, 0.9)], s)
        drifts.append(np.abs(inv[0] - c0[0]) + np.abs(inv[1] - c0[1]) + np.abs(inv[2] - c0[2]))
    ratio = np.median(drifts[0] / drifts[1])
    assert 12.0 < ratio < 20.0, ratio


def test_hamiltonian_and_christoffel_integrations_agree(orc):
    """Both formulations approximate the same geodesic; at config-2-like h the two RK4
    maps differ only at truncation level (mixed relative 1e-7)."""
    rc, s0, _, _ = orc.ic_constants(13, [(1.0, 0.9)], 32, KERR_RANGES)
    n, h = 2000, 0.02
    sc, _, _ = orc.integrate([(1.0, 0.9)], s0, h, n, r_escape=1e300, horizon_factor=0.0)
    z0 = s0.copy()
    for i in range(s0.shape[1]):
        g = orc.metric(1.0, 0.9, s0[1, i], s0[2, i])
        z0[4:, i] = g @ s0[4:, i]
    zh, _, _ = orc.integrate([(1.0, 0.9)], z0, h, n, hamiltonian=True, r_escape=1e300,
                             horizon_factor=0.0)
    uh = np.zeros_like(zh[4:])
    for i in range(zh.shape[1]):
        gi = orc.inverse_metric(1.0, 0.9, zh[1, i], zh[2, i])
        uh[:, i] = gi @ zh[4:, i]
    yh = np.concatenate([zh[:4], uh])
    err = (np.abs(yh - sc) / (np.abs(sc) + 1)).max()
    assert err < 1e-7, err


@pytest.fixture(scope="module")
def mp_rk4():
    """RK4 in 40-digit arithmetic with Christoffels from sympy's symbolic derivative
    of the metric of Section 2, eq. kerr."""
    sp = pytest.importorskip("sympy")
    mp = pytest.importorskip("mpmath")
    r, th, M, a = sp.symbols("r theta M a", real=True)
    rho2 = r ** 2 + a ** 2 * sp.cos(th) ** 2
    Delta = r ** 2 - 2 * M * r + a ** 2
    Sigma = (r ** 2 + a ** 2) ** 2 - a ** 2 * Delta * sp.sin(th) ** 2
    g = sp.zeros(4, 4)
    g[0, 0] = -(Delta - a ** 2 * sp.sin(th) ** 2) / rho2
    g[0, 3] = g[3, 0] = -2 * a * M * r * sp.sin(th) ** 2 / rho2
    g[1, 1] = rho2 / Delta
    g[2, 2] = rho2
    g[3, 3] = Sigma / rho2 * sp.sin(th) ** 2
    X = [None, r, th, None]
    dg = [[[sp.diff(g[i, j], X[l]) if X[l] is not None else sp.Integer(0) for j in range(4)]
           for i in range(4)] for l in range(4)]
    fg = sp.lambdify((M, a, r, th), g, "mpmath")
    fdg = sp.lambdify((M, a, r, th), dg, "mpmath")

    def f(Mv, av, y):
        G0 = mp.matrix(fg(Mv, av, y[1], y[2]))
        Gi = G0 ** -1
        D = fdg(Mv, av, y[1], y[2])
        u = y[4:]
        acc = [mp.mpf(0)] * 4
        for mu in range(4):
            s = mp.mpf(0)
            for al in range(4):
                for be in range(4):
                    Gm = mp.mpf(0)
                    for nu in range(4):
                        Gm += Gi[mu, nu] * (D[al][nu][be] + D[be][nu][al] - D[nu][al][be])
                    s += Gm / 2 * u[al] * u[be]
            acc[mu] = -s
        return list(u) + acc

    def run(Mv, av, h, n, y0):
        with mp.workdps(40):
            Mv, av, h = mp.mpf(Mv), mp.mpf(av), mp.mpf(h)
            y = [mp.mpf(v) for v in y0]
            for _ in range(n):
                k1 = f(Mv, av, y)
                k2 = f(Mv, av, [y[i] + h / 2 * k1[i] for i in range(8)])
                k3 = f(Mv, av, [y[i] + h / 2 * k2[i] for i in range(8)])
                k4 = f(Mv, av, [y[i] + h * k3[i] for i in range(8)])
                y = [y[i] + h / 6 * (k1[i] + 2 * k2[i] + 2 * k3[i] + k4[i]) for i in range(8)]
            return np.array([float(v) for v in y])
    return run


@pytest.mark.slow
def test_brute_force_high_precision_rk4(orc, mp_rk4):
    rc, s0, _, _ = orc.ic_constants(14, [(1.0, 0.9)], 3, KERR_RANGES)
    for i in range(3):
        want = mp_rk4(1.0, 0.9, 0.02, 8, s0[:, i])
        got, _, _ = orc.integrate([(1.0, 0.9)], s0[:, i:i + 1], 0.02, 8)
        assert (np.abs(got[:, 0] - want) / (np.abs(want) + 1)).max() < 1e-13
    # a near-horizon null ray of the camera configuration
    y0 = orc.ray_ic(1.0, 0.998, 8.0, 1.0, 3.0, 2.0)
    want = mp_rk4(1.0, 0.998, 0.1, 6, y0)
    got, _, _ = orc.integrate([(1.0, 0.998)], y0.reshape(8, 1), 0.1, 6)
    assert (np.abs(got[:, 0] - want) / (np.abs(want) + 1)).max() < 1e-13


def test_splitmix64_published_outputs(orc):
    """SplitMix64 (Steele, Lea & Flood 2014) seeded with 0 outputs 0xe220a8397b1dcdaf,
    0x6e789e6aa1b965f4, ...; draw k of lane 0 / attempt 0 is output k + 1."""
    assert orc.draw_u64(0, 0, 0, 0) == 0xE220A8397B1DCDAF
    assert orc.draw_u64(0, 0, 0, 1) == 0x6E789E6AA1B965F4
    assert orc.draw_u64(5, 0, 0, 0) != orc.draw_u64(5, 1, 0, 0)


def test_constants_sampler_round_trip(orc):
    rc, s, c, att = orc.ic_constants(2, [(1.0, 0.9)], 512, KERR_RANGES)
    assert rc == 0 and np.all(att >= 1)
    inv = orc.invariants([(1.0, 0.9)], s)
    assert np.abs(inv[0] - c[0]).max() < 1e-13
    assert np.abs(inv[1] - c[1]).max() < 1e-12
    assert np.abs(inv[2] - c[2]).max() < 1e-11 * 12
    assert np.abs(inv[3] + 1.0).max() < 1e-13
    for k, (lo, hi) in enumerate(KERR_RANGES):
        v = s[1 + k] if k < 2 else c[k - 2]
        assert np.all(v >= lo) and np.all(v <= hi)
    for i in range(0, 512, 37):
        assert orc.potential_R(1.0, 0.9, c[0, i], c[1, i], c[2, i], 1.0, s[1, i]) >= 0
    # a sub-batch starting at lane0 draws the same lanes
    rc, s2, _, att2 = orc.ic_constants(2, [(1.0, 0.9)], 100, KERR_RANGES, lane0=200)
    assert np.array_equal(s2, s[:, 200:300]) and np.array_equal(att2, att[200:300])
    # acceptance (R >= 0 and Theta >= 0) is a few percent at a = 0.9
    acc = 512 / att.sum()
    assert 0.02 < acc < 0.12


def test_constants_sampler_exhaustion(orc):
    rc, s, _, att = orc.ic_constants(3, [(1.0, 0.9)], 4, ((5, 6), (1, 2), (0.1, 0.2), (9, 10), (0, 1)),
                                     max_attempts=5)
    assert rc == -5 and np.all(np.isnan(s)) and np.all(att == 5)


def test_circular_builder(orc):
    s = orc.ic_circular(1, 1.0, 0.0, 1024, 6.5, 20.0, 1e-3)
    assert np.all(s[1] >= 6.5) and np.all(s[1] < 20.0)
    assert np.all(s[2] == math.pi / 2) and np.all(s[5] == 0) and np.all(s[6] == 0)
    inv = orc.invariants([(1.0, 0.0)], s)
    assert np.abs(inv[3] + 1).max() < 1e-14
    Lc = np.array([orc.schwarzschild_circular(1.0, r)[1] for r in s[1]])
    rel = inv[1] / Lc - 1
    assert np.abs(rel).max() <= 1e-3 * (1 + 1e-12) and np.abs(rel).max() > 9e-4
    s2 = orc.ic_circular(1, 1.0, 0.0, 10, 6.5, 20.0, 1e-3, lane0=100)
    assert np.array_equal(s2, s[:, 100:110])


def test_termination_rules(orc):
    # a plunging lane ends at the horizon with the crossing state stored
    rows = paper_rows([3.5])
    rows[0, 7] *= 0.8  # too little angular momentum: plunge
    s0 = orc.ic_canonical(1.0, 0.0, rows)
    s, st, steps = orc.integrate([(1.0, 0.0)], s0, 0.01, 100000)
    assert st[0] == 1 and steps[0] < 100000
    s_prev, st_prev, _ = orc.integrate([(1.0, 0.0)], s0, 0.01, int(steps[0]) - 1)
    assert st_prev[0] == 0 and s_prev[1, 0] > 2.02
    if s[1, 0] > 2.02:
        # a stage point of the last step entered r <= 1.01 r_+: the step's start is kept
        assert np.array_equal(s, s_prev)
    else:
        assert s[1, 0] > 2.0
    # resumable: two half calls equal one call
    rc, s0, _, _ = orc.ic_constants(4, [(1.0, 0.9)], 16, KERR_RANGES)
    full, st_f, sp_f = orc.integrate([(1.0, 0.9)], s0, 0.02, 400)
    half, st_h, sp_h = orc.integrate([(1.0, 0.9)], s0, 0.02, 200)
    half, st_h, sp_h = orc.integrate([(1.0, 0.9)], half, 0.02, 200, status=st_h, steps=sp_h)
    assert np.array_equal(full, half) and np.array_equal(sp_f, sp_h)
    # non-finite input -> NONFINITE after one evaluated step, state untouched;
    # inactive lanes do not step
    bad = s0[:, :2].copy()
    bad[5, 0] = np.nan
    s, st, steps = orc.integrate([(1.0, 0.9)], bad, 0.02, 10, status=np.array([0, 2], np.int32))
    assert st[0] == 4 and steps[0] == 1 and np.isnan(s[5, 0]) and np.array_equal(s[:, 1], bad[:, 1])
    assert st[1] == 2 and steps[1] == 0
