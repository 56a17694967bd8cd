"""Pins of the oracle's metric, Christoffel symbols and geodesic right-hand side.

- g g^{-1} = I; a = 0 gives the textbook Schwarzschild metric and Christoffels;
- analytic metric partials equal complex-step partials of the metric;
- Christoffels equal a symbolic derivation (sympy) of the Kerr metric of
  Section 2, eq. kerr, evaluated in 30-digit arithmetic;
- the Christoffel right-hand side reproduces the paper's Hamilton equations:
  Schwarzschild (Section 4) and equatorial Kerr (Section 3);
- E, L_z, Carter Q and g(u,u) are first integrals of the right-hand side.
"""
import math

import numpy as np
import pytest

RNG = np.random.default_rng(20240611)


def random_points(n, a_max=0.998):
    a = RNG.uniform(0.0, a_max, n)
    rp = 1 + np.sqrt(1 - a * a)
    r = rp * 1.2 + RNG.uniform(0, 40, n)
    th = RNG.uniform(0.15, math.pi - 0.15, n)
    return a, r, th


def test_metric_inverse_identity(orc):
    for a, r, th in zip(*random_points(200)):
        g = orc.metric(1.0, a, r, th)
        gi = orc.inverse_metric(1.0, a, r, th)
        assert np.abs(g @ gi - np.eye(4)).max() < 1e-13
        assert np.allclose(g, g.T, rtol=0, atol=0)


def test_schwarzschild_limit_metric_and_christoffels(orc):
    """a = 0: textbook Schwarzschild metric and its 9 independent nonzero Christoffels."""
    M = 1.3
    for r, th in [(3.0, 0.7), (7.5, 1.2), (25.0, 2.9)]:
        f = 1 - 2 * M / r
        g = orc.metric(M, 0.0, r, th)
        want = np.diag([-f, 1 / f, r * r, r * r * math.sin(th) ** 2])
        assert np.allclose(g, want, rtol=1e-15, atol=0)
        G = orc.christoffel(M, 0.0, r, th)
        E = np.zeros((4, 4, 4))
        s, c = math.sin(th), math.cos(th)
        E[0, 0, 1] = E[0, 1, 0] = M / (r * (r - 2 * M))
        E[1, 0, 0] = M * (r - 2 * M) / r ** 3
        E[1, 1, 1] = -M / (r * (r - 2 * M))
        E[1, 2, 2] = -(r - 2 * M)
        E[1, 3, 3] = -(r - 2 * M) * s * s
        E[2, 1, 2] = E[2, 2, 1] = 1 / r
        E[2, 3, 3] = -s * c
        E[3, 1, 3] = E[3, 3, 1] = 1 / r
        E[3, 2, 3] = E[3, 3, 2] = c / s
        assert np.abs(G - E).max() < 1e-14 * max(1.0, np.abs(E).max())


def test_analytic_partials_equal_complex_step(orc):
    for a, r, th in zip(*random_points(200)):
        d1 = orc.metric_partials(1.0, a, r, th)
        d2 = orc.metric_partials_complex_step(1.0, a, r, th)
        scale = np.abs(d2).max()
        assert np.abs(d1 - d2).max() <= 1e-13 * scale


def test_christoffel_symmetry_and_count(orc):
    a, r, th = 0.9, 4.2, 1.1
    G = orc.christoffel(1.0, a, r, th)
    assert np.abs(G - G.transpose(0, 2, 1)).max() == 0.0
    independent = sum(1 for m in range(4) for i in range(4) for j in range(i, 4)
                      if abs(G[m, i, j]) > 1e-14)
    assert independent == 20  # generic Kerr point


@pytest.fixture(scope="module")
def sympy_christoffel():
    """Christoffels of the paper's Kerr metric by symbolic differentiation (sympy),
    evaluated with mpmath at 30 digits.  Independent of the oracle's hand-written
    partials and of its Gauss-Jordan inverse."""
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

    def gamma(Mv, av, rv, tv):
        with mp.workdps(30):
            args = [mp.mpf(Mv), mp.mpf(av), mp.mpf(rv), mp.mpf(tv)]
            G0 = mp.matrix(fg(*args))
            Gi = G0 ** -1
            D = fdg(*args)
            out = np.zeros((4, 4, 4))
            for mu in range(4):
                for al in range(4):
                    for be in range(4):
                        s = mp.mpf(0)
                        for nu in range(4):
                            s += Gi[mu, nu] * (D[al][nu][be] + D[be][nu][al] - D[nu][al][be])
                        out[mu, al, be] = float(s / 2)
            return out
    return gamma


def test_christoffel_matches_symbolic(orc, sympy_christoffel):
    for a, r, th in list(zip(*random_points(12))) + [(0.998, 1.3, 0.4), (0.5, 60.0, 2.0)]:
        G = orc.christoffel(1.0, a, r, th)
        Gs = sympy_christoffel(1.0, a, r, th)
        scale = np.abs(Gs).max()
        assert np.abs(G - Gs).max() <= 2e-14 * scale, (a, r, th)


def _momentum_rate(orc, M, a, y):
    """dp_mu/dtau implied by the Christoffel RHS: d(g_{mu nu} u^nu)/dtau
    = (d_l g_{mu nu}) u^l u^nu + g_{mu nu} du^nu/dtau, partials by complex step."""
    f = orc.rhs(M, a, y)
    g = orc.metric(M, a, y[1], y[2])
    dg = orc.metric_partials_complex_step(M, a, y[1], y[2])
    u = y[4:]
    return np.einsum("lmn,l,n->m", dg, u, u) + g @ f[4:], f


def test_rhs_reproduces_paper_schwarzschild_equations(orc):
    """Section 4 printed Hamilton equations (paper sign p_t = +E)."""
    M = 1.0
    for _ in range(100):
        r = RNG.uniform(2.5, 40.0)
        th = RNG.uniform(0.2, math.pi - 0.2)
        u = RNG.normal(size=4)
        y = np.array([0.0, r, th, 0.3, *u])
        g = orc.metric(M, 0.0, r, th)
        p = g @ u
        pt, pr, pth, pph = -p[0], p[1], p[2], p[3]
        f2 = 1 - 2 * M / r
        s, c = math.sin(th), math.cos(th)
        xdot = np.array([pt / f2, f2 * pr, pth / r ** 2, pph / (r ** 2 * s * s)])
        pdot_paper = np.array([0.0,
                               -M * pt ** 2 / (-r + 2 * M) ** 2 - M * pr ** 2 / r ** 2
                               + pth ** 2 / r ** 3 + pph ** 2 / (r ** 3 * s * s),
                               pph ** 2 * c / (r ** 2 * s ** 3),
                               0.0])
        pdot, f = _momentum_rate(orc, M, 0.0, y)
        pdot_std = pdot.copy()
        pdot_std[0] = -pdot_std[0]  # paper p_t = -p_t(standard)
        scale = max(1.0, np.abs(pdot_paper).max())
        assert np.abs(f[:4] - xdot).max() <= 1e-14 * max(1, np.abs(xdot).max())
        assert np.abs(pdot_std - pdot_paper).max() <= 1e-13 * scale


def test_rhs_reproduces_paper_equatorial_kerr_equations(orc):
    """Section 3 printed equatorial Kerr equations (theta = pi/2, p_theta = 0, p_t = +E)."""
    M = 1.0
    for _ in range(100):
        a = RNG.uniform(0, 0.999)
        r = (1 + math.sqrt(1 - a * a)) * 1.1 + RNG.uniform(0, 30)
        u = RNG.normal(size=4)
        u[2] = 0.0
        y = np.array([0.0, r, math.pi / 2, 0.0, *u])
        g = orc.metric(M, a, r, math.pi / 2)
        p = g @ u
        pt, pr, pph = -p[0], p[1], p[3]
        D = 2 * M * r - a * a - r * r
        tdot = (-(2 * M * a * a + a * a * r + r ** 3) * pt + 2 * a * M * pph) / (r * D)
        rdot = -D / r ** 2 * pr
        phidot = (-2 * M * a * pt + (2 * M - r) * pph) / (r * D)
        prdot = (-(M * r - a * a) / r ** 3 * pr ** 2
                 + M * (4 * M * a * a * r - a ** 4 - 2 * a * a * r * r - r ** 4) / (r * r * D * D) * pt ** 2
                 - 2 * M * a * (4 * M * r - a * a - 3 * r * r) / (r * r * D * D) * pt * pph
                 + (4 * M * M * r - M * a * a - 4 * M * r * r + r ** 3) / (r * r * D * D) * pph ** 2)
        pdot, f = _momentum_rate(orc, M, a, y)
        xs = np.abs([tdot, rdot, phidot]).max()
        assert abs(f[0] - tdot) <= 1e-13 * xs
        assert abs(f[1] - rdot) <= 1e-13 * xs
        assert abs(f[3] - phidot) <= 1e-13 * xs
        assert abs(f[2]) == 0.0
        ps = max(1.0, abs(prdot))
        assert abs(pdot[1] - prdot) <= 1e-12 * ps
        # d p_t / dtau = d p_theta / dtau = d p_phi / dtau = 0
        assert np.abs(pdot[[0, 2, 3]]).max() <= 1e-12 * ps
        assert abs(f[6]) <= 1e-14  # u^theta stays zero in the plane


@pytest.mark.parametrize("mu2", [1.0, 0.0])
def test_invariants_are_first_integrals(orc, mu2):
    """dI/dtau = grad I . f = 0 for I in (E, L_z, Q, g(u,u)), by central differences
    of the oracle's invariants along the oracle's RHS, at random Kerr states."""
    M = 1.0
    worst = 0.0
    for _ in range(300):
        a = RNG.uniform(0, 0.998)
        r = (1 + math.sqrt(1 - a * a)) * 1.3 + RNG.uniform(0, 30)
        th = RNG.uniform(0.3, math.pi - 0.3)
        E = RNG.uniform(0.9, 1.2)
        Lz = RNG.uniform(-5, 5)
        Q = RNG.uniform(0, 15)
        R = orc.potential_R(M, a, E, Lz, Q, mu2, r)
        T = orc.potential_Theta(a, E, Lz, Q, mu2, th)
        if R < 0 or T < 0:
            continue
        u = orc.velocity_from_constants(M, a, E, Lz, Q, mu2, r, th, RNG.choice([-1, 1]),
                                        RNG.choice([-1, 1]))
        y = np.array([0.0, r, th, 0.0, *u])
        f = orc.rhs(M, a, y)
        eps = 1e-5
        Ip = orc.invariants_one(M, a, y + eps * f)
        Im = orc.invariants_one(M, a, y - eps * f)
        dI = (Ip - Im) / (2 * eps)
        scale = np.array([abs(E), max(abs(Lz), 1), max(Q, 1), 1.0]) * max(1.0, np.abs(f).max())
        worst = max(worst, (np.abs(dI) / scale).max())
    assert worst < 1e-7


def test_rhs_vanishes_radially_on_circular_orbits(orc):
    for a in (0.0, 0.5, 0.9):
        for prograde in (True, False):
            r = orc.r_isco(1.0, a, prograde) * 1.3
            E, L = orc.circular_EL(1.0, a, r, prograde)
            gi = orc.inverse_metric(1.0, a, r, math.pi / 2)
            u = [gi[0, 0] * -E + gi[0, 3] * L, 0.0, 0.0, gi[3, 0] * -E + gi[3, 3] * L]
            f = orc.rhs(1.0, a, [0, r, math.pi / 2, 0, *u])
            assert np.abs(f[[1, 2, 4, 5, 6, 7]]).max() < 1e-15
            assert orc.invariants_one(1.0, a, [0, r, math.pi / 2, 0, *u])[3] == pytest.approx(-1, abs=1e-14)


def test_hamiltonian_and_christoffel_rhs_agree(orc):
    """dx/dtau of the Hamiltonian form equals u; dp/dtau equals the rate implied by the
    Christoffel form (same state, two formulations of Section 2, eq. Ham)."""
    for _ in range(100):
        a = RNG.uniform(0, 0.998)
        r = (1 + math.sqrt(1 - a * a)) * 1.2 + RNG.uniform(0, 30)
        th = RNG.uniform(0.2, math.pi - 0.2)
        u = RNG.normal(size=4)
        y = np.array([1.0, r, th, 0.5, *u])
        g = orc.metric(1.0, a, r, th)
        z = np.concatenate([y[:4], g @ u])
        fh = orc.rhs_hamiltonian(1.0, a, z)
        pdot, f = _momentum_rate(orc, 1.0, a, y)
        assert np.abs(fh[:4] - u).max() <= 1e-13 * np.abs(u).max()
        assert np.abs(fh[4:] - pdot).max() <= 1e-12 * max(1, np.abs(pdot).max())
        assert fh[4] == 0.0 and fh[7] == 0.0
