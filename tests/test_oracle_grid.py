"""Pins of the oracle's gridded 3+1 metric (Section 2, eq. ADM with the Kerr lapse,
shift and spatial metric): the 3+1 functions reproduce the Kerr metric of eq. kerr,
the interpolant is exact on cubic data with the right derivatives, its error falls
as the fourth power of the spacing, and RK4 in the gridded Kerr metric converges to
RK4 in the analytic one."""
import math

import numpy as np
import pytest

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))


@pytest.mark.parametrize("a", [0.0, 0.6, 0.998])
def test_3p1_functions_reproduce_the_kerr_metric(orc, a):
    for r, th in ((2.5, 0.4), (7.0, 1.5707), (30.0, 2.8)):
        if r <= 1 + math.sqrt(1 - a * a):
            continue
        al, be, grr, gthth, gpp_s2 = orc.kerr_3p1(1.0, a, r, th)
        g = orc.metric(1.0, a, r, th)
        gpp = gpp_s2 * math.sin(th) ** 2
        # ds^2 = -alpha^2 dt^2 + gamma_ij (dx^i + beta^i dt)(dx^j + beta^j dt)
        assert g[0, 0] == pytest.approx(-al * al + gpp * be * be, abs=1e-14)
        assert g[0, 3] == pytest.approx(gpp * be, abs=1e-14)
        assert g[1, 1] == pytest.approx(grr, rel=1e-14)
        assert g[2, 2] == pytest.approx(gthth, rel=1e-14)
        assert g[3, 3] == pytest.approx(gpp, rel=1e-14)


def test_interpolant_is_exact_on_cubics(orc):
    nr, nth, r0, dr, th0, dth = 12, 9, 3.0, 0.5, 0.3, 0.25
    rr = r0 + dr * np.arange(nr)
    tt = th0 + dth * np.arange(nth)
    R, T = np.meshgrid(rr, tt, indexing="ij")
    def poly(k, r, t):
        return (1.0 + k) * r ** 3 - 2.0 * r * t ** 2 + 0.5 * t ** 3 + k * r * t + 3.0
    nodes = np.stack([poly(k, R, T) for k in range(5)], axis=-1)
    G = orc.Grid(nodes, r0, dr, th0, dth)
    for r, t in ((3.7, 0.61), (6.9, 1.9), (3.01, 2.2), (8.4, 0.33)):
        F, Fr, Ft = orc.grid_eval(G, r, t)
        for k in range(5):
            assert F[k] == pytest.approx(poly(k, r, t), rel=1e-12)
            assert Fr[k] == pytest.approx(3 * (1 + k) * r * r - 2 * t * t + k * t, rel=1e-11)
            assert Ft[k] == pytest.approx(-4 * r * t + 1.5 * t * t + k * r, rel=1e-11, abs=1e-11)


def test_interpolation_error_is_fourth_order(orc):
    pts = [(4.3, 0.9), (9.1, 1.4), (15.7, 2.0)]
    errs = []
    for f in (1, 2, 4):
        nr, nth = 60 * f + 1, 30 * f + 1
        G = orc.grid_kerr(1.0, 0.9, nr, nth, 2.5, 20.0 / (nr - 1), 0.3, (math.pi - 0.6) / (nth - 1))
        errs.append(max(np.abs(orc.grid_eval(G, r, t)[0] - orc.kerr_3p1(1.0, 0.9, r, t)).max()
                        for r, t in pts))
    assert 10.0 < errs[0] / errs[1] < 25.0 and 10.0 < errs[1] / errs[2] < 25.0, errs


def test_grid_rhs_and_integration_converge_to_analytic_kerr(orc):
    st = [(1.0, 0.9)]
    rc, s0, _, _ = orc.ic_constants(81, st, 16, ((6.0, 20.0),) + KERR_RANGES[1:])
    z0 = s0.copy()
    for i in range(s0.shape[1]):
        z0[4:, i] = orc.metric(1.0, 0.9, s0[1, i], s0[2, i]) @ s0[4:, i]
    ref, rst, _ = orc.integrate(st, z0, 0.02, 2000, hamiltonian=True)
    errs = []
    for f in (1, 2):
        nr, nth = 400 * f + 1, 200 * f + 1
        dr, dth = 60.0 / (nr - 1), (math.pi - 0.2) / (nth - 1)
        G = orc.grid_kerr(1.0, 0.9, nr, nth, 1.5, dr, 0.1, dth)
        # the right-hand side itself
        f0 = orc.grid_rhs(G, z0[:, 0])
        assert np.abs(f0 - orc.rhs_hamiltonian(1.0, 0.9, z0[:, 0])).max() < 1e-5
        z, zst, _ = orc.integrate_grid(G, z0, 0.02, 2000, r_stop=1.01 * 1.4359, r_escape=50.0)
        assert np.array_equal(zst, rst)
        errs.append((np.abs(z - ref) / (np.abs(ref) + 1)).max())
    assert errs[1] < errs[0] / 8.0, errs  # interpolation error ~ h^4
    assert errs[1] < 1e-4
