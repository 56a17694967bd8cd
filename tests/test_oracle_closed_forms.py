"""Pins of the oracle's closed forms against the numbers the paper prints.

Paper passages: Section 3 (equatorial circular orbits, eq1, eq2, energia,
momento, ISCO, extreme-Kerr limits, omega), Section 4 (Schwarzschild circular
orbits, gralorbits), Section 5.2 (ISCO tables).
"""
import math

import numpy as np
import pytest

from conftest import load_golden


def paper_eq1_rhs(M, a, r, pt, pphi):
    """Section 3, eq1: p_r^2 as a function of (p_t, p_phi), paper sign p_t = +E."""
    den = (M * r - a * a) * (2 * M * r - a * a - r * r) ** 2
    return (r * (4 * M * M * r - M * a * a - 4 * M * r * r + r ** 3) / den * pphi ** 2
            - 2 * r * a * M * (4 * M * r - a * a - 3 * r * r) / den * pt * pphi
            + r * M * (4 * M * a * a * r - a ** 4 - 2 * a * a * r * r - r ** 4) / den * pt ** 2)


def paper_eq2_rhs(M, a, r, pt, pphi):
    """Section 3, eq2: the constraint 2L = -1 evaluated on circular orbits."""
    den = r * (M * r - a * a) * (2 * M * r - a * a - r * r)
    return (-(M - r) * (2 * M * r + a * a - r * r) / den * pphi ** 2
            + 2 * M * a * (2 * M * r + a * a - 3 * r * r) / den * pt * pphi
            - (2 * M * M * a * a * r + M * a ** 4 - 3 * M * a * a * r * r - 2 * M * r ** 4
               + a ** 4 * r + a * a * r ** 3) / den * pt ** 2)


@pytest.mark.parametrize("table,prograde", [("isco_corotating.txt", True),
                                            ("isco_counterrotating.txt", False)])
def test_isco_radius_matches_tables(orc, table, prograde):
    rows = load_golden(table)
    for a, r, _, _ in rows:
        # the tables carry ~4e-11 scatter in their last printed digits
        assert abs(orc.r_isco(1.0, a, prograde) - r) <= 1e-10, (a, r)


@pytest.mark.parametrize("paper_form", [False, True])
@pytest.mark.parametrize("table,prograde", [("isco_corotating.txt", True),
                                            ("isco_counterrotating.txt", False)])
def test_circular_E_L_match_tables(orc, table, prograde, paper_form):
    rows = load_golden(table)
    for a, r, pt, pphi in rows:
        if a == 1.0 and prograde:
            continue  # the r -> M+ limit is checked separately
        E, L = orc.circular_EL(1.0, a, r, prograde, paper_form=paper_form)
        assert abs(E - pt) <= 2e-12, (a, E, pt)
        assert abs(L - pphi) <= 2e-12, (a, L, pphi)


@pytest.mark.parametrize("table,prograde", [("isco_corotating.txt", True),
                                            ("isco_counterrotating.txt", False)])
def test_circular_E_L_solve_paper_eq1_eq2(orc, table, prograde):
    """The closed forms solve the paper's own circular-orbit system (eq1 = 0, eq2 = -1)
    at the table radii and at radii outside them."""
    rows = load_golden(table)
    for a, r_tab, _, _ in rows:
        if a == 1.0:
            continue
        for r in (r_tab, r_tab + 1.7, 3.0 * r_tab):
            E, L = orc.circular_EL(1.0, a, r, prograde)
            scale = max(1.0, abs(r * L * L / (r * r)))
            assert abs(paper_eq1_rhs(1.0, a, r, E, L)) <= 1e-10 * scale
            assert abs(paper_eq2_rhs(1.0, a, r, E, L) + 1.0) <= 1e-11


def test_extreme_kerr_limits(orc):
    """Section 3, eqs. exKerr+ / exKerr-; E+ is 1/sqrt(3) (the a = 1 table row), the
    printed 1/3 is read as a typo."""
    assert orc.r_isco(1.0, 1.0, True) == pytest.approx(1.0, abs=1e-14)
    assert orc.r_isco(1.0, 1.0, False) == pytest.approx(9.0, abs=1e-14)
    # co-rotating: right-hand limit r -> M+
    for eps in (1e-4, 1e-5, 1e-6):
        E, L = orc.circular_EL(1.0, 1.0, 1.0 + eps, True)
        assert abs(E - 1 / math.sqrt(3)) < 3 * eps ** 0.5
        assert abs(L - 2 / math.sqrt(3)) < 3 * eps ** 0.5
    E, L = orc.circular_EL(1.0, 1.0, 9.0, False)
    assert E == pytest.approx(5 / (3 * math.sqrt(3)), rel=1e-14)
    assert L == pytest.approx(-22 / (3 * math.sqrt(3)), rel=1e-14)
    rows = load_golden("isco_counterrotating.txt")
    assert E == pytest.approx(rows[-1, 2], abs=1e-12)
    assert L == pytest.approx(rows[-1, 3], abs=1e-12)
    rows = load_golden("isco_corotating.txt")
    assert 1 / math.sqrt(3) == pytest.approx(rows[-1, 2], abs=1e-12)
    assert 2 / math.sqrt(3) == pytest.approx(rows[-1, 3], abs=1e-12)


def test_schwarzschild_isco_and_forms(orc):
    """Section 4: r = 6M, E = sqrt(8/9), L = sqrt(12) M; COrbit/COrbit2 equal the
    general form at a = 0; dE/dr vanishes only at r = 6M, with the magnitude of the
    printed derivative (whose overall sign is read as a typo)."""
    E, L = orc.schwarzschild_circular(1.0, 6.0)
    assert E == pytest.approx(math.sqrt(8 / 9), rel=1e-15)
    assert L == pytest.approx(math.sqrt(12), rel=1e-15)
    assert orc.r_isco(1.0, 0.0, True) == pytest.approx(6.0, abs=1e-14)
    for r in (3.5, 4.0, 6.0, 7.3, 20.0):
        Eg, Lg = orc.circular_EL(1.0, 0.0, r, True)
        Es, Ls = orc.schwarzschild_circular(1.0, r)
        assert Eg == pytest.approx(Es, rel=1e-14)
        assert Lg == pytest.approx(Ls, rel=1e-14)
        h = 1e-5
        dE = (orc.schwarzschild_circular(1.0, r + h)[0] - orc.schwarzschild_circular(1.0, r - h)[0]) / (2 * h)
        printed = 1.0 * (6.0 - r) / (2 * r ** 1.5 * (r - 3.0) ** 1.5)
        assert abs(abs(dE) - abs(printed)) < 1e-8
    M = 2.5  # mass scaling
    E, L = orc.schwarzschild_circular(M, 6 * M)
    assert E == pytest.approx(math.sqrt(8 / 9), rel=1e-15)
    assert L == pytest.approx(math.sqrt(12) * M, rel=1e-15)


def test_r_kM_rows_match_ic_table(orc):
    """Section 5 IC table rows equal eq. gralorbits (Section 4) to the printed digits."""
    rows = load_golden("ic_rows.txt")
    for row in rows:
        k = row[1]
        pt = math.sqrt((k * k - 4 * k + 4) / (k * (k - 3)))
        pphi = k / math.sqrt(k - 3)
        assert abs(pt - row[4]) <= 5.01e-5
        assert abs(pphi - row[7]) <= 5.01e-5
        E, L = orc.schwarzschild_circular(1.0, k)
        assert E == pytest.approx(pt, rel=1e-14)
        assert L == pytest.approx(pphi, rel=1e-14)
        assert row[2] == pytest.approx(math.pi / 2, abs=5.1e-5)


def test_omega_and_period(orc):
    """Section 3, eq. omega / periodo: dphi/dtau of the circular orbit built by the
    oracle (u^phi = g^{phi nu} p_nu) equals the printed omega with p_t = +E; at a = 0
    the period is 2 pi r^2 / p_phi (Section 4)."""
    for a in (0.0, 0.3, 0.9):
        for prograde in (True, False):
            r = orc.r_isco(1.0, a, prograde) + 2.0
            E, L = orc.circular_EL(1.0, a, r, prograde)
            gi = orc.inverse_metric(1.0, a, r, math.pi / 2)
            uphi = gi[3, 0] * (-E) + gi[3, 3] * L
            omega = (-2 * a * E + (2 - r) * L) / (r * (2 * r - a * a - r * r))
            assert uphi == pytest.approx(omega, rel=1e-13)
            if a == 0.0:
                assert 2 * math.pi / uphi == pytest.approx(2 * math.pi * r * r / L, rel=1e-13)


def test_horizon(orc):
    """Section 3: r_+ = M + sqrt(M^2 - a^2); Section 5 stop radius 1 + sqrt(1 - a^2) at M = 1."""
    for a in (0.0, 0.5, 0.9, 0.998, 1.0):
        assert orc.r_horizon(1.0, a) == pytest.approx(1 + math.sqrt(1 - a * a), rel=1e-15)
        gi = orc.inverse_metric(1.0, a, orc.r_horizon(1.0, a) * (1 + 1e-6), 1.0)
        assert abs(gi[1, 1]) < 3e-6  # g^rr = Delta / rho^2 vanishes at the horizon
