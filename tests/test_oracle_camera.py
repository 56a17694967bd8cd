"""Pins of the oracle's camera (backward null rays, thin disk).

The paper only claims null-geodesic support; the image-plane model is a reading
(Bardeen image plane).  What pins it:
- the photon state is null and Theta(theta_obs) = beta^2;
- Schwarzschild capture boundary b = 3 sqrt(3) M (photon sphere r = 3M, the
  timelike circular-orbit limit of Section 4);
- Kerr a = 0.998 critical curve from spherical photon orbits R = R' = 0;
- flat-space (M -> 0) straight-line disk-crossing geometry.
"""
import math

import numpy as np
import pytest

NO_DISK = dict(disk_r_in=1.0, disk_r_out=-1.0)


def test_photon_state(orc):
    for a in (0.0, 0.9, 0.998):
        for alpha, beta in [(3.0, 2.0), (-7.5, 0.3), (0.2, -9.0)]:
            incl = math.radians(60)
            y = orc.ray_ic(1.0, a, 1000.0, incl, alpha, beta)
            inv = orc.invariants_one(1.0, a, -np.concatenate([-y[:4], y[4:]]))
            E, Lz, Q, norm = orc.invariants_one(1.0, a, y)
            # backward ray: 4-velocity negated, so E -> -1, L_z -> alpha sin i
            assert E == pytest.approx(-1.0, rel=1e-13)
            assert Lz == pytest.approx(alpha * math.sin(incl), rel=1e-12)
            assert abs(norm) < 1e-12
            Qw = beta ** 2 + math.cos(incl) ** 2 * (alpha ** 2 - a * a)
            assert Q == pytest.approx(Qw, rel=1e-9, abs=1e-9)
            Th = orc.potential_Theta(a, 1.0, -alpha * math.sin(incl), Qw, 0.0, incl)
            assert Th == pytest.approx(beta ** 2, rel=1e-12)
            assert y[5] < 0  # ingoing when traced backward
            assert np.sign(y[6]) == -np.sign(beta)
            del inv


def test_schwarzschild_shadow_radius(orc):
    bc = 3 * math.sqrt(3)
    incl = math.radians(60)
    phis = np.linspace(0, 2 * math.pi, 12, endpoint=False) + 0.1
    for fac, want in ((0.99, 1), (1.01, 2)):
        b = bc * fac
        st, steps, _ = orc.trace_rays(1.0, 0.0, 1000.0, incl, b * np.cos(phis), b * np.sin(phis),
                                      **NO_DISK)
        assert np.all(st == want), (fac, st)


def critical_curve(a, incl, n=9):
    """Spherical photon orbits of Kerr (E = 1): xi = L_z, eta = Q as functions of r."""
    M = 1.0
    r = np.linspace(1.0, 4.0, 20001)[1:]
    xi = -(r ** 3 - 3 * M * r ** 2 + a * a * r + a * a * M) / (a * (r - M))
    eta = -r ** 3 * (r ** 3 - 6 * M * r ** 2 + 9 * M * M * r - 4 * a * a * M) / (a * a * (r - M) ** 2)
    b2 = eta + a * a * math.cos(incl) ** 2 - xi ** 2 / math.tan(incl) ** 2
    ok = np.flatnonzero(b2 > 0)
    pick = ok[np.linspace(0, ok.size - 1, n).astype(int)]
    return r[pick], xi[pick], eta[pick], -xi[pick] / math.sin(incl), np.sqrt(b2[pick])


def test_kerr_critical_curve(orc):
    a, incl = 0.998, math.radians(60)
    r, xi, eta, alpha, beta = critical_curve(a, incl)
    # rays with L_z near 0 pass next to the poles, where a fixed step cannot resolve
    # the 1/sin^2 terms of Boyer-Lindquist coordinates; keep |L_z| >= 0.5
    keep = np.abs(xi) >= 0.5
    r, xi, eta, alpha, beta = r[keep], xi[keep], eta[keep], alpha[keep], beta[keep]
    assert keep.sum() >= 7
    for rr, x, e in zip(r, xi, eta):
        # R(r) = R'(r) = 0 on a spherical photon orbit
        R = orc.potential_R(1.0, a, 1.0, x, e, 0.0, rr)
        dR = (orc.potential_R(1.0, a, 1.0, x, e, 0.0, rr + 1e-6)
              - orc.potential_R(1.0, a, 1.0, x, e, 0.0, rr - 1e-6)) / 2e-6
        assert abs(R) < 1e-8 * rr ** 4 and abs(dR) < 1e-6 * rr ** 3
    for sgn in (1, -1):
        st_in, _, _ = orc.trace_rays(1.0, a, 1000.0, incl, 0.97 * alpha, 0.97 * sgn * beta, **NO_DISK)
        st_out, _, _ = orc.trace_rays(1.0, a, 1000.0, incl, 1.03 * alpha, 1.03 * sgn * beta, **NO_DISK)
        assert np.all(st_in == 1), st_in
        assert np.all(st_out == 2), st_out


def test_flat_space_disk_crossing(orc):
    """M -> 0: rays are straight lines.  The photon with image-plane point (alpha, beta)
    arrives at the observer x_obs = r_obs (sin i, 0, cos i) with unit direction
    p = p_r r_hat + (beta / r_obs) theta_hat - (alpha / r_obs) phi_hat (so that
    L_z = -alpha sin i and Theta(i) = beta^2); traced back it crosses z = 0 at
    x_obs - s p, s = z_obs / p_z."""
    M, incl, r_obs = 1e-6, math.radians(60), 1000.0
    alpha = np.array([3.0, -5.0, 1.0, 12.0, -0.5])
    beta = np.array([4.0, 2.0, -6.0, 1.5, -1.0])
    st, steps, hit = orc.trace_rays(M, 0.0, r_obs, incl, alpha, beta, h0=0.1, h_r0=10.0,
                                    disk_r_in=0.0, disk_r_out=100.0)
    assert np.all(st == 3)
    si, ci = math.sin(incl), math.cos(incl)
    rhat, thhat, phhat = np.array([si, 0, ci]), np.array([ci, 0, -si]), np.array([0, 1.0, 0])
    xo = r_obs * rhat
    for q in range(alpha.size):
        pth, pph = beta[q] / r_obs, -alpha[q] / r_obs
        p = math.sqrt(1 - pth ** 2 - pph ** 2) * rhat + pth * thhat + pph * phhat
        x = xo - (xo[2] / p[2]) * p
        assert hit[0, q] == pytest.approx(math.hypot(x[0], x[1]), rel=1e-3)
        dphi = math.remainder(hit[1, q] - math.atan2(x[1], x[0]), 2 * math.pi)
        assert abs(dphi) < 1e-3
    # outside [r_in, r_out] the ray passes through the plane and escapes
    st, _, hit = orc.trace_rays(M, 0.0, r_obs, incl, alpha, beta, disk_r_in=0.0, disk_r_out=1.0)
    assert np.all(st == 2) and np.all(np.isnan(hit))


def test_pixel_grid_matches_ray_list(orc):
    cam = dict(M=1.0, a=0.998, r_obs=1000.0, incl=math.radians(60), half_width=25.0, nx=16, ny=12,
               h0=0.1, h_r0=10.0, r_escape=1500.0, horizon_factor=1.01, disk_r_in=-1.0,
               disk_r_out=30.0, max_steps=100000)
    pix = np.arange(16 * 12)
    out = orc.trace_camera(cam, pix)
    i, j = pix % 16, pix // 16
    alpha = -25.0 + (i + 0.5) * 50.0 / 16
    beta = -25.0 + (j + 0.5) * 50.0 / 12
    st, steps, hit = orc.trace_rays(1.0, 0.998, 1000.0, cam["incl"], alpha, beta,
                                    disk_r_in=orc.r_isco(1.0, 0.998, True), disk_r_out=30.0)
    assert np.array_equal(st, out["status"]) and np.array_equal(steps, out["steps"])
    assert np.array_equal(np.isnan(hit), np.isnan(out["hit"]))
    assert set(np.unique(st)) <= {1, 2, 3}
    assert (st == 3).sum() > 0 and (st == 2).sum() > 0
    assert orc.r_isco(1.0, 0.998, True) == pytest.approx(1.2369706, abs=1e-6)
    # budget: a tiny step allowance stops every ray with BUDGET
    cam2 = dict(cam, max_steps=5)
    out2 = orc.trace_camera(cam2, pix[:10])
    assert np.all(out2["status"] == 5) and np.all(out2["steps"] == 5)
