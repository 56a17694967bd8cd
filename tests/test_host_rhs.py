"""The kernels' right-hand sides and RK4 steps, compiled for the host with g++ from
the same headers the GPU kernels include (csrc/kerr_accel.hpp, csrc/ham_accel.hpp),
against the oracle: a CPU check of the kernels' algebra (the GPU tests check the
compiled kernels themselves)."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

from conftest import ROOT

KERR_RANGES = ((5.0, 50.0), (math.pi / 4, 3 * math.pi / 4), (0.92, 0.98), (2.5, 4.5), (0.0, 12.0))

SRC = r"""
#include <cmath>
#include "dp45.hpp"
#include "ham_accel.hpp"
#include "kerr_accel.hpp"
struct Chr {
    double M, a;
    void operator()(int, double r, double th, double ut, double ur, double uth, double uph,
                    double &at, double &ar, double &ath, double &aph) const {
        malbec::kerr_accel<double>(M, a, r, std::sin(th), std::cos(th), ut, ur, uth, uph,
                                   at, ar, ath, aph);
    }
};
struct Ham {
    double M, a;
    malbec::HamConst<double> P;
    void operator()(int, double r, double th, double pr, double pth, double &dt, double &dr,
                    double &dth, double &dph, double &dpr, double &dpth) const {
        malbec::kerr_ham<double>(M, a, r, std::sin(th), std::cos(th), pr, pth, P, dt, dr, dth,
                                 dph, dpr, dpth);
    }
};
extern "C" void chr_rhs(double M, double a, const double *y, double *f) {
    f[0] = y[4]; f[1] = y[5]; f[2] = y[6]; f[3] = y[7];
    Chr{M, a}(0, y[1], y[2], y[4], y[5], y[6], y[7], f[4], f[5], f[6], f[7]);
}
extern "C" void chr_rhs_direct(double M, double a, const double *y, double *f) {
    f[0] = y[4]; f[1] = y[5]; f[2] = y[6]; f[3] = y[7];
    malbec::kerr_accel_direct<double>(M, a, y[1], std::sin(y[2]), std::cos(y[2]), y[4], y[5],
                                      y[6], y[7], f[4], f[5], f[6], f[7]);
}
// The acceleration with its transposed Jacobian, for rk4_vjp (host trigonometry).
struct ChrVjp {
    double M, a;
    void operator()(int, double r, double th, double ut, double ur, double uth, double uph,
                    double &at, double &ar, double &ath, double &aph) const {
        malbec::kerr_accel<double>(M, a, r, std::sin(th), std::cos(th), ut, ur, uth, uph,
                                   at, ar, ath, aph);
    }
    double Ys[4][6];
    double &Y(int st, int k) { return Ys[st][k]; }
    void keep() const {}
    void prepare(int, double) const {}
    void vjp(int, double r, double th, double ut, double ur, double uth, double uph, double bat,
             double bar, double bath, double baph, double &rb, double &thb, double ub[4]) const {
        const double s = std::sin(th), c = std::cos(th);
        double sb, cb;
        malbec::kerr_accel_vjp<double>(M, a, r, s, c, ut, ur, uth, uph, bat, bar, bath, baph,
                                       rb, sb, cb, ub);
        thb = sb * c - cb * s;
    }
};
// y^T-side of one acceleration: out = (d a / d(r, theta, u))^T b, 6 values
extern "C" void chr_accel_vjp(double M, double a, const double *y, const double *b, double *out) {
    double ub[4];
    ChrVjp{M, a}.vjp(0, y[1], y[2], y[4], y[5], y[6], y[7], b[0], b[1], b[2], b[3], out[0],
                     out[1], ub);
    for (int k = 0; k < 4; ++k) out[2 + k] = ub[k];
}
extern "C" void chr_step_vjp(double M, double a, double h, const double *y, double *lam) {
    ChrVjp f{M, a};
    malbec::rk4_vjp(f, h, y, lam);
}
extern "C" void ham_rhs(double M, double a, const double *z, double *f) {
    Ham h{M, a, malbec::ham_const(a, z[4], z[7])};
    h(0, z[1], z[2], z[5], z[6], f[0], f[1], f[2], f[3], f[5], f[6]);
    f[4] = 0.0; f[7] = 0.0;
}
extern "C" void chr_step(double M, double a, double h, const double *y, double *y1) {
    Chr f{M, a};
    double sr[3];
    malbec::rk4_step(f, h, y, y1, sr);
}
extern "C" void dp45(double M, double a, double h, const double *y, double *y1, double *e) {
    Chr f{M, a};
    malbec::Deriv<double> k1, k7;
    for (int c = 0; c < 4; ++c) k1.u[c] = y[4 + c];
    f(0, y[1], y[2], y[4], y[5], y[6], y[7], k1.acc[0], k1.acc[1], k1.acc[2], k1.acc[3]);
    double sr[5];
    malbec::dp45_attempt(f, h, y, k1, y1, e, k7, sr);
}
extern "C" void ham_step(double M, double a, double h, const double *z, double *z1) {
    Ham f{M, a, malbec::ham_const(a, z[4], z[7])};
    double sr[3];
    malbec::rk4_ham_step(f, h, z, z1, sr);
}
"""


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostrhs")
    src = d / "host_rhs.cpp"
    src.write_text(SRC)
    so = d / "libhost_rhs.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-I", os.path.join(ROOT, "paper_1803_08320_amd", "csrc"), str(src), "-o",
                    str(so)], check=True)
    lib = C.CDLL(str(so))
    dp = C.POINTER(C.c_double)
    for name in ("chr_rhs", "chr_rhs_direct", "ham_rhs"):
        getattr(lib, name).argtypes = [C.c_double, C.c_double, dp, dp]
    for name in ("chr_step", "ham_step", "chr_step_vjp"):
        getattr(lib, name).argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    lib.chr_accel_vjp.argtypes = [C.c_double, C.c_double, dp, dp, dp]
    lib.dp45.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp, dp]
    return lib


def _p(x):
    return x.ctypes.data_as(C.POINTER(C.c_double))


def sample_states(orc, a, n, seed):
    """Bound-orbit states of the Kerr draws, with r pulled towards the hole."""
    rc, s0, _, _ = orc.ic_constants(seed, [(1.0, a)], n, KERR_RANGES)
    rng = np.random.default_rng(seed)
    rp = 1.0 + math.sqrt(1.0 - a * a)
    s0[1] = 1.2 * rp + (s0[1] - 1.2 * rp) * rng.uniform(0.02, 1.0, n)
    return s0


def lower(orc, a, y):
    z = y.copy()
    z[4:] = orc.metric(1.0, a, y[1], y[2]) @ y[4:]
    return z


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.998])
def test_right_hand_sides_match_oracle(orc, host, a):
    """Both evaluations of the Christoffel acceleration (the regrouped one the kernels
    use and the direct coefficients-then-contraction one the adjoint differentiates) and
    Hamilton's equations, against the oracle's generic Christoffel contraction and its
    canonical equations; the sample includes states near the horizon and near the poles."""
    s0 = sample_states(orc, a, 200, 51)
    rng = np.random.default_rng(54)
    pole = rng.uniform(0.02, 0.3, 40)
    s0[2, :40] = np.where(np.arange(40) % 2 == 0, pole, math.pi - pole)
    for i in range(s0.shape[1]):
        y = np.ascontiguousarray(s0[:, i])
        ref = orc.rhs(1.0, a, y)
        for fn in (host.chr_rhs, host.chr_rhs_direct):
            f = np.zeros(8)
            fn(1.0, a, _p(y), _p(f))
            assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))
        z = lower(orc, a, y)
        fh = np.zeros(8)
        host.ham_rhs(1.0, a, _p(z), _p(fh))
        refh = orc.rhs_hamiltonian(1.0, a, z)
        assert np.max(np.abs(fh - refh)) <= 1e-13 * np.max(np.abs(refh))
        assert fh[4] == 0.0 and fh[7] == 0.0


@pytest.mark.parametrize("a", [0.0, 0.9])
def test_rk4_steps_match_oracle(orc, host, a):
    s0 = sample_states(orc, a, 64, 52)
    ref, _, _ = orc.integrate([(1.0, a)], s0, 0.02, 1, r_escape=1e300, horizon_factor=0.0)
    z0 = np.stack([lower(orc, a, s0[:, i]) for i in range(s0.shape[1])], axis=1)
    refh, _, _ = orc.integrate([(1.0, a)], z0, 0.02, 1, hamiltonian=True, r_escape=1e300,
                               horizon_factor=0.0)
    for i in range(s0.shape[1]):
        y1 = np.zeros(8)
        host.chr_step(1.0, a, 0.02, _p(np.ascontiguousarray(s0[:, i])), _p(y1))
        assert np.max(np.abs(y1 - ref[:, i]) / (np.abs(ref[:, i]) + 1.0)) <= 1e-14
        z1 = np.zeros(8)
        host.ham_step(1.0, a, 0.02, _p(np.ascontiguousarray(z0[:, i])), _p(z1))
        assert np.max(np.abs(z1 - refh[:, i]) / (np.abs(refh[:, i]) + 1.0)) <= 1e-14
        assert z1[4] == z0[4, i] and z1[7] == z0[7, i]


@pytest.mark.parametrize("a", [0.0, 0.9])
def test_dp45_attempt_matches_oracle(orc, host, a):
    """One Dormand-Prince attempt: 5th-order result and embedded error estimate."""
    s0 = sample_states(orc, a, 64, 53)
    for i in range(s0.shape[1]):
        y = np.ascontiguousarray(s0[:, i])
        for h in (0.05, 0.8):
            y1, e = np.zeros(8), np.zeros(8)
            host.dp45(1.0, a, h, _p(y), _p(y1), _p(e))
            ry1, re = orc.dp45_attempt(1.0, a, h, y)
            assert np.max(np.abs(y1 - ry1) / (np.abs(ry1) + 1.0)) <= 1e-14
            # e is a difference of two solutions (cancellation): its rounding is
            # absolute, ~ h ulp(f)
            assert np.max(np.abs(e - re)) <= 1e-14 * h * (np.max(np.abs(y[4:])) + 1.0)


@pytest.mark.parametrize("a", [0.0, 0.7, 0.998])
def test_acceleration_vjp_matches_complex_step(orc, host, a):
    """The reverse mode of the regrouped acceleration (the adjoint's transposed Jacobian)
    against the oracle: each column of d a / d(r, theta, u) is a central difference of
    the oracle's right-hand side with a step that balances truncation and rounding
    (1e-5 of the coordinate: error ~1e-10 of the column's scale), and b^T J is compared
    column by column."""
    s0 = sample_states(orc, a, 60, 55)
    rng = np.random.default_rng(56)
    for i in range(s0.shape[1]):
        y = np.ascontiguousarray(s0[:, i])
        b = np.ascontiguousarray(rng.standard_normal(4))
        out = np.zeros(6)
        host.chr_accel_vjp(1.0, a, _p(y), _p(b), _p(out))
        for j, k in enumerate((1, 2, 4, 5, 6, 7)):
            e = 1e-5 * max(abs(y[k]), 1e-2)
            yp, ym = y.copy(), y.copy()
            yp[k] += e
            ym[k] -= e
            col = (orc.rhs(1.0, a, yp)[4:] - orc.rhs(1.0, a, ym)[4:]) / (2 * e)
            want = b @ col
            scale = np.abs(b) @ np.abs(col) + 1e-300
            assert abs(out[j] - want) <= 1e-7 * scale + 1e-12, (i, k, out[j], want)


@pytest.mark.parametrize("a", [0.0, 0.9])
def test_rk4_vjp_is_the_transpose_of_the_oracle_tangent(orc, host, a):
    """<lam, J v> = <J^T lam, v> for one RK4 step, J v from the oracle's complex-step
    tangent (exact up to rounding) and J^T lam from the transposed step that the
    adjoint kernel runs (rk4_vjp with the reverse-mode acceleration)."""
    s0 = sample_states(orc, a, 64, 57)
    rng = np.random.default_rng(58)
    for i in range(s0.shape[1]):
        y = np.ascontiguousarray(s0[:, i])
        v = rng.standard_normal(8)
        lam = rng.standard_normal(8)
        _, jv = orc.tangent(1.0, a, 0.02, 1, y, v)
        jt = lam.copy()
        host.chr_step_vjp(1.0, a, 0.02, _p(y), _p(jt))
        lhs, rhs_ = lam @ jv, jt @ v
        scale = np.abs(lam) @ np.abs(jv) + np.abs(jt) @ np.abs(v)
        assert abs(lhs - rhs_) <= 1e-13 * scale, (i, lhs, rhs_)
