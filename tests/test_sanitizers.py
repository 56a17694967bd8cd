"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc / g++ on the
CPU; no GPU code is built here): the oracle's C library, and the header-only
arithmetic that the kernels share with host builds (kerr_accel.hpp, ham_accel.hpp,
dp45.hpp), each driven through its entry points by a small program of its own.  Any
out-of-bounds access, use of uninitialised heap, signed overflow, misaligned or null
access, or leak ends the program with a sanitizer report and a non-zero status."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

ORACLE_DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int oracle_ic_constants(uint64_t, const double *, const int32_t *, int64_t, int64_t,
                        const double *, double, int64_t, double *, double *, int64_t *);
int oracle_ic_circular(uint64_t, double, double, int64_t, int64_t, double, double, double, int,
                       int, double *);
int oracle_integrate(const double *, const int32_t *, int64_t, double *, int32_t *, int32_t *,
                     double, int64_t, double, double, int, int);
int oracle_integrate_monitored(const double *, const int32_t *, int64_t, double *, int32_t *,
                               int32_t *, double, int64_t, double, double, int, int64_t, int,
                               double *, int);
int oracle_invariants(const double *, const int32_t *, int64_t, const double *, double *);
int oracle_integrate_adaptive(const double *, const int32_t *, int64_t, double *, double *,
                              double *, int32_t *, int32_t *, int32_t *, double, double, double,
                              double, double, double, int64_t, double, double, int);
void oracle_grid_fill_kerr(double, double, int64_t, int64_t, double, double, double, double,
                           double *);
int oracle_integrate_grid(int64_t, int64_t, double, double, double, double, const double *,
                          int64_t, double *, int32_t *, int32_t *, double, int64_t, double,
                          double, int);
int oracle_trace_camera(double, double, double, double, double, int64_t, int64_t, double, double,
                        double, double, double, double, int64_t, int64_t, const int64_t *,
                        int32_t *, int32_t *, double *, double *, int);
void oracle_tangent(double, double, double, int64_t, const double *, const double *, double *,
                    double *);
int oracle_grad_ic(double, double, double, int64_t, int64_t, const double *, const double *,
                   const double *, double *, double *, int);
double oracle_r_isco(double, double, int);
int oracle_inverse_metric(double, double, double, double, double *);
void oracle_christoffel(double, double, double, double, double *);
void oracle_metric_partials_complex_step(double, double, double, double, double *);

#define N 48
int main(void)
{
    const double Ma[4] = {1.0, 0.9, 1.0, 0.3};
    const double ranges[10] = {5.0, 50.0, 0.785, 2.356, 0.92, 0.98, 2.5, 4.5, 0.0, 12.0};
    int32_t *sol = malloc(N * sizeof(int32_t));
    for (int i = 0; i < N; ++i) sol[i] = i % 2;
    double *state = malloc(8 * N * sizeof(double)), *consts = malloc(4 * N * sizeof(double));
    int64_t *att = malloc(N * sizeof(int64_t));
    if (oracle_ic_constants(7, Ma, sol, N, 0, ranges, 1.0, 100000, state, consts, att) != 0) return 2;
    double *circ = malloc(8 * N * sizeof(double));
    oracle_ic_circular(3, 1.0, 0.0, N, 0, 6.5, 20.0, 1e-3, 1, 1, circ);
    int32_t *status = calloc(N, sizeof(int32_t)), *steps = calloc(N, sizeof(int32_t));
    double *s2 = malloc(8 * N * sizeof(double));
    memcpy(s2, state, 8 * N * sizeof(double));
    oracle_integrate(Ma, sol, N, s2, status, steps, 0.02, 300, 1.01, 1e4, 0, 0);
    double *inv = malloc(4 * N * sizeof(double));
    oracle_invariants(Ma, sol, N, s2, inv);
    double *mon = malloc(8 * N * sizeof(double));
    memcpy(s2, state, 8 * N * sizeof(double));
    memset(status, 0, N * sizeof(int32_t)); memset(steps, 0, N * sizeof(int32_t));
    oracle_integrate_monitored(Ma, sol, N, s2, status, steps, 0.02, 200, 1.01, 1e4, 0, 50, 1, mon, 0);
    double *tau = calloc(N, sizeof(double)), *hh = malloc(N * sizeof(double));
    int32_t *rej = calloc(N, sizeof(int32_t));
    for (int i = 0; i < N; ++i) hh[i] = 0.1;
    memcpy(s2, state, 8 * N * sizeof(double));
    memset(status, 0, N * sizeof(int32_t)); memset(steps, 0, N * sizeof(int32_t));
    oracle_integrate_adaptive(Ma, sol, N, s2, tau, hh, status, steps, rej, 30.0, 1e-10, 1e-10,
                              0.9, 0.2, 5.0, 100000, 1.01, 1e4, 0);
    const int64_t nr = 40, nth = 30;
    double *nodes = malloc(5 * nr * nth * sizeof(double));
    oracle_grid_fill_kerr(1.0, 0.9, nr, nth, 4.0, 1.0, 0.3, 0.09, nodes);
    memcpy(s2, state, 8 * N * sizeof(double));
    memset(status, 0, N * sizeof(int32_t)); memset(steps, 0, N * sizeof(int32_t));
    oracle_integrate_grid(nr, nth, 4.0, 1.0, 0.3, 0.09, nodes, N, s2, status, steps, 0.02, 100,
                          2.0, 40.0, 0);
    const int64_t nx = 8, ny = 6, np = nx * ny;
    int64_t *pix = malloc(np * sizeof(int64_t));
    for (int64_t p = 0; p < np; ++p) pix[p] = p;
    int32_t *cst = malloc(np * sizeof(int32_t)), *csp = malloc(np * sizeof(int32_t));
    double *hit = malloc(2 * np * sizeof(double)), *fs = malloc(8 * np * sizeof(double));
    oracle_trace_camera(1.0, 0.998, 1000.0, 1.047, 25.0, nx, ny, 0.1, 10.0, 1500.0, 1.01, 0.0,
                        30.0, 200000, np, pix, cst, csp, hit, fs, 0);
    double y[8], v[8], yo[8], dy[8];
    for (int k = 0; k < 8; ++k) { y[k] = state[k * N]; v[k] = 0.1 * (k + 1); }
    oracle_tangent(1.0, 0.9, 0.02, 50, y, v, yo, dy);
    double p[5 * 4], E[4], tgt[3 * 4], grad[5 * 4], loss[4];
    for (int i = 0; i < 4; ++i) {
        p[0 * 4 + i] = state[1 * N + i]; p[1 * 4 + i] = state[2 * N + i];
        p[2 * 4 + i] = state[5 * N + i]; p[3 * 4 + i] = state[6 * N + i];
        p[4 * 4 + i] = consts[1 * N + i]; E[i] = consts[i];
        for (int k = 0; k < 3; ++k) tgt[k * 4 + i] = 1.0 + k;
    }
    oracle_grad_ic(1.0, 0.7, 0.02, 50, 4, p, E, tgt, grad, loss, 0);
    double g16[16], G64[64], dg64[64];
    oracle_inverse_metric(1.0, 0.5, 7.0, 1.0, g16);
    oracle_christoffel(1.0, 0.5, 7.0, 1.0, G64);
    oracle_metric_partials_complex_step(1.0, 0.5, 7.0, 1.0, dg64);
    double s = oracle_r_isco(1.0, 0.9, 1) + oracle_r_isco(1.0, 0.9, 0);
    for (int i = 0; i < 8 * N; ++i) s += isfinite(s2[i]) ? 0.0 * s2[i] : 0.0;
    free(sol); free(state); free(consts); free(att); free(circ); free(status); free(steps);
    free(s2); free(inv); free(mon); free(tau); free(hh); free(rej); free(nodes); free(pix);
    free(cst); free(csp); free(hit); free(fs);
    printf("ok %.6f\n", s);
    return 0;
}
"""

HEADER_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include "dp45.hpp"
#include "ham_accel.hpp"
#include "kerr_accel.hpp"
struct Chr {
    double M, a, Ys[4][6];
    void operator()(int, double r, double th, double ut, double ur, double uth, double uph,
                    double &at, double &ar, double &ath, double &aph) const {
        malbec::kerr_accel<double>(M, a, r, std::sin(th), std::cos(th), ut, ur, uth, uph,
                                   at, ar, ath, aph);
    }
    double &Y(int st, int k) { return Ys[st][k]; }
    void keep() const {}
    void prepare(int, double) const {}
    void vjp(int, double r, double th, double ut, double ur, double uth, double uph, double bat,
             double bar, double bath, double baph, double &rb, double &thb, double ub[4]) const {
        double sb, cb;
        malbec::kerr_accel_vjp<double>(M, a, r, std::sin(th), std::cos(th), ut, ur, uth, uph, bat,
                                       bar, bath, baph, rb, sb, cb, ub);
        thb = sb * std::cos(th) - cb * std::sin(th);
    }
};
struct ChrF {
    float M, a;
    void operator()(int, float r, float th, float ut, float ur, float uth, float uph, float &at,
                    float &ar, float &ath, float &aph) const {
        malbec::kerr_accel<float>(M, a, r, std::sin(th), std::cos(th), ut, ur, uth, uph, at, ar,
                                  ath, aph);
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
int main() {
    double y[8] = {0.0, 9.0, 1.2, 0.0, 1.1, 0.05, 0.01, 0.03}, y1[8], sr[5], e[8];
    double s = 0.0;
    for (int rep = 0; rep < 200; ++rep) {
        Chr f{1.0, 0.9, {}};
        malbec::rk4_step(f, 0.02, y, y1, sr);
        double lam[8] = {1, 2, 3, 4, 5, 6, 7, 8};
        malbec::rk4_vjp(f, 0.02, y, lam);
        malbec::Deriv<double> k1, k7;
        for (int c = 0; c < 4; ++c) k1.u[c] = y[4 + c];
        f(0, y[1], y[2], y[4], y[5], y[6], y[7], k1.acc[0], k1.acc[1], k1.acc[2], k1.acc[3]);
        double yd[8];
        malbec::dp45_attempt(f, 0.1, y, k1, yd, e, k7, sr);
        Ham hm{1.0, 0.9, malbec::ham_const(0.9, -0.95, 3.0)};
        double z[8] = {0.0, 9.0, 1.2, 0.0, -0.95, 0.05, 0.3, 3.0}, z1[8];
        malbec::rk4_ham_step(hm, 0.02, z, z1, sr);
        float yf[8] = {0.f, 9.f, 1.2f, 0.f, 1.1f, 0.05f, 0.01f, 0.03f}, yf1[8], srf[3];
        ChrF ff{1.0f, 0.9f};
        malbec::rk4_step(ff, 0.02f, yf, yf1, srf);
        double ad[8];
        malbec::kerr_accel_direct<double>(1.0, 0.9, y[1], std::sin(y[2]), std::cos(y[2]), y[4],
                                          y[5], y[6], y[7], ad[0], ad[1], ad[2], ad[3]);
        for (int k = 0; k < 8; ++k) { s += lam[k] + yd[k] + z1[k] + yf1[k]; y[k] = y1[k]; }
        s += ad[0] + ad[1];
    }
    std::printf("ok %.6f\n", s);
    return std::isfinite(s) ? 0 : 3;
}
"""


def _have(tool):
    return shutil.which(tool) is not None


def _build_and_run(tmp_path, compiler, src_name, src, extra):
    src_path = tmp_path / src_name
    src_path.write_text(src)
    exe = tmp_path / (src_name + ".exe")
    r = subprocess.run([compiler] + SAN + [str(src_path)] + extra + ["-o", str(exe), "-lm"],
                       capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime unavailable: %s" % r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0 and run.stdout.startswith("ok"), (run.stdout[-500:], run.stderr[-4000:])
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-4000:]


@pytest.mark.skipif(not _have("gcc"), reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    """Every oracle entry point the tests use, on small inputs, one thread (the OpenMP
    pragmas are ignored without -fopenmp)."""
    _build_and_run(tmp_path, "gcc", "oracle_driver.c", ORACLE_DRIVER,
                   [os.path.join(ROOT, "oracle", "malbec_oracle.c"), "-std=gnu11",
                    "-ffp-contract=off", "-Wno-unknown-pragmas"])


@pytest.mark.skipif(not _have("g++"), reason="g++ not found")
def test_shared_headers_under_address_and_undefined_sanitizers(tmp_path):
    """The kernels' header-only arithmetic compiled for the host: RK4 steps (FP64 and
    FP32), the transposed RK4 step with the reverse-mode acceleration, a Dormand-Prince
    attempt and the Hamiltonian-form step."""
    _build_and_run(tmp_path, "g++", "headers_driver.cpp", HEADER_DRIVER,
                   ["-std=c++17", "-I", os.path.join(ROOT, "paper_1803_08320_amd", "csrc")])
