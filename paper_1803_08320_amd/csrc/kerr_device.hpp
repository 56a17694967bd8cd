// Device-side geodesic RK4 step and termination rules (gfx950).  The geodesic
// acceleration itself is in kerr_accel.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ham_accel.hpp"
#include "kerr_accel.hpp"
#include "sincos_table.hpp"

namespace malbec {

enum : int32_t { kActive = 0, kHorizon = 1, kEscape = 2, kDisk = 3, kNonfinite = 4, kBudget = 5 };

// The value x, hidden from the optimiser.  A work item's store computes its
// addresses from opaque(i): otherwise the compiler keeps the eight per-lane state
// addresses of the load alive across the whole step loop (16 VGPRs) instead of
// recomputing them once at the end.
__device__ __forceinline__ int64_t opaque(int64_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Per-spacetime constants held in registers or LDS.
struct Spacetime {
    double M, a, r_stop;  // r_stop = horizon_factor * r_+
    double r_zone;        // F32_KAHAN: r below which steps run in FP64
};

// sin and cos of theta + d from those of theta, for |d| <= kRotMax and
// |d| <= sin(theta) / 2: Taylor polynomials of sin d (through d^7) and cos d (through
// d^8), whose truncation is below 2e-17 relative there, and the angle-addition
// formulas (sin within 4 ulp; the second bound keeps sin(theta + d) >= sin(theta) / 2,
// so the addition does not cancel; cos is accurate in absolute terms, which is how the
// right-hand sides use it).  At the step sizes of the workloads (h <= 0.1 with
// |u^theta| well below 1) stage points stay within 0.04 of the step's start.
// SHORT: sin d through d^5 and cos d through d^4 for |d| <= kRotMaxShort, where the
// truncation is below 1.6e-20 absolute (d^7 / 7!) and 2.2e-17 (d^6 / 6!): with
// sin(theta) >= 2 |d| that is below 0.2 ulp relative in sin(theta + d).  Measured on
// gfx950 from the table base below, with half of 4M offsets at the limit: sin within
// 4.9 ulp (99.9 % within 2.0), cos within 1.3 ulp of 1.
constexpr double kRotMax = 0.04;
constexpr double kRotMaxShort = 0.005;

// a * b + c as one three-address v_fma_f64 with the constant addend c read from a
// scalar register pair.  Used for the polynomial steps below: the compiler's own
// choice there is the two-address v_fmac_f64 plus a copy of the constant into the
// destination, and a constant kept in vector registers costs two VGPRs per lane
// (or, under register pressure, moves inside the loop).  One scalar source per
// VOP3 instruction is within the constant-bus limit.  c must be the same in every
// lane (a literal constant): a scalar register holds one value per wavefront.
__device__ __forceinline__ double fma3c(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// Inverse factorials used by the rotation's Taylor polynomials.
constexpr double kF2 = 1.0 / 2.0, kF3 = 1.0 / 6.0, kF4 = 1.0 / 24.0, kF5 = 1.0 / 120.0,
                 kF6 = 1.0 / 720.0, kF7 = 1.0 / 5040.0, kF8 = 1.0 / 40320.0;

template <bool SHORT = false>
__device__ __forceinline__ void rotate(double s0, double c0, double d, double &s, double &c)
{
    const double d2 = d * d;
    // sin d = d + d^3 ps(d^2);  cos d = 1 + d^2 pc(d^2) (SHORT), 1 - d^2 pc(d^2)
    double ps, pc;
    if (SHORT) {
        ps = fma3c(d2, kF5, -kF3);
        pc = fma(d2, kF4, -kF2);  // -1/2 is an inline constant: kF4 takes the scalar operand
    } else {
        ps = fma3c(d2, -kF7, kF5);
        ps = fma3c(d2, ps, -kF3);
        pc = fma3c(d2, -kF8, kF6);
        pc = fma3c(d2, pc, -kF4);
        pc = fma(d2, pc, kF2);
    }
    const double sd = fma(d * d2, ps, d);
    const double cd = SHORT ? fma(d2, pc, 1.0) : fma(-d2, pc, 1.0);
    s = fma(s0, cd, c0 * sd);
    c = fma(c0, cd, -s0 * sd);
}

// Cody-Waite reduction x = theta - k pi/2, k = rint(theta / (pi/2)), with pi/2 split
// in two parts so that k * kPio2Hi is exact (|k| < 2^20), then minimax polynomials on
// |x| <= pi/4: sin x = x + x^3 P(x^2) with P of degree 5 and cos x = 1 - x^2 Q(x^2)
// with Q of degree 6, coefficients from the Remez exchange of gen_minimax.py
// (relative error of the rounded polynomials below 2.1e-17 and 6e-19; sin and cos
// measured within 1.5 ulp on gfx950).
__device__ __forceinline__ double sincos_reduce(double th, double &sx, double &cx)
{
    constexpr double kPio2Hi = 1.5707963267341256e+00;  // 33 significant bits of pi/2
    constexpr double kPio2Lo = 6.0771005065061922e-11;  // pi/2 - kPio2Hi
    constexpr double k2OverPi = 0.63661977236758134308;
    const double k = rint(th * k2OverPi);
    const double x = fma(-k, kPio2Lo, fma(-k, kPio2Hi, th));
    const double x2 = x * x;
    double ps = fma3c(x2, 1.5918142569704396e-10, -2.5051132049727266e-08);
    ps = fma3c(x2, ps, 2.7557316103657487e-06);
    ps = fma3c(x2, ps, -0.00019841269836761008);
    ps = fma3c(x2, ps, 0.00833333333333095);
    ps = fma3c(x2, ps, -0.16666666666666666);
    sx = fma(x * x2, ps, x);
    double pc = fma3c(x2, 1.1368006029792042e-11, -2.08758868745436e-09);
    pc = fma3c(x2, pc, 2.755731556728916e-07);
    pc = fma3c(x2, pc, -2.480158729369649e-05);
    pc = fma3c(x2, pc, 0.001388888888888078);
    pc = fma3c(x2, pc, -0.04166666666666664);
    pc = fma(x2, pc, 0.5);
    cx = fma(-x2, pc, 1.0);
    return k;
}

// Where the table is read from: the global copy, through the vector cache (TabGlobal),
// or a kernel's own copy in LDS (for kernels at one or two waves per SIMD, where too few
// other waves cover the cache's latency).  Both hold the same values, so results are the same.
struct TabGlobal {
    __device__ static __forceinline__ const double *row(uint32_t j) { return kTrigTab[j]; }
};
// The LDS copy: one array per kernel that uses it (a function-scope LDS variable), which
// every thread of the block fills (fill(), then a barrier) before any thread reads it.
struct TabLds {
    __device__ static __forceinline__ double (*table())[2]
    {
        __shared__ double t[kTrigTabN + 1][2];
        return t;
    }
    __device__ static __forceinline__ const double *row(uint32_t j) { return table()[j]; }
    __device__ static __forceinline__ void fill()
    {
        for (int k = threadIdx.x; k < 2 * (kTrigTabN + 1); k += blockDim.x)
            (&table()[0][0])[k] = (&kTrigTab[0][0])[k];
    }
};

// sin and cos of theta in [0, pi] (every accepted state has theta in (0, pi)) from the
// nearest angle of the table, theta_j = j pi / N: j = rint(theta N / pi), formed as
// the low word of theta N / pi + 1.5 * 2^52 (one rounding, to nearest), d = theta -
// theta_j with the split step (|d| <= pi / 2N < kRotMaxShort), and the short rotation
// of the correctly rounded (sin theta_j, cos theta_j) by d.  The rotation cancels by
// at most one bit (for j >= 1, sin theta >= sin theta_j / 2; j = 0 gives sin d
// itself): measured on gfx950 over 4M angles in [0, pi], sin within 2.3 ulp (99.9 %
// within 1.3) and cos within 0.8 ulp of 1, against 1.3 and 0.5 for the minimax
// evaluation of sincos_reduce, at 18 instructions instead of 29.  An angle outside
// [0, pi] (not a state the integrators produce) reads an entry within the table and
// gives meaningless values.
template <typename Tab = TabGlobal>
__device__ __forceinline__ void sincos_tab(double th, double &s, double &c)
{
    constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
    const double jb = fma(th, kTrigTabInvStep, kRound);
    const double j = jb - kRound;
    const double d = fma(-j, kTrigStepLo, fma(-j, kTrigStepHi, th));
    uint32_t ji = (uint32_t)__double_as_longlong(jb);
    ji = ji < (uint32_t)kTrigTabN ? ji : (uint32_t)kTrigTabN;
    const double *e = Tab::row(ji);
    rotate<true>(e[0], e[1], d, s, c);
}

// sin and cos of any moderate theta (|theta| < 1e6; stage points may leave (0, pi)):
// the same reduction with the quadrant k taken modulo 4.
__device__ __forceinline__ void sincos_any(double th, double &s, double &c)
{
    double sx, cx;
    const int q = ((int)sincos_reduce(th, sx, cx)) & 3;  // k mod 4, negative k too
    const double ss = (q & 1) ? cx : sx, cc = (q & 1) ? sx : cx;
    s = (q & 2) ? -ss : ss;
    c = ((q + 1) & 2) ? -cc : cc;
}

// Reference angle of the stage rotations: theta_b with its sin and cos (from the
// table) and the largest |d| = |theta - theta_b| that the rotation by d may take
// from it, min(kRotMax, sin(theta_b) / 2) (kRotMaxShort with the SHORT polynomials).
template <bool SHORT, typename Tab = TabGlobal>
struct TrigBase {
    double th, s, c, lim;
    __device__ __forceinline__ void set(double theta)
    {
        sincos_tab<Tab>(theta, s, c);
        th = theta;
        lim = fmin(SHORT ? kRotMaxShort : kRotMax, 0.5 * s);
    }
    // sin and cos of theta: the base pair rotated by the exactly computed d = theta -
    // theta_b, or a fresh evaluation when |d| exceeds the limit (a stage far from the
    // base, or a base close to a pole, where the rotation's cancellation would cost
    // relative accuracy in sin theta).
    __device__ __forceinline__ void at(double theta, double &so, double &co) const
    {
        const double d = theta - th;
        rotate<SHORT>(s, c, d, so, co);
        if (!(fabs(d) <= lim)) sincos_any(theta, so, co);
    }
};

// sin and cos of the theta of RK4 stage `stage`: stage 0 evaluates them afresh at the
// step's own theta and keeps them as the base; the later stages of the same step rotate
// that pair, so the trigonometry of a step depends on the step's start state alone (and
// rotations never chain from step to step).  SHORT: the short rotation polynomials,
// for fixed steps whose stage points stay within h |u^theta| <= 0.005 of the start
// (the Kerr bound-orbit workloads at h = 0.02: below 0.004); larger offsets fall back
// to a fresh evaluation.
template <bool SHORT, typename Tab = TabGlobal>
struct StageTrigT {
    TrigBase<SHORT, Tab> B;
    __device__ __forceinline__ void operator()(int stage, double th, double &s, double &c)
    {
        if (stage == 0) {
            B.set(th);
            s = B.s;
            c = B.c;
        } else {
            B.at(th, s, c);
        }
    }
};
using StageTrig = StageTrigT<false>;

// FP64 geodesic acceleration (Christoffel form) as a functor for rk4_stages.
template <typename Trig>
struct AccelF64T {
    double M, a;
    Trig trig;
    __device__ __forceinline__ void operator()(int stage, double r, double th, double ut, double ur,
                                               double uth, double uph, double &at, double &ar,
                                               double &ath, double &aph)
    {
        double s, c;
        trig(stage, th, s, c);
        kerr_accel<double>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};
using AccelF64 = AccelF64T<StageTrig>;

// One FP64 RK4 step (Christoffel form).  SHORT = true for the fixed-step integrators
// (small stage offsets), false for steps whose stage points move further (the camera's
// h = h0 max(1, r / h_r0)).  Tab: where the trigonometry table is read from.
template <bool SHORT = true, typename Tab = TabGlobal>
__device__ __forceinline__ void rk4_step_f64(const Spacetime &S, double h, const double y[8],
                                             double y1[8], double sr[3])
{
    AccelF64T<StageTrigT<SHORT, Tab>> f{S.M, S.a, {}};
    rk4_step(f, h, y, y1, sr);
}

// FP64 canonical right-hand side (Hamiltonian form) as a functor for rk4_ham_step.
template <typename Trig>
struct HamF64T {
    double M, a;
    const HamConst<double> &P;
    Trig trig;
    __device__ __forceinline__ void operator()(int stage, double r, double th, double pr, double pth,
                                               double &dt, double &dr, double &dth, double &dph,
                                               double &dpr, double &dpth)
    {
        double s, c;
        trig(stage, th, s, c);
        kerr_ham<double>(M, a, r, s, c, pr, pth, P, dt, dr, dth, dph, dpr, dpth);
    }
};

__device__ __forceinline__ void rk4_step_ham_f64(const Spacetime &S, const HamConst<double> &P,
                                                 double h, const double z[8], double z1[8],
                                                 double sr[3])
{
    HamF64T<StageTrigT<true>> f{S.M, S.a, P, {}};
    rk4_ham_step(f, h, z, z1, sr);
}

// A step result is usable when all components are finite and theta stays in (0, pi).
__device__ __forceinline__ bool usable(const double y[8])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) ok = ok && __builtin_isfinite(y[k]);
    return ok && (y[2] > 0.0) && (y[2] < 3.14159265358979323846);
}

// Termination after a step from y to y1 (integrate rules: no disk).  Returns the new
// status and whether y1 replaces y.
__device__ __forceinline__ int32_t terminate_f64(const Spacetime &S, double r_escape,
                                                 const double sr[3], const double y1[8],
                                                 bool &accept)
{
    accept = false;
    if (sr[0] <= S.r_stop || sr[1] <= S.r_stop || sr[2] <= S.r_stop) return kHorizon;
    if (!usable(y1)) return kNonfinite;
    accept = true;
    if (y1[1] <= S.r_stop) return kHorizon;
    if (y1[1] >= r_escape) return kEscape;
    return kActive;
}

// The common outcome of terminate_f64 tested first: true only when it would return
// kActive with y1 accepted (every stage radius above r_stop, y1's r inside
// (r_stop, r_escape) and theta inside (0, pi), which rule out a NaN there, and the
// other six components finite).  When it returns false (a NaN stage radius included)
// the caller applies terminate_f64, which may still give kActive.
__device__ __forceinline__ bool still_active_f64(const Spacetime &S, double r_escape,
                                                 const double sr[3], const double y1[8])
{
    bool ok = sr[0] > S.r_stop && sr[1] > S.r_stop && sr[2] > S.r_stop;
    ok = ok && y1[1] > S.r_stop && y1[1] < r_escape;
    ok = ok && y1[2] > 0.0 && y1[2] < 3.14159265358979323846;
    ok = ok && __builtin_isfinite(y1[0]) && __builtin_isfinite(y1[3]);
#pragma unroll
    for (int k = 4; k < 8; ++k) ok = ok && __builtin_isfinite(y1[k]);
    return ok;
}

}  // namespace malbec
