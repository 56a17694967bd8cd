// Device-side geodesic RK4 step and termination rules (gfx950).  The geodesic
// acceleration itself is in kerr_accel.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kerr_accel.hpp"

namespace malbec {

enum : int32_t { kActive = 0, kHorizon = 1, kEscape = 2, kDisk = 3, kNonfinite = 4, kBudget = 5 };

// Per-spacetime constants held in registers or LDS.
struct Spacetime {
    double M, a, r_stop;  // r_stop = horizon_factor * r_+
    double r_zone;        // F32_KAHAN: r below which steps run in FP64
};

// sin and cos of theta + d from those of theta, for |d| <= kRotMax: Taylor
// polynomials of sin d (through d^9) and cos d (through d^10), whose truncation is
// below 3e-18 there, and the angle-addition formulas.
constexpr double kRotMax = 0.125;

__device__ __forceinline__ void rotate(double s0, double c0, double d, double &s, double &c)
{
    const double d2 = d * d;
    double ps = fma(d2, 1.0 / 362880.0, -1.0 / 5040.0);
    ps = fma(d2, ps, 1.0 / 120.0);
    ps = fma(d2, ps, -1.0 / 6.0);
    const double sd = fma(d * d2, ps, d);
    double pc = fma(d2, -1.0 / 3628800.0, 1.0 / 40320.0);
    pc = fma(d2, pc, -1.0 / 720.0);
    pc = fma(d2, pc, 1.0 / 24.0);
    pc = fma(d2, pc, -0.5);
    const double cd = fma(d2, pc, 1.0);
    s = fma(s0, cd, c0 * sd);
    c = fma(c0, cd, -s0 * sd);
}

// FP64 geodesic right-hand side as a functor for rk4_stages.  Stage 0 evaluates
// sincos(theta); the later stages of the same step, whose theta differs from the
// stage-0 theta by an exactly computed small d, rotate that pair instead.
struct AccelF64 {
    double M, a;
    double th0, s0, c0;
    __device__ __forceinline__ void operator()(int stage, double r, double th, double ut, double ur,
                                               double uth, double uph, double &at, double &ar,
                                               double &ath, double &aph)
    {
        double s, c;
        const double d = th - th0;
        if (stage == 0 || !(fabs(d) <= kRotMax)) {
            sincos(th, &s, &c);
            if (stage == 0) { th0 = th; s0 = s; c0 = c; }
        } else {
            rotate(s0, c0, d, s, c);
        }
        kerr_accel<double>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};

__device__ __forceinline__ void rk4_step_f64(const Spacetime &S, double h, const double y[8],
                                             double y1[8], double sr[3])
{
    AccelF64 f{S.M, S.a, 0.0, 0.0, 1.0};
    rk4_step(f, h, y, y1, sr);
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

}  // namespace malbec
