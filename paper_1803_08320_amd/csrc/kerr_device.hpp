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

// FP64 geodesic right-hand side as a functor for rk4_step.
struct AccelF64 {
    double M, a;
    __device__ __forceinline__ void operator()(double r, double th, double ut, double ur, double uth,
                                               double uph, double &at, double &ar, double &ath,
                                               double &aph) const
    {
        double s, c;
        sincos(th, &s, &c);
        kerr_accel<double>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};

__device__ __forceinline__ void rk4_step_f64(const Spacetime &S, double h, const double y[8],
                                             double y1[8], double sr[3])
{
    rk4_step(AccelF64{S.M, S.a}, h, y, y1, sr);
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
