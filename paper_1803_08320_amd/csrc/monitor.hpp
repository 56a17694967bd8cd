// Invariant monitor inside the step loop.
//
// The conserved quantities of a Kerr geodesic: E = -p_t and L_z = p_phi (the metric
// of Section 2, eq. kerr, depends on neither t nor phi; Sections 3-4 use exactly
// this), the norm g(u,u) = g^{mu nu} p_mu p_nu (-1 timelike, 0 null; the constraint
// of eq. geo) and Carter's constant
//   Q = p_theta^2 + cos^2 theta [a^2 (mu^2 - E^2) + L_z^2 / sin^2 theta],
//   mu^2 = -g(u,u), p_theta = rho^2 u^theta.
// lane_invariants() evaluates them for a state of either formulation: (x, u) with the
// metric lowering u, or (x, p) with p_t, p_phi read directly and the norm from the
// inverse metric.  MonProg wraps the work item of an integrator (the Prog interface
// of persistent.hpp) and, after every step whose global index (the lane's step count
// over all calls) is a multiple of K, folds |I - I_0| into a running maximum per
// invariant.
#pragma once

#include "ic_device.hpp"
#include "kerr_device.hpp"

namespace malbec {

// (E, L_z, Q, g(u,u)) of the state y (component-major values of one lane).
// HAM = false: y = (x^mu, u^mu); HAM = true: y = (x^mu, p_mu).
template <bool HAM>
__device__ __forceinline__ void lane_invariants(double M, double a, const double y[8], double out[4])
{
    const double r = y[1];
    double s, c;
    sincos_any(y[2], s, c);
    const double a2 = a * a, s2 = s * s, r2 = r * r;
    const double rho2 = r2 + a2 * c * c;
    double E, Lz, norm, pth;
    if (HAM) {
        double itt, itp, ipp, irr, ithth;
        inverse_metric(M, a, r, s, c, itt, itp, ipp, irr, ithth);
        E = -y[4];
        Lz = y[7];
        norm = itt * y[4] * y[4] + 2.0 * itp * y[4] * y[7] + ipp * y[7] * y[7] +
               irr * y[5] * y[5] + ithth * y[6] * y[6];
        pth = y[6];
    } else {
        const double ut = y[4], ur = y[5], uth = y[6], uph = y[7];
        const double Delta = r2 - 2.0 * M * r + a2;
        const double q = 2.0 * M * r / rho2;
        const double gtt = q - 1.0;
        const double gtp = -a * q * s2;
        const double gpp = (r2 + a2 + a2 * q * s2) * s2;
        const double grr = rho2 / Delta;
        norm = gtt * ut * ut + 2.0 * gtp * ut * uph + gpp * uph * uph + grr * ur * ur +
               rho2 * uth * uth;
        E = -(gtt * ut + gtp * uph);
        Lz = gtp * ut + gpp * uph;
        pth = rho2 * uth;
    }
    out[0] = E;
    out[1] = Lz;
    out[2] = pth * pth + c * c * (a2 * (-norm - E * E) + Lz * Lz / s2);
    out[3] = norm;
}

// Monitor buffer of a call: mon[k n + i], k = 0..3 the reference invariants I_0 of
// lane i, k = 4..7 the running maxima of |I - I_0|.
struct MonArgs {
    double *mon;
    const int32_t *steps;  // the lanes' step counts at the start of the launch
    int64_t n;
    int32_t every;         // K >= 1
    int32_t reset;         // 1: I_0 from the state at load, maxima cleared
};

// Base provides the Prog interface plus
//   static void state64(const Lane&, double y[8])   -- the lane's state in FP64
//   Lane::S                                         -- the lane's Spacetime
// While a lane is in flight its I_0 and running maxima live in the thread's slot of
// an LDS array (8 doubles per thread, the block's threads interleaved: kMonLanes
// apart), not in registers and not in the monitor buffer: the buffer is read when the
// lane is taken (unless reset) and written when it is stored, once per launch, so
// the monitored steps add no memory traffic (the persistent kernels take lanes
// scattered over the batch, where each 8-byte access of the component-major buffer
// would fetch a cache line of its own).
constexpr int kMonLanes = 256;  // block size bound of the monitored kernels
template <class Base, bool HAM>
struct MonProg {
    Base base;
    MonArgs M;
    double *slot;  // this thread's LDS slot: value k at slot[k * kMonLanes]
    struct Lane {
        typename Base::Lane b;
        int64_t i;     // the lane's index in the batch
        int32_t left;  // steps until the next monitored one
    };
    __device__ __forceinline__ bool load(int64_t i, Lane &L)
    {
        const int32_t s0 = M.steps[i];  // read before the base's store can change it
        if (!base.load(i, L.b)) return false;
        if (M.reset) {
            double y[8], I0[4];
            Base::state64(L.b, y);
            lane_invariants<HAM>(L.b.S.M, L.b.S.a, y, I0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                slot[k * kMonLanes] = I0[k];
                slot[(4 + k) * kMonLanes] = 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) slot[k * kMonLanes] = M.mon[k * M.n + i];
        }
        L.i = i;
        const int32_t r = s0 % M.every;
        L.left = M.every - (r < 0 ? r + M.every : r);
        return true;
    }
    __device__ __forceinline__ bool step(Lane &L)
    {
        const bool done = base.step(L.b);
        if (--L.left == 0) {
            L.left = M.every;
            double y[8], I[4];
            Base::state64(L.b, y);
            lane_invariants<HAM>(L.b.S.M, L.b.S.a, y, I);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double &D = slot[(4 + k) * kMonLanes];
                D = fmax(D, fabs(I[k] - slot[k * kMonLanes]));
            }
        }
        return done;
    }
    __device__ __forceinline__ void store(int64_t item, const Lane &L)
    {
        base.store(item, L.b);
        const int64_t i = opaque(L.i);
#pragma unroll
        for (int k = M.reset ? 0 : 4; k < 8; ++k) M.mon[k * M.n + i] = slot[k * kMonLanes];
    }
};

}  // namespace malbec
