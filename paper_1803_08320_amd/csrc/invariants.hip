// Invariants (E, L_z, Carter Q, g(u,u)) of each lane in FP64, from lane_invariants of
// monitor.hpp:
//   E   = -(g_tt u^t + g_tphi u^phi)            (conserved: dp_t/dtau = 0, Sections 3-4)
//   L_z = g_tphi u^t + g_phiphi u^phi           (conserved: dp_phi/dtau = 0)
//   Q   = (rho^2 u^theta)^2 + cos^2 [a^2 (mu^2 - E^2) + L_z^2 / sin^2],  mu^2 = -g(u,u)
//   g(u,u) = -1 timelike (Section 2, eq. geo), 0 null.
//
// State conversion between the formulations: p_mu = g_{mu nu} u^nu (lower) and
// u^mu = g^{mu nu} p_nu (raise), Section 2, eq. kerr.
#include "ic_device.hpp"
#include "internal.hpp"
#include "monitor.hpp"

namespace malbec {

namespace {

__global__ void __launch_bounds__(256) invariants_kernel(const double *__restrict__ state,
                                                         double *__restrict__ out,
                                                         const int32_t *__restrict__ st_of_lane,
                                                         int64_t n, StTable T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t sid = st_of_lane ? st_of_lane[i] : 0;
    if (sid < 0 || sid >= T.n_st) {  // invalid spacetime index
        for (int k = 0; k < 4; ++k) out[k * n + i] = __builtin_nan("");
        return;
    }
    const Spacetime S = T.st[sid];
    double y[8], v[4];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = state[k * n + i];
    lane_invariants<false>(S.M, S.a, y, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k * n + i] = v[k];
}

__global__ void __launch_bounds__(256) convert_kernel(double *__restrict__ state,
                                                      const int32_t *__restrict__ st_of_lane,
                                                      int64_t n, StTable T, int32_t to_momenta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t sid = st_of_lane ? st_of_lane[i] : 0;
    if (sid < 0 || sid >= T.n_st) {  // invalid spacetime index
        for (int k = 4; k < 8; ++k) state[k * n + i] = __builtin_nan("");
        return;
    }
    const Spacetime S = T.st[sid];
    const double M = S.M, a = S.a;
    const double r = state[1 * n + i], th = state[2 * n + i];
    const double v0 = state[4 * n + i], v1 = state[5 * n + i];
    const double v2 = state[6 * n + i], v3 = state[7 * n + i];
    double s, c;
    sincos(th, &s, &c);
    double w0, w1, w2, w3;
    if (to_momenta) {
        const double a2 = a * a, s2 = s * s, r2 = r * r;
        const double rho2 = r2 + a2 * c * c;
        const double Delta = r2 - 2.0 * M * r + a2;
        const double q = 2.0 * M * r / rho2;
        const double gtt = q - 1.0;
        const double gtp = -a * q * s2;
        const double gpp = (r2 + a2 + a2 * q * s2) * s2;
        w0 = gtt * v0 + gtp * v3;
        w1 = rho2 / Delta * v1;
        w2 = rho2 * v2;
        w3 = gtp * v0 + gpp * v3;
    } else {
        double itt, itp, ipp, irr, ithth;
        inverse_metric(M, a, r, s, c, itt, itp, ipp, irr, ithth);
        w0 = itt * v0 + itp * v3;
        w1 = irr * v1;
        w2 = ithth * v2;
        w3 = itp * v0 + ipp * v3;
    }
    state[4 * n + i] = w0;
    state[5 * n + i] = w1;
    state[6 * n + i] = w2;
    state[7 * n + i] = w3;
}

}  // namespace

int launch_convert(const StTable &T, const int32_t *st_of_lane, int64_t n, double *state,
                   int32_t to_momenta, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n, block)), dim3(block), 0, s, state,
                       T.n_st > 1 ? st_of_lane : nullptr, n, T, to_momenta);
    MALBEC_LAUNCH_CHECK("convert_kernel");
    return MALBEC_OK;
}

int launch_invariants(const StTable &T, const int32_t *st_of_lane, int64_t n, const double *state,
                      double *out, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(invariants_kernel, dim3(grid_for(n, block)), dim3(block), 0, s, state, out,
                       T.n_st > 1 ? st_of_lane : nullptr, n, T);
    MALBEC_LAUNCH_CHECK("invariants_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
