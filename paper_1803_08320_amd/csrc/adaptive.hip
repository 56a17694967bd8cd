// Adaptive FP64 integration with the Dormand-Prince 5(4) pair (csrc/dp45.hpp) and a
// per-lane step size.  Each lane advances its affine parameter tau towards tau_end
// in attempts; an attempt is accepted when the weighted RMS of the embedded error
// estimate is <= 1, and the next step size follows the standard controller
// h_new = h min(facmax', max(facmin, fac err^(-1/5))) (facmax' = 1 right after a
// rejection).  The last attempt of a call is shortened to land on tau_end.  Stop
// rules as in malbec_integrate, applied to attempts: a stage point at r <= r_stop
// ends the lane as HORIZON and a non-finite or off-range result or error as
// NONFINITE (start state kept); an accepted step that reaches r <= r_stop or
// r >= r_escape ends it as HORIZON or ESCAPE; max_attempts attempts in one call
// without reaching tau_end end it as BUDGET.
//
// Lanes need different numbers of attempts, so the work-queue driver of
// persistent.hpp (one attempt per "step") keeps the wavefronts full; a
// one-thread-per-lane kernel gives the same bits.  The queue hands out work item k as
// lane order[k] when a work order is given (schedule.hip: smallest periapsis, i.e.
// longest expected lane, first), else lane k.
#include "dp45.hpp"
#include "internal.hpp"
#include "persistent.hpp"

namespace malbec {

namespace {

struct AdArgs {
    int64_t n;
    double *state;
    double *tau;
    double *h;
    int32_t *status;
    int32_t *steps;
    int32_t *rejects;
    const int32_t *st_of_lane;
    const uint32_t *order;  // persistent: lane of work item k (nullptr: k itself)
    double tau_end, rtol, atol, fac, facmin, facmax, r_escape;
    int64_t max_attempts;
};

// err^(-1/5) for err > 0: a single-precision estimate from the hardware log2 and
// exp2, then two Newton steps for err y^5 = 1 in FP64, y <- y (6 - err y^5) / 5, each
// squaring the estimate's relative error (~1e-6 -> 1e-12 -> below rounding).  Outside
// the single-precision range the estimate is taken at the range's edge; the step-size
// factor is then clamped to facmin or facmax either way.
__device__ __forceinline__ double rpow5(double err)
{
    const float ef = (float)fmin(fmax(err, 1e-37), 1e37);
    double y = (double)__builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(ef));
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double y2 = y * y;
        y = (y * 0.2) * fma(-err, y2 * y2 * y, 6.0);
    }
    return y;
}

// The acceleration with the trigonometry table read from the block's LDS copy: at the
// kernels' two waves per SIMD the vector cache's latency would otherwise show.
using AccelAd = AccelF64T<StageTrigT<false, TabLds>>;

struct AdProg {
    const AdArgs &A;
    const Spacetime *table;  // LDS copy of the spacetimes (mixed batch)
    bool multi;
    int32_t n_st;
    Spacetime st0;           // the one spacetime of a single-spin batch (kernel argument)
    struct Lane {
        double y[8];
        double k1a[4];  // acceleration at y (k1 = (y[4..7], k1a): its velocity part is y's)
        int32_t sid;    // spacetime index (its parameters are read when needed)
        double tau, h;
        int32_t st, acc, rej;  // acc + rej = the attempts of this call so far
        bool capped;           // the last attempt was rejected: no growth in the next
    };
    __device__ __forceinline__ Spacetime space(const Lane &L) const { return multi ? table[L.sid] : st0; }
    __device__ __forceinline__ void deriv0(Lane &L)
    {
        const Spacetime S = space(L);
        AccelAd f{S.M, S.a, {}};
        f(0, L.y[1], L.y[2], L.y[4], L.y[5], L.y[6], L.y[7], L.k1a[0], L.k1a[1], L.k1a[2],
          L.k1a[3]);
    }
    __device__ __forceinline__ int64_t lane_of(int64_t item) const
    {
        return A.order ? (int64_t)A.order[item] : item;
    }
    __device__ __forceinline__ bool load(int64_t item, Lane &L)
    {
        const int64_t i = lane_of(item);
        L.st = A.status[i];
        if (L.st != kActive) return false;
        int32_t sid = 0;
        if (multi) {
            sid = A.st_of_lane[i];
            if (sid < 0 || sid >= n_st) {
                A.status[i] = kNonfinite;
                return false;
            }
        }
        L.sid = sid;
        L.tau = A.tau[i];
        if (!(L.tau < A.tau_end)) return false;
#pragma unroll
        for (int k = 0; k < 8; ++k) L.y[k] = A.state[k * A.n + i];
        L.h = A.h[i];
        L.capped = false;
        L.acc = 0;
        L.rej = 0;
        deriv0(L);
        return true;
    }
    // one attempt; true when the lane is finished for this call
    __device__ __forceinline__ bool step(Lane &L)
    {
        if ((int64_t)L.acc + L.rej == A.max_attempts) {
            L.st = kBudget;
            return true;
        }
        double hh = L.h;
        bool last = false;
        if (L.tau + hh >= A.tau_end) {
            hh = A.tau_end - L.tau;
            last = true;
        }
        // stage 0 of the rotation base is the start point: sin and cos evaluated fresh
        const Spacetime S = space(L);
        AccelAd f{S.M, S.a, {}};
        {
            double s, c;
            f.trig(0, L.y[2], s, c);
        }
        double y1[8], e[8], sr[5];
        Deriv<double> k1, k7;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            k1.u[c] = L.y[4 + c];
            k1.acc[c] = L.k1a[c];
        }
        dp45_attempt(f, hh, L.y, k1, y1, e, k7, sr);
        const double rs = S.r_stop;
        if (sr[0] <= rs || sr[1] <= rs || sr[2] <= rs || sr[3] <= rs || sr[4] <= rs) {
            L.st = kHorizon;
            return true;
        }
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double sc = fma(A.rtol, fmax(fabs(L.y[c]), fabs(y1[c])), A.atol);
            const double q = e[c] * recip(sc);
            sum = fma(q, q, sum);
        }
        const double err = sqrt(sum * 0.125);
        if (!usable(y1) || !__builtin_isfinite(err)) {
            L.st = kNonfinite;
            return true;
        }
        const double grow = err > 0.0 ? A.fac * rpow5(err) : A.facmax;
        if (err <= 1.0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) L.y[c] = y1[c];
#pragma unroll
            for (int c = 0; c < 4; ++c) L.k1a[c] = k7.acc[c];
            L.tau = last ? A.tau_end : L.tau + hh;
            ++L.acc;
            L.h = hh * fmin(L.capped ? 1.0 : A.facmax, fmax(A.facmin, grow));
            L.capped = false;
            if (L.y[1] <= rs) L.st = kHorizon;
            else if (L.y[1] >= A.r_escape) L.st = kEscape;
        } else {
            ++L.rej;
            L.h = hh * fmin(1.0, fmax(A.facmin, grow));
            L.capped = true;
        }
        return L.st != kActive || !(L.tau < A.tau_end);
    }
    __device__ __forceinline__ void store(int64_t item, const Lane &L)
    {
        // the index is laundered so that the addresses of the loads are not kept
        // live across the attempts for reuse here
        const int64_t i = lane_of(opaque(item));
#pragma unroll
        for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = L.y[k];
        A.tau[i] = L.tau;
        A.h[i] = L.h;
        A.status[i] = L.st;
        A.steps[i] += L.acc;
        A.rejects[i] += L.rej;
    }
};

template <bool MULTI>
__global__ void __launch_bounds__(256) dp45_kernel(AdArgs A, StTable T)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    TabLds::fill();
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    AdProg P{A, lds_st, MULTI, T.n_st, T.st[0]};
    AdProg::Lane L;
    if (!P.load(i, L)) return;
    while (!P.step(L)) {
    }
    P.store(i, L);
}

template <bool MULTI>
__global__ void __launch_bounds__(256) dp45_persistent_kernel(AdArgs A, StTable T,
                                                              unsigned long long *counter,
                                                              int32_t chunk)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    TabLds::fill();
    __syncthreads();
    AdProg P{A, lds_st, MULTI, T.n_st, T.st[0]};
    persistent_loop(P, A.n, counter, chunk);
}

}  // namespace

int launch_adaptive(const malbec_adaptive &ad, const StTable &T, const int32_t *st_of_lane,
                    int64_t n, double *state, double *tau, double *h, int32_t *status,
                    int32_t *steps, int32_t *rejects, const uint32_t *order, void *ws,
                    hipStream_t s)
{
    const int block = ad.block > 0 ? ad.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    AdArgs A;
    A.n = n;
    A.state = state;
    A.tau = tau;
    A.h = h;
    A.status = status;
    A.steps = steps;
    A.rejects = rejects;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.order = ad.persistent ? order : nullptr;
    A.tau_end = ad.tau_end;
    A.rtol = ad.rtol;
    A.atol = ad.atol;
    A.fac = ad.fac;
    A.facmin = ad.facmin;
    A.facmax = ad.facmax;
    A.r_escape = ad.r_escape;
    A.max_attempts = ad.max_attempts;
    if (ad.persistent) {
        const int32_t sub = ad.steps_per_chunk > 0 ? ad.steps_per_chunk : 8;
        int grid = 0;
        int rc = persistent_grid(multi ? (const void *)dp45_persistent_kernel<true>
                                       : (const void *)dp45_persistent_kernel<false>,
                                 block, n, grid);
        if (rc) return rc;
        unsigned long long *counter = (unsigned long long *)ws;
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, counter);
        MALBEC_LAUNCH_CHECK("zero_u64_kernel");
        if (multi)
            hipLaunchKernelGGL((dp45_persistent_kernel<true>), dim3(grid), dim3(block), 0, s, A, T,
                               counter, sub);
        else
            hipLaunchKernelGGL((dp45_persistent_kernel<false>), dim3(grid), dim3(block), 0, s, A, T,
                               counter, sub);
        MALBEC_LAUNCH_CHECK("dp45_persistent_kernel");
        return MALBEC_OK;
    }
    if (multi)
        hipLaunchKernelGGL((dp45_kernel<true>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
    else
        hipLaunchKernelGGL((dp45_kernel<false>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
    MALBEC_LAUNCH_CHECK("dp45_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
