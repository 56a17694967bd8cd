// Mixed-precision RK4 integrator: FP32 state with a compensated update, FP64 steps
// near the horizon.
//
// Each lane holds its state as an unevaluated float pair y = hi + lo.  A step that
// starts at r >= r_zone (= fp64_zone_factor * r_+) evaluates the four RK4 stages in
// FP32 on hi and adds the increment d = h/6 (k1 + 2k2 + 2k3 + k4) with an exact
// two-sum (Knuth): t = hi + (d + lo), lo <- rounding error of that sum, hi <- t.  So
// the state keeps ~48 significant bits while the stage arithmetic is FP32.  A step
// that starts inside r_zone runs entirely in FP64 on hi + lo and splits the result
// back.  The double state in HBM is hi + lo at load (split) and at store (sum).
#include "internal.hpp"

namespace malbec {

namespace {

struct AccelF32 {
    float M, a;
    __device__ __forceinline__ void operator()(int, float r, float th, float ut, float ur,
                                               float uth, float uph, float &at, float &ar,
                                               float &ath, float &aph) const
    {
        float s, c;
        sincosf(th, &s, &c);
        kerr_accel<float>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};

struct MixArgs {
    int64_t n;
    double *state;
    int32_t *status;
    int32_t *steps;
    const int32_t *st_of_lane;
    double h;
    double r_escape;
    int32_t n_steps;
};

// hi + lo = x exactly for |x| within float range: hi = fl32(x), lo = fl32(x - hi).
__device__ __forceinline__ void split(double x, float &hi, float &lo)
{
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

// Knuth's two-sum without contraction: s = fl(a + b), e = (a + b) - s exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
#pragma clang fp contract(off)
    s = a + b;
    const float bp = s - a;
    const float ap = s - bp;
    e = (a - ap) + (b - bp);
}

template <bool MULTI>
__global__ void __launch_bounds__(256) rk4_f32k_kernel(MixArgs A, StTable T)
{
    __shared__ Spacetime lds_st[kMaxSt];
    if (MULTI) {
        for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t st = A.status[i];
    int32_t sid = 0;
    if (MULTI) {
        sid = A.st_of_lane[i];
        if (sid < 0 || sid >= T.n_st) {
            sid = 0;
            if (st == kActive) st = kNonfinite;
            A.status[i] = st;
        }
    }
    if (st != kActive) return;
    const Spacetime S = MULTI ? lds_st[sid] : T.st[0];
    AccelF32 f32{(float)S.M, (float)S.a};
    const float h32 = (float)A.h;

    float hi[8], lo[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) split(A.state[k * A.n + i], hi[k], lo[k]);
    int32_t taken = 0;

    for (int32_t k = 0; k < A.n_steps; ++k) {
        ++taken;
        const double r_now = (double)hi[1] + (double)lo[1];
        if (r_now < S.r_zone) {
            double y[8], y1[8], sr[3];
#pragma unroll
            for (int c = 0; c < 8; ++c) y[c] = (double)hi[c] + (double)lo[c];
            rk4_step_f64(S, A.h, y, y1, sr);
            bool accept;
            st = terminate_f64(S, A.r_escape, sr, y1, accept);
            if (accept) {
#pragma unroll
                for (int c = 0; c < 8; ++c) split(y1[c], hi[c], lo[c]);
            }
        } else {
            float d[8], sr[3];
            rk4_delta(f32, h32, hi, d, sr);
            if ((double)sr[0] <= S.r_stop || (double)sr[1] <= S.r_stop || (double)sr[2] <= S.r_stop) {
                st = kHorizon;
            } else {
                float nh[8], nl[8];
                bool ok = true;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    two_sum(hi[c], d[c] + lo[c], nh[c], nl[c]);
                    ok = ok && __builtin_isfinite(nh[c]) && __builtin_isfinite(nl[c]);
                }
                const double th = (double)nh[2] + (double)nl[2];
                if (!(ok && th > 0.0 && th < 3.14159265358979323846)) {
                    st = kNonfinite;
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) { hi[c] = nh[c]; lo[c] = nl[c]; }
                    const double r1 = (double)hi[1] + (double)lo[1];
                    if (r1 <= S.r_stop) st = kHorizon;
                    else if (r1 >= A.r_escape) st = kEscape;
                }
            }
        }
        if (st != kActive) break;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = (double)hi[k] + (double)lo[k];
    A.status[i] = st;
    A.steps[i] += taken;
}

}  // namespace

int launch_integrate_f32k(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                          int64_t n, double *state, int32_t *status, int32_t *steps, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const int64_t total = run.n_steps;
    const int64_t chunk = run.steps_per_chunk > 0 ? run.steps_per_chunk : total;
    MixArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    for (int64_t k0 = 0; k0 < total; k0 += chunk) {
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        if (multi)
            hipLaunchKernelGGL((rk4_f32k_kernel<true>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
        else
            hipLaunchKernelGGL((rk4_f32k_kernel<false>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
        MALBEC_LAUNCH_CHECK("rk4_f32k_kernel");
    }
    return MALBEC_OK;
}

}  // namespace malbec
