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
#include "monitor.hpp"
#include "persistent.hpp"

namespace malbec {

namespace {

// FP32 sin and cos of a moderate theta (stage points, |theta| < 1e3): Cody-Waite
// reduction by pi/2 in two FMA steps (pi/2 = hi + lo in single precision), minimax
// polynomials sin x = x + x^3 P(x^2) (P of degree 2) and cos x = 1 - x^2 Q(x^2) (Q of
// degree 3) on |x| <= pi/4 from gen_minimax.py (relative error 1.3e-8 and 1e-9 with
// the coefficients rounded to single precision), and the quadrant taken mod 4.
__device__ __forceinline__ void sincos_f32(float th, float &s, float &c)
{
    const float k = rintf(th * 0.636619772f);
    const float x = fmaf(-k, -4.37113883e-08f, fmaf(-k, 1.57079637f, th));
    const float z = x * x;
    const float ps = fmaf(fmaf(z, -1.95880086e-04f, 8.33274890e-03f), z, -1.66666642e-01f);
    const float sx = fmaf(x * z, ps, x);
    const float pc = fmaf(fmaf(fmaf(z, -2.44638868e-05f, 1.38875900e-03f), z, -4.16666493e-02f), z, 0.5f);
    const float cx = fmaf(-z, pc, 1.0f);
    const int q = ((int)k) & 3;  // k mod 4, negative k too
    const float ss = (q & 1) ? cx : sx, cc = (q & 1) ? sx : cx;
    s = (q & 2) ? -ss : ss;
    c = ((q + 1) & 2) ? -cc : cc;
}

// FP32 sin and cos of the stage theta.  Stage 0 evaluates them (sincos_f32) and sets
// the rotation limit min(0.01, sin(theta_0) / 2); later stages rotate that pair by the
// small angle difference d, with sin d = d - d^3/6 and cos d = 1 - d^2/2 (truncation
// below 8.4e-13 and 4.2e-10 absolute for |d| <= 0.01, far under FP32 rounding; the
// second bound keeps sin(theta_0 + d) >= sin(theta_0) / 2), or evaluate afresh beyond
// the limit.
struct StageTrigF32 {
    float th0, s0, c0, lim;
    __device__ __forceinline__ void operator()(int stage, float th, float &s, float &c)
    {
        if (stage == 0) {
            sincos_f32(th, s, c);
            th0 = th;
            s0 = s;
            c0 = c;
            lim = fminf(0.01f, 0.5f * s);
            return;
        }
        const float d = th - th0;
        if (!(fabsf(d) <= lim)) {
            sincos_f32(th, s, c);
        } else {
            const float d2 = d * d;
            const float sd = fmaf(d * d2, -1.0f / 6.0f, d);
            const float cd = fmaf(d2, -0.5f, 1.0f);
            s = fmaf(s0, cd, c0 * sd);
            c = fmaf(c0, cd, -s0 * sd);
        }
    }
};

// FP32 right-hand sides: the Christoffel form and Hamilton's equations.
struct AccelF32 {
    float M, a;
    StageTrigF32 trig;
    __device__ __forceinline__ void operator()(int stage, float r, float th, float ut, float ur,
                                               float uth, float uph, float &at, float &ar,
                                               float &ath, float &aph)
    {
        float s, c;
        trig(stage, th, s, c);
        kerr_accel<float>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};

struct HamF32 {
    float M, a;
    const HamConst<float> &P;
    StageTrigF32 trig;
    __device__ __forceinline__ void operator()(int stage, float r, float th, float pr, float pth,
                                               float &dt, float &dr, float &dth, float &dph,
                                               float &dpr, float &dpth)
    {
        float s, c;
        trig(stage, th, s, c);
        kerr_ham<float>(M, a, r, s, c, pr, pth, P, dt, dr, dth, dph, dpr, dpth);
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

// One lane as a work item: load splits the double state, step advances one step
// (FP64 inside the zone, FP32 + two-sum outside), store recombines hi + lo.  HAM:
// the state is (x^mu, p_mu) and the step is that of Hamilton's equations; p_t and
// p_phi never change (their increment is exactly 0, and the two-sum keeps hi + lo).
template <bool HAM>
struct MixProg {
    const MixArgs &A;
    const Spacetime *table;
    bool multi;
    int32_t n_st;
    struct Lane {
        float hi[8], lo[8];
        Spacetime S;
        float rs32;  // the largest float not above S.r_stop
        HamConst<double> P64;
        HamConst<float> P32;
        int32_t st, taken;
    };
    __device__ __forceinline__ bool load(int64_t i, Lane &L)
    {
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
        L.S = table[sid];
        L.rs32 = (float)L.S.r_stop;  // r_stop > 0: one step down is the bit pattern minus one
        if ((double)L.rs32 > L.S.r_stop) L.rs32 = __int_as_float(__float_as_int(L.rs32) - 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) split(A.state[k * A.n + i], L.hi[k], L.lo[k]);
        if (HAM) {
            L.P64 = ham_const(L.S.a, (double)L.hi[4] + (double)L.lo[4], (double)L.hi[7] + (double)L.lo[7]);
            L.P32 = ham_const((float)L.S.a, L.hi[4], L.hi[7]);
        }
        L.taken = 0;
        return A.n_steps > 0;
    }
    __device__ __forceinline__ bool step(Lane &L)
    {
        ++L.taken;
        const Spacetime &S = L.S;
        const double r_now = (double)L.hi[1] + (double)L.lo[1];
        if (r_now < S.r_zone) {
            double y[8], y1[8], sr[3];
#pragma unroll
            for (int c = 0; c < 8; ++c) y[c] = (double)L.hi[c] + (double)L.lo[c];
            if (HAM)
                rk4_step_ham_f64(S, L.P64, A.h, y, y1, sr);
            else
                rk4_step_f64(S, A.h, y, y1, sr);
            bool accept;
            L.st = terminate_f64(S, A.r_escape, sr, y1, accept);
            // a step that is not accepted ends the lane (HORIZON at a stage point, or
            // NONFINITE), which keeps y: splitting y again gives a pair whose sum is y
            // exactly, so the stored state is the same, while hi and lo need not stay
            // live across the FP64 step (16 registers fewer)
#pragma unroll
            for (int c = 0; c < 8; ++c) split(accept ? y1[c] : y[c], L.hi[c], L.lo[c]);
        } else {
            float d[8], sr[3];
            if (HAM) {
                HamF32 f32{(float)S.M, (float)S.a, L.P32, {0.0f, 0.0f, 1.0f, 0.0f}};
                rk4_ham_delta(f32, (float)A.h, L.hi, d, sr);
            } else {
                AccelF32 f32{(float)S.M, (float)S.a, {0.0f, 0.0f, 1.0f, 0.0f}};
                rk4_delta(f32, (float)A.h, L.hi, d, sr);
            }
            // (double)x <= r_stop exactly when x <= rs32, the largest float not above r_stop
            if (sr[0] <= L.rs32 || sr[1] <= L.rs32 || sr[2] <= L.rs32) {
                L.st = kHorizon;
            } else {
                float nh[8], nl[8];
                bool ok = true;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    // the two-sum's error term of a finite sum is finite (and exact), so
                    // a finite nh implies a finite nl
                    two_sum(L.hi[c], d[c] + L.lo[c], nh[c], nl[c]);
                    ok = ok && __builtin_isfinite(nh[c]);
                }
                const double th = (double)nh[2] + (double)nl[2];
                if (!(ok && th > 0.0 && th < 3.14159265358979323846)) {
                    L.st = kNonfinite;
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) { L.hi[c] = nh[c]; L.lo[c] = nl[c]; }
                    const double r1 = (double)L.hi[1] + (double)L.lo[1];
                    if (r1 <= S.r_stop) L.st = kHorizon;
                    else if (r1 >= A.r_escape) L.st = kEscape;
                }
            }
        }
        return L.st != kActive || L.taken == A.n_steps;
    }
    __device__ __forceinline__ void store(int64_t item, const Lane &L)
    {
        const int64_t i = opaque(item);
#pragma unroll
        for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = (double)L.hi[k] + (double)L.lo[k];
        A.status[i] = L.st;
        A.steps[i] += L.taken;
    }
    __device__ static __forceinline__ void state64(const Lane &L, double y[8])
    {
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = (double)L.hi[k] + (double)L.lo[k];
    }
};

// The Christoffel-form kernels are held to 128 registers, four waves per SIMD (the
// FP64 zone step sets the peak; the FP32 step alone needs about 80); the Hamiltonian
// form's zone step needs about 150 and keeps the compiler's default (three waves).
template <bool MULTI, bool HAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HAM ? 1 : 4, HAM ? 8 : 4)))
rk4_f32k_kernel(MixArgs A, StTable T)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    MixProg<HAM> P{A, lds_st, MULTI, T.n_st};
    typename MixProg<HAM>::Lane L;
    if (!P.load(i, L)) return;
    while (!P.step(L)) {
    }
    P.store(i, L);
}

template <bool MULTI, bool HAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HAM ? 1 : 4, HAM ? 8 : 4)))
rk4_f32k_persistent_kernel(MixArgs A, StTable T, unsigned long long *counter, int32_t chunk)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    MixProg<HAM> P{A, lds_st, MULTI, T.n_st};
    persistent_loop(P, A.n, counter, chunk);
}

// The compensated step with the invariant monitor (FP64, on hi + lo) every K steps.
template <bool HAM>
__global__ void __launch_bounds__(256) rk4_f32k_monitor_kernel(MixArgs A, StTable T, MonArgs MA,
                                                               int32_t multi)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    __shared__ double lds_mon[8 * kMonLanes];
    MonProg<MixProg<HAM>, HAM> P{MixProg<HAM>{A, lds_st, multi != 0, T.n_st}, MA, &lds_mon[threadIdx.x]};
    typename MonProg<MixProg<HAM>, HAM>::Lane L;
    if (!P.load(i, L)) return;
    while (!P.step(L)) {
    }
    P.store(i, L);
}

template <bool HAM>
__global__ void __launch_bounds__(256) rk4_f32k_monitor_persistent_kernel(MixArgs A, StTable T,
                                                                          MonArgs MA, int32_t multi,
                                                                          unsigned long long *counter,
                                                                          int32_t chunk)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    __shared__ double lds_mon[8 * kMonLanes];
    MonProg<MixProg<HAM>, HAM> P{MixProg<HAM>{A, lds_st, multi != 0, T.n_st}, MA, &lds_mon[threadIdx.x]};
    persistent_loop(P, A.n, counter, chunk);
}

template <bool HAM>
int launch_monitor(const MixArgs &A, const StTable &T, const MonArgs &MA, bool multi, int block,
                   bool persistent, int32_t sub, unsigned long long *counter, hipStream_t s)
{
    if (persistent) {
        int grid = 0;
        int rc = persistent_grid((const void *)rk4_f32k_monitor_persistent_kernel<HAM>, block, A.n, grid);
        if (rc) return rc;
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, counter);
        MALBEC_LAUNCH_CHECK("zero_u64_kernel");
        hipLaunchKernelGGL((rk4_f32k_monitor_persistent_kernel<HAM>), dim3(grid), dim3(block), 0, s,
                           A, T, MA, (int32_t)multi, counter, sub);
        MALBEC_LAUNCH_CHECK("rk4_f32k_monitor_persistent_kernel");
        return MALBEC_OK;
    }
    hipLaunchKernelGGL((rk4_f32k_monitor_kernel<HAM>), dim3(grid_for(A.n, block)), dim3(block), 0, s,
                       A, T, MA, (int32_t)multi);
    MALBEC_LAUNCH_CHECK("rk4_f32k_monitor_kernel");
    return MALBEC_OK;
}

}  // namespace

template <bool MULTI, bool HAM>
int launch_f32k(const MixArgs &A, const StTable &T, bool persistent, int32_t sub, int block,
                void *ws, hipStream_t s)
{
    if (persistent) {
        int grid = 0;
        int rc = persistent_grid((const void *)rk4_f32k_persistent_kernel<MULTI, HAM>, block, A.n, grid);
        if (rc) return rc;
        unsigned long long *counter = (unsigned long long *)ws;
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, counter);
        MALBEC_LAUNCH_CHECK("zero_u64_kernel");
        hipLaunchKernelGGL((rk4_f32k_persistent_kernel<MULTI, HAM>), dim3(grid), dim3(block), 0, s,
                           A, T, counter, sub);
        MALBEC_LAUNCH_CHECK("rk4_f32k_persistent_kernel");
        return MALBEC_OK;
    }
    hipLaunchKernelGGL((rk4_f32k_kernel<MULTI, HAM>), dim3(grid_for(A.n, block)), dim3(block), 0, s,
                       A, T);
    MALBEC_LAUNCH_CHECK("rk4_f32k_kernel");
    return MALBEC_OK;
}

int launch_integrate_f32k(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                          int64_t n, double *state, int32_t *status, int32_t *steps, void *ws,
                          hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const bool ham = run.formulation == MALBEC_FORM_HAMILTONIAN;
    const int64_t total = run.n_steps;
    MixArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    auto go = [&](bool persistent, int32_t sub) {
        if (multi)
            return ham ? launch_f32k<true, true>(A, T, persistent, sub, block, ws, s)
                       : launch_f32k<true, false>(A, T, persistent, sub, block, ws, s);
        return ham ? launch_f32k<false, true>(A, T, persistent, sub, block, ws, s)
                   : launch_f32k<false, false>(A, T, persistent, sub, block, ws, s);
    };
    if (run.persistent) {
        A.n_steps = (int32_t)total;
        return go(true, run.steps_per_chunk > 0 ? run.steps_per_chunk : 64);
    }
    const int64_t chunk = run.steps_per_chunk > 0 ? run.steps_per_chunk : total;
    for (int64_t k0 = 0; k0 < total; k0 += chunk) {
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        int rc = go(false, 0);
        if (rc) return rc;
    }
    return MALBEC_OK;
}

int launch_monitor_f32k(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                        int64_t n, double *state, int32_t *status, int32_t *steps, int32_t every,
                        int32_t reset, double *mon, void *ws, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const bool ham = run.formulation == MALBEC_FORM_HAMILTONIAN;
    const int64_t total = run.n_steps;
    MixArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    MonArgs MA{mon, steps, n, every, reset};
    unsigned long long *counter = (unsigned long long *)ws;
    if (run.persistent) {
        A.n_steps = (int32_t)total;
        const int32_t sub = run.steps_per_chunk > 0 ? run.steps_per_chunk : 64;
        return ham ? launch_monitor<true>(A, T, MA, multi, block, true, sub, counter, s)
                   : launch_monitor<false>(A, T, MA, multi, block, true, sub, counter, s);
    }
    const int64_t chunk = run.steps_per_chunk > 0 ? run.steps_per_chunk : total;
    for (int64_t k0 = 0; k0 < total; k0 += chunk) {
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        MA.reset = (k0 == 0) ? reset : 0;
        int rc = ham ? launch_monitor<true>(A, T, MA, multi, block, false, 0, counter, s)
                     : launch_monitor<false>(A, T, MA, multi, block, false, 0, counter, s);
        if (rc) return rc;
    }
    return MALBEC_OK;
}

}  // namespace malbec
