// Discrete adjoint of the FP64 RK4 integrator (exact gradient of the computed map).
//
// Forward: malbec_integrate with checkpoint_every = K stores the state every K steps.
// Backward, per lane and per segment s = last .. 0: recompute the K step-start
// states from checkpoint s into the workspace (coalesced [K][8][n] doubles), then
// walk them in reverse applying the transposed RK4 step (rk4_vjp):
//     lam_y  = lam + J(Y4)^T lam_k4 + J(Y3)^T lam_k3 + J(Y2)^T lam_k2 + J(y)^T lam_k1,
//     lam_k4 = h/6 lam, lam_k3 = h/3 lam + h J(Y4)^T lam_k4,
//     lam_k2 = h/3 lam + h/2 J(Y3)^T lam_k3, lam_k1 = h/6 lam + h/2 J(Y2)^T lam_k2,
// where J = df/dy.  f = (u, a(r, theta, u)); the transposed Jacobian of the
// acceleration is the hand-written reverse mode of the regrouped acceleration the
// forward kernels evaluate (kerr_accel_vjp), at the stage points the forward step
// forms.  Steps a lane did not take (after it stopped, or a terminal step whose result
// was discarded) are the identity.  The next state of the reverse walk is loaded
// while the current one is transposed.
#include "dual.hpp"
#include "internal.hpp"

namespace malbec {

namespace {

struct AdjArgs {
    int64_t n;
    const double *ckpt;
    const int32_t *status;
    const int32_t *steps;
    const double *g_final;
    double *g_initial;
    const double *E_fixed;  // nullable
    double *g_named;        // nullable, 5n
    double *scratch;        // [K][8][n]
    const int32_t *st_of_lane;
    double h, r_escape;
    int32_t N, K;
};

// The acceleration of the forward kernels (the same stage trigonometry: a fresh sin
// and cos at the step's start, short rotations at the later stages) with its
// transposed Jacobian for rk4_vjp.  The stage points and the sin and cos of each (the
// last stage's formed by prepare) are kept from the forward pass, so the reverse pass
// evaluates no trigonometry.  (Keeping them in LDS instead of registers, to lower the
// register count, measured 4 % slower at the one wave per SIMD that 65,536 lanes give.)
struct AdjAccel {
    double M, a;
    StageTrigT<true, TabLds> trig;
    double Ys[4][6], sk[4], ck[4];
    __device__ __forceinline__ double &Y(int st, int k) { return Ys[st][k]; }
    __device__ __forceinline__ void keep() {}
    __device__ __forceinline__ void operator()(int stage, double r, double th, double ut, double ur,
                                               double uth, double uph, double &at, double &ar,
                                               double &ath, double &aph)
    {
        trig(stage, th, sk[stage], ck[stage]);
        kerr_accel<double>(M, a, r, sk[stage], ck[stage], ut, ur, uth, uph, at, ar, ath, aph);
    }
    __device__ __forceinline__ void prepare(int stage, double th) { trig(stage, th, sk[stage], ck[stage]); }
    __device__ __forceinline__ void vjp(int stage, double r, double, double ut, double ur, double uth,
                                        double uph, double bat, double bar, double bath, double baph,
                                        double &rb, double &thb, double ub[4])
    {
        const double s = sk[stage], c = ck[stage];
        double sb, cb;
        kerr_accel_vjp<double>(M, a, r, s, c, ut, ur, uth, uph, bat, bar, bath, baph, rb, sb, cb, ub);
        thb = fma(sb, c, -cb * s);  // d/dtheta through s = sin theta, c = cos theta
    }
};

template <bool MULTI>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs A, StTable T)
{
    __shared__ Spacetime lds_st[kMaxSt];
    if (MULTI)
        for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    // one wave per SIMD (the kernel's register count): nothing would cover the latency
    // of the trigonometry table's reads through the vector cache, which the workspace
    // streams through, so each block reads its own LDS copy
    TabLds::fill();
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t sid = MULTI ? A.st_of_lane[i] : 0;
    const bool bad = sid < 0 || sid >= T.n_st;
    if (bad) sid = 0;
    const Spacetime S = MULTI ? lds_st[sid] : T.st[0];
    const int64_t n = A.n;
    const int32_t status = A.status[i];
    const int32_t taken = A.steps[i];

    double lam[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) lam[k] = bad ? __builtin_nan("") : A.g_final[k * n + i];

    const int32_t nseg = (A.N + A.K - 1) / A.K;
    for (int32_t s = nseg - 1; s >= 0 && !bad; --s) {
        const int32_t g0 = s * A.K;
        if (g0 >= taken) continue;  // the lane had stopped before this segment
        int32_t len = A.N - g0 < A.K ? A.N - g0 : A.K;
        if (taken - g0 < len) len = taken - g0;
        // recompute the step-start states of the segment
        double y[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = A.ckpt[((int64_t)s * 8 + k) * n + i];
        for (int32_t j = 0; j < len; ++j) {
#pragma unroll
            for (int k = 0; k < 8; ++k) A.scratch[((int64_t)j * 8 + k) * n + i] = y[k];
            if (j + 1 < len) {
                double y1[8], sr[3];
                rk4_step_f64<true, TabLds>(S, A.h, y, y1, sr);
#pragma unroll
                for (int k = 0; k < 8; ++k) y[k] = y1[k];
            }
        }
        // reverse sweep; yn holds the state of step j, loaded one step ahead
        double yn[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) yn[k] = A.scratch[((int64_t)(len - 1) * 8 + k) * n + i];
        for (int32_t j = len - 1; j >= 0; --j) {
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = yn[k];
            if (j > 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k) yn[k] = A.scratch[((int64_t)(j - 1) * 8 + k) * n + i];
            }
            bool accepted = true;
            if (g0 + j == taken - 1 && status != kActive) {
                // terminal step: its result was kept only if the termination rule accepted it
                double y1[8], sr[3];
                rk4_step_f64<true, TabLds>(S, A.h, y, y1, sr);
                terminate_f64(S, A.r_escape, sr, y1, accepted);
            }
            if (accepted) {
                AdjAccel f{S.M, S.a, {}, {}, {}, {}};
                rk4_vjp(f, A.h, y, lam);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) A.g_initial[k * n + i] = lam[k];

    if (A.g_named) {
        // initial-condition map with E fixed: p = (r0, theta0, u^r0, u^theta0, L_z) ->
        // y0 = (0, r0, theta0, 0, u^t, u^r0, u^theta0, u^phi),
        // (u^t, u^phi) = G^{-1} (-E, L_z), G the (t, phi) block of the metric
        typedef Dual2<double> D;
        const double r0 = A.ckpt[1 * n + i], th0 = A.ckpt[2 * n + i];
        double s0, c0;
        sincos(th0, &s0, &c0);
        KerrCoef<D> Kd;
        kerr_coef<D>(D(S.M), D(S.a), D(r0, 1.0, 0.0), D(s0, 0.0, c0), D(c0, 0.0, -s0), Kd);
        // inverse (t, phi) block: g^tt = -Rtt/2, g^tphi = Rtp/2, g^phiphi = -Rpp/2
        const D itt = Kd.Rtt * D(-0.5), itp = Kd.Rtp * D(0.5), ipp = Kd.Rpp * D(-0.5);
        const double ut0 = A.ckpt[4 * n + i], uph0 = A.ckpt[7 * n + i];
        // lower with the block itself: G = inverse of the inverse block
        const double det = itt.v * ipp.v - itp.v * itp.v;
        const double gtt = ipp.v / det, gtp = -itp.v / det, gpp = itt.v / det;
        const double E = A.E_fixed ? A.E_fixed[i] : -(gtt * ut0 + gtp * uph0);
        const double Lz = fma(gtp, ut0, gpp * uph0);
        // u^t = itt (-E) + itp Lz, u^phi = itp (-E) + ipp Lz
        const double dut_r = fma(itt.dr, -E, itp.dr * Lz), dut_th = fma(itt.dth, -E, itp.dth * Lz);
        const double duph_r = fma(itp.dr, -E, ipp.dr * Lz), duph_th = fma(itp.dth, -E, ipp.dth * Lz);
        A.g_named[0 * n + i] = fma(lam[4], dut_r, fma(lam[7], duph_r, lam[1]));
        A.g_named[1 * n + i] = fma(lam[4], dut_th, fma(lam[7], duph_th, lam[2]));
        A.g_named[2 * n + i] = lam[5];
        A.g_named[3 * n + i] = lam[6];
        A.g_named[4 * n + i] = fma(lam[4], itp.v, lam[7] * ipp.v);
    }
}

}  // namespace

int launch_adjoint(const malbec_run &run, const StTable &T, const int32_t *st_of_lane, int64_t n,
                   const double *checkpoints, const int32_t *status, const int32_t *steps,
                   const double *g_final, double *g_initial, const double *E_fixed,
                   double *g_named, void *ws, hipStream_t s)
{
    AdjArgs A;
    A.n = n;
    A.ckpt = checkpoints;
    A.status = status;
    A.steps = steps;
    A.g_final = g_final;
    A.g_initial = g_initial;
    A.E_fixed = E_fixed;
    A.g_named = g_named;
    A.scratch = (double *)ws;
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    A.N = (int32_t)run.n_steps;
    A.K = run.checkpoint_every;
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    if (multi)
        hipLaunchKernelGGL((adjoint_kernel<true>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
    else
        hipLaunchKernelGGL((adjoint_kernel<false>), dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
    MALBEC_LAUNCH_CHECK("adjoint_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
