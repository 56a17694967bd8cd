// Discrete adjoint of the FP64 RK4 integrator (exact gradient of the computed map).
//
// Forward: malbec_integrate with checkpoint_every = K stores the state every K steps.
// Backward, per lane and per segment s = last .. 0: recompute the K step-start
// states from checkpoint s into the workspace (coalesced [K][8][n] doubles), then
// walk them in reverse applying the transposed RK4 step
//     lam_y  = lam + J(Y4)^T lam_k4 + J(Y3)^T lam_k3 + J(Y2)^T lam_k2 + J(y)^T lam_k1,
//     lam_k4 = h/6 lam, lam_k3 = h/3 lam + h J(Y4)^T lam_k4,
//     lam_k2 = h/3 lam + h/2 J(Y3)^T lam_k3, lam_k1 = h/6 lam + h/2 J(Y2)^T lam_k2,
// where J = df/dy.  f = (u, a(r, theta, u)); the transposed Jacobian of the
// acceleration is taken in reverse mode through the contraction (kerr_contract,
// written out below) and in forward mode (dual numbers in r, theta) through the
// position-dependent coefficients (kerr_coef).  Steps a lane did not take (after
// it stopped, or a terminal step whose result was discarded) are the identity.
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

// dL/d(r, theta, u) of the acceleration given dL/d(at, ar, ath, aph).
__device__ __forceinline__ void vjp_accel(double M, double a, double r, double th, double ut,
                                          double ur, double uth, double uph, double b_at,
                                          double b_ar, double b_ath, double b_aph, double &rbar,
                                          double &thbar, double ubar[4])
{
    typedef Dual2<double> D;
    double s, c;
    sincos_any(th, s, c);
    // pass 1: primal coefficients -> contraction -> cotangents of the coefficients
    KerrCoef<double> K;
    kerr_coef<double>(M, a, r, s, c, K);
    double at, ar, ath, aph;
    KerrContr<double> X;
    kerr_contract(K, ut, ur, uth, uph, at, ar, ath, aph, &X);

    KerrCoef<double> B;  // dL/d(coefficient)
    // at = Rtt Wt - Rtp Wp, aph = Rpp Wp - Rtp Wt
    B.Rtt = b_at * X.Wt;
    B.Rtp = -fma(b_at, X.Wp, b_aph * X.Wt);
    B.Rpp = b_aph * X.Wp;
    const double bWt = fma(b_at, K.Rtt, -b_aph * K.Rtp);
    const double bWp = fma(b_aph, K.Rpp, -b_at * K.Rtp);
    // ar = Fr Dirho2, ath = Fth irho2
    const double bFr = b_ar * K.Dirho2;
    B.Dirho2 = b_ar * X.Fr;
    const double bFth = b_ath * K.irho2;
    B.irho2 = b_ath * X.Fth;
    // Fr = Qr - dgrr_r urur + r uthuth + c1 uruth2
    // Fth = Qth - c1 urur + a2sc uthuth - r uruth2,   uruth2 = 2 ur uth
    const double urur = ur * ur, uthuth = uth * uth, uruth2 = (ur + ur) * uth;
    const double bQr = bFr, bQth = bFth;
    B.dgrr_r = -bFr * urur;
    B.c1 = fma(bFr, uruth2, -bFth * urur);
    B.r = fma(bFr, uthuth, -bFth * uruth2);
    B.a2sc = bFth * uthuth;
    const double burur = -fma(bFr, K.dgrr_r, bFth * K.c1);
    const double buthuth = fma(bFr, K.r, bFth * K.a2sc);
    const double buruth2 = fma(bFr, K.c1, -bFth * K.r);
    double bur = 2.0 * fma(ur, burur, uth * buruth2);
    double buth = 2.0 * fma(uth, buthuth, ur * buruth2);
    // Qr = ut Pt_r + uph Pp_r, Qth = ut Pt_th + uph Pp_th
    double but = fma(bQr, X.Pt_r, bQth * X.Pt_th);
    double buph = fma(bQr, X.Pp_r, bQth * X.Pp_th);
    double bPt_r = bQr * ut, bPp_r = bQr * uph, bPt_th = bQth * ut, bPp_th = bQth * uph;
    // Wt = ur Pt_r + uth Pt_th, Wp = ur Pp_r + uth Pp_th
    bur = fma(bWt, X.Pt_r, fma(bWp, X.Pp_r, bur));
    buth = fma(bWt, X.Pt_th, fma(bWp, X.Pp_th, buth));
    bPt_r = fma(bWt, ur, bPt_r);
    bPt_th = fma(bWt, uth, bPt_th);
    bPp_r = fma(bWp, ur, bPp_r);
    bPp_th = fma(bWp, uth, bPp_th);
    // Pt_r = dgtt_r ut + dgtp_r uph, Pt_th = dgtt_th ut + dgtp_th uph,
    // Pp_r = dgtp_r ut + dgpp_r uph, Pp_th = dgtp_th ut + dgpp_th uph
    B.dgtt_r = bPt_r * ut;
    B.dgtp_r = fma(bPt_r, uph, bPp_r * ut);
    B.dgpp_r = bPp_r * uph;
    B.dgtt_th = bPt_th * ut;
    B.dgtp_th = fma(bPt_th, uph, bPp_th * ut);
    B.dgpp_th = bPp_th * uph;
    but = fma(bPt_r, K.dgtt_r, fma(bPt_th, K.dgtt_th, fma(bPp_r, K.dgtp_r, fma(bPp_th, K.dgtp_th, but))));
    buph = fma(bPt_r, K.dgtp_r, fma(bPt_th, K.dgtp_th, fma(bPp_r, K.dgpp_r, fma(bPp_th, K.dgpp_th, buph))));
    ubar[0] = but;
    ubar[1] = bur;
    ubar[2] = buth;
    ubar[3] = buph;
    // pass 2: the coefficients again in dual numbers (d/dr, d/dtheta), each folded into
    // the r and theta cotangents as soon as it is formed
    KerrCoef<D> Kd;
    kerr_coef<D>(D(M), D(a), D(r, 1.0, 0.0), D(s, 0.0, c), D(c, 0.0, -s), Kd);
    double sr = 0.0, st = 0.0;
#define MALBEC_C(f) sr = fma(B.f, Kd.f.dr, sr); st = fma(B.f, Kd.f.dth, st);
    MALBEC_C(r) MALBEC_C(Rtt) MALBEC_C(Rtp) MALBEC_C(Rpp) MALBEC_C(irho2)
    MALBEC_C(Dirho2) MALBEC_C(a2sc) MALBEC_C(dgtt_r) MALBEC_C(dgtt_th) MALBEC_C(dgtp_r)
    MALBEC_C(dgtp_th) MALBEC_C(dgpp_r) MALBEC_C(dgpp_th) MALBEC_C(dgrr_r) MALBEC_C(c1)
#undef MALBEC_C
    rbar = sr;
    thbar = st;
}

// mu = J(Y)^T lam_k for f = (u, a): mu_t = mu_phi = 0, mu_{r,theta} from a,
// mu_u = lam_k[x] + (da/du)^T lam_k[a].  Y = (r, th, ut, ur, uth, uph).
__device__ __forceinline__ void jt(const Spacetime &S, const double Y[6], const double lk[8], double mu[8])
{
    double rbar, thbar, ub[4];
    vjp_accel(S.M, S.a, Y[0], Y[1], Y[2], Y[3], Y[4], Y[5], lk[4], lk[5], lk[6], lk[7], rbar, thbar, ub);
    mu[0] = 0.0;
    mu[1] = rbar;
    mu[2] = thbar;
    mu[3] = 0.0;
    mu[4] = lk[0] + ub[0];
    mu[5] = lk[1] + ub[1];
    mu[6] = lk[2] + ub[2];
    mu[7] = lk[3] + ub[3];
}

// lam <- (d y_{n+1} / d y_n)^T lam for the RK4 step from y (same stage arithmetic as
// rk4_stages).
__device__ __forceinline__ void vjp_step(const Spacetime &S, double h, const double y[8], double lam[8])
{
    AccelF64 f{S.M, S.a, {}};
    const double hh = 0.5 * h;
    double Y1[6] = {y[1], y[2], y[4], y[5], y[6], y[7]};
    double at, ar, ath, aph;
    f(0, Y1[0], Y1[1], Y1[2], Y1[3], Y1[4], Y1[5], at, ar, ath, aph);
    double Y2[6] = {fma(hh, y[5], y[1]), fma(hh, y[6], y[2]), fma(hh, at, y[4]), fma(hh, ar, y[5]),
                    fma(hh, ath, y[6]), fma(hh, aph, y[7])};
    f(1, Y2[0], Y2[1], Y2[2], Y2[3], Y2[4], Y2[5], at, ar, ath, aph);
    double Y3[6] = {fma(hh, Y2[3], y[1]), fma(hh, Y2[4], y[2]), fma(hh, at, y[4]), fma(hh, ar, y[5]),
                    fma(hh, ath, y[6]), fma(hh, aph, y[7])};
    f(2, Y3[0], Y3[1], Y3[2], Y3[3], Y3[4], Y3[5], at, ar, ath, aph);
    double Y4[6] = {fma(h, Y3[3], y[1]), fma(h, Y3[4], y[2]), fma(h, at, y[4]), fma(h, ar, y[5]),
                    fma(h, ath, y[6]), fma(h, aph, y[7])};

    const double h6 = h * (1.0 / 6.0), h3 = 2.0 * h6;
    double ly[8], lk[8], mu[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { ly[k] = lam[k]; lk[k] = h6 * lam[k]; }
    jt(S, Y4, lk, mu);  // k4
#pragma unroll
    for (int k = 0; k < 8; ++k) { ly[k] += mu[k]; lk[k] = fma(h3, lam[k], h * mu[k]); }
    jt(S, Y3, lk, mu);  // k3
#pragma unroll
    for (int k = 0; k < 8; ++k) { ly[k] += mu[k]; lk[k] = fma(h3, lam[k], hh * mu[k]); }
    jt(S, Y2, lk, mu);  // k2
#pragma unroll
    for (int k = 0; k < 8; ++k) { ly[k] += mu[k]; lk[k] = fma(h6, lam[k], hh * mu[k]); }
    jt(S, Y1, lk, mu);  // k1
#pragma unroll
    for (int k = 0; k < 8; ++k) lam[k] = ly[k] + mu[k];
}

template <bool MULTI>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs A, StTable T)
{
    __shared__ Spacetime lds_st[kMaxSt];
    if (MULTI) {
        for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
        __syncthreads();
    }
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
                rk4_step_f64(S, A.h, y, y1, sr);
#pragma unroll
                for (int k = 0; k < 8; ++k) y[k] = y1[k];
            }
        }
        // reverse sweep
        for (int32_t j = len - 1; j >= 0; --j) {
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = A.scratch[((int64_t)j * 8 + k) * n + i];
            bool accepted = true;
            if (g0 + j == taken - 1 && status != kActive) {
                // terminal step: its result was kept only if the termination rule accepted it
                double y1[8], sr[3];
                rk4_step_f64(S, A.h, y, y1, sr);
                terminate_f64(S, A.r_escape, sr, y1, accepted);
            }
            if (accepted) vjp_step(S, A.h, y, lam);
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
