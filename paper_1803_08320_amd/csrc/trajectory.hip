// FP64 integration with the paper's trajectory output: every `record_every` steps
// each lane writes (tau, t, x, y, z), the affine parameter, coordinate time and the
// Cartesian position of Section 2, eq. coord (x = sqrt(r^2 + a^2) sin(theta) cos(phi),
// y = sqrt(r^2 + a^2) sin(theta) sin(phi), z = r cos(theta)), into a decimated
// component-major buffer traj[(s * 5 + k) * n + i].  The paper prints this stream at
// every step from the host (Section 5); here it is produced in the kernel and the
// caller moves it off the device in chunks.
//
// Same step and stop rules as rk4_f64_kernel (either formulation).  One thread per
// lane; the state stays in registers between records.
#include "internal.hpp"

namespace malbec {

namespace {

struct RecArgs {
    int64_t n;
    double *state;
    int32_t *status;
    int32_t *steps;
    const int32_t *st_of_lane;
    double *traj;
    double h;
    double r_escape;
    int32_t record_every;
    int32_t n_rec;
};

__device__ __forceinline__ void copy8(double dst[8], const double src[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) dst[c] = src[c];
}

// One step of either formulation from y into y1; returns the status and sets `accept`
// (y1 is the lane's state after the step).
template <bool HAM>
__device__ __forceinline__ int32_t rec_step(const RecArgs &A, const Spacetime &S,
                                            const HamConst<double> &P, const double y[8],
                                            double y1[8], bool &accept)
{
    double sr[3];
    if (HAM)
        rk4_step_ham_f64(S, P, A.h, y, y1, sr);
    else
        rk4_step_f64(S, A.h, y, y1, sr);
    return terminate_f64(S, A.r_escape, sr, y1, accept);
}

__device__ __forceinline__ void put_record(const RecArgs &A, int64_t i, int32_t s, double a,
                                           const double y[8], int32_t steps_done)
{
    double st, ct, sp, cp;
    sincos(y[2], &st, &ct);
    sincos(y[3], &sp, &cp);
    const double rr = sqrt(fma(y[1], y[1], a * a));
    double *base = A.traj + (int64_t)s * 5 * A.n + i;
    base[0 * A.n] = A.h * (double)steps_done;
    base[1 * A.n] = y[0];
    base[2 * A.n] = rr * st * cp;
    base[3 * A.n] = rr * st * sp;
    base[4 * A.n] = y[1] * ct;
}

template <bool MULTI, bool HAM>
__global__ void __launch_bounds__(256) rk4_record_kernel(RecArgs A, StTable T)
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
    const Spacetime S = MULTI ? lds_st[sid] : T.st[0];
    // first thread of this wavefront (a scalar); the lane's index is rebuilt from it
    // at each record, so no per-lane address stays live across the step loop
    const int32_t wave0 = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x) & ~63;
    double y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = A.state[k * A.n + i];
    const HamConst<double> P = ham_const(S.a, y[4], y[7]);
    const int32_t steps0 = A.steps[i];
    int32_t taken = 0;
    for (int32_t s = 0; s < A.n_rec; ++s) {
        // steps of this record interval, two per iteration with y and y1 swapping
        // roles (no copy of an accepted step); y holds the state between iterations
        int32_t left = st == kActive ? A.record_every : 0;
        double y1[8];
        bool accept;
        while (left >= 2) {
            ++taken;
            st = rec_step<HAM>(A, S, P, y, y1, accept);
            if (st != kActive) {
                if (accept) copy8(y, y1);
                break;
            }
            ++taken;
            st = rec_step<HAM>(A, S, P, y1, y, accept);
            if (st != kActive) {
                if (!accept) copy8(y, y1);
                break;
            }
            left -= 2;
        }
        if (st == kActive && left == 1) {
            ++taken;
            st = rec_step<HAM>(A, S, P, y, y1, accept);
            if (accept) copy8(y, y1);
        }
        const int64_t ie = (int64_t)blockIdx.x * blockDim.x + wave0 +
                           (int32_t)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        put_record(A, ie, s, S.a, y, steps0 + taken);
    }
    const int64_t ie = (int64_t)blockIdx.x * blockDim.x + wave0 +
                       (int32_t)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int k = 0; k < 8; ++k) A.state[k * A.n + ie] = y[k];
    A.status[ie] = st;
    A.steps[ie] = steps0 + taken;
}

}  // namespace

int launch_integrate_record(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                            int64_t n, double *state, int32_t *status, int32_t *steps,
                            int32_t record_every, double *traj, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const bool ham = run.formulation == MALBEC_FORM_HAMILTONIAN;
    RecArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.traj = traj;
    A.h = run.h;
    A.r_escape = run.r_escape;
    A.record_every = record_every;
    A.n_rec = (int32_t)(run.n_steps / record_every);
    const dim3 grid(grid_for(n, block)), blk(block);
    if (multi && ham)
        hipLaunchKernelGGL((rk4_record_kernel<true, true>), grid, blk, 0, s, A, T);
    else if (multi)
        hipLaunchKernelGGL((rk4_record_kernel<true, false>), grid, blk, 0, s, A, T);
    else if (ham)
        hipLaunchKernelGGL((rk4_record_kernel<false, true>), grid, blk, 0, s, A, T);
    else
        hipLaunchKernelGGL((rk4_record_kernel<false, false>), grid, blk, 0, s, A, T);
    MALBEC_LAUNCH_CHECK("rk4_record_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
