// FP64 fixed-step RK4 integrator: one lane (thread) per geodesic.
//
// Each lane loads its 8-component state once (coalesced, component-major), runs
// the steps of the launch with all stage values in registers and stores the state
// once.  The only global traffic is 64 B in + 64 B out + status/steps per lane per
// launch; the work is FP64 VALU arithmetic.  Spacetime constants come from the
// kernel arguments (uniform batch) or from an LDS copy of the table (mixed batch).
#include "internal.hpp"
#include "monitor.hpp"
#include "persistent.hpp"

namespace malbec {

namespace {

struct IntArgs {
    int64_t n;
    double *state;
    int32_t *status;
    int32_t *steps;
    const int32_t *st_of_lane;
    double *ckpt;      // checkpoint slots or nullptr
    double h;
    double r_escape;
    int32_t n_steps;   // steps in this launch
    int32_t k0;        // index of this launch's first step within the call
    int32_t ck_every;  // K (0 = none)
    int32_t ck_last;   // index of the last slot of the call
};

__device__ __forceinline__ void put_slot(const IntArgs &A, int64_t i, int32_t slot, const double y[8])
{
    double *base = A.ckpt + (int64_t)slot * 8 * A.n;
#pragma unroll
    for (int k = 0; k < 8; ++k) base[k * A.n + i] = y[k];
}

__device__ __forceinline__ void copy8(double dst[8], const double src[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) dst[c] = src[c];
}

// One FP64 RK4 step of either formulation: the Christoffel form on (x, u), or
// Hamilton's equations on (x, p) with the lane's constants p_t, p_phi in P.
template <bool HAM>
__device__ __forceinline__ void step_f64(const Spacetime &S, const HamConst<double> &P, double h,
                                         const double y[8], double y1[8], double sr[3])
{
    if (HAM)
        rk4_step_ham_f64(S, P, h, y, y1, sr);
    else
        rk4_step_f64(S, h, y, y1, sr);
}

// UNIT_M: the batch's one spacetime has M = 1 (the unit of the paper's runs), known at
// compile time, which removes the multiplications by M (exact: the results are the
// bits of the general kernel).
template <bool MULTI, bool CKPT, bool HAM, bool UNIT_M = false>
__global__ void __launch_bounds__(256) rk4_f64_kernel(IntArgs A, StTable T)
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
        if (sid < 0 || sid >= T.n_st) {  // invalid spacetime index: the lane cannot step
            sid = 0;
            if (st == kActive) st = kNonfinite;
            A.status[i] = st;
        }
    }
    Spacetime S = MULTI ? lds_st[sid] : T.st[0];
    if (UNIT_M) S.M = 1.0;
    // first thread of this wavefront (wave-uniform, held in a scalar register)
    const int32_t wave0 = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x) & ~63;

    double y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = A.state[k * A.n + i];
    const HamConst<double> P = ham_const(S.a, y[4], y[7]);
    int32_t taken = 0;
    int32_t next_slot = 0;
    if (CKPT) next_slot = (A.k0 + A.ck_every - 1) / A.ck_every;  // first slot at or after k0

    if (!CKPT && st == kActive) {
        // Two steps per iteration, the second with the roles of y and y1 swapped, so
        // that an accepted step never copies the state.  The common outcome of the stop
        // rules is tested first.  A launch always has n_steps >= 1 (the launcher makes
        // none for a call of zero steps).
        double y1[8];
        int32_t ks = 0;
        for (;;) {
            double sr[3];
            bool accept = true;
            step_f64<HAM>(S, P, A.h, y, y1, sr);
            ++ks;
            if (!still_active_f64(S, A.r_escape, sr, y1))
                st = terminate_f64(S, A.r_escape, sr, y1, accept);
            if (st != kActive || ks == A.n_steps) {
                if (accept) copy8(y, y1);
                break;
            }
            step_f64<HAM>(S, P, A.h, y1, y, sr);
            ++ks;
            accept = true;
            if (!still_active_f64(S, A.r_escape, sr, y))
                st = terminate_f64(S, A.r_escape, sr, y, accept);
            if (st != kActive || ks == A.n_steps) {
                if (!accept) copy8(y, y1);
                break;
            }
        }
        taken = ks;
        // the lane's index rebuilt from wave-uniform values and its position in the
        // wavefront: no per-lane address stays live across the loop
        const int64_t ie = (int64_t)blockIdx.x * blockDim.x + wave0 +
                           (int32_t)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
        for (int k = 0; k < 8; ++k) A.state[k * A.n + ie] = y[k];
        A.status[ie] = st;
        A.steps[ie] += taken;
    } else if (st == kActive) {
        for (int32_t k = 0; k < A.n_steps; ++k) {
            if (CKPT && (A.k0 + k) == next_slot * A.ck_every) {
                put_slot(A, i, next_slot, y);
                ++next_slot;
            }
            double y1[8], sr[3];
            step_f64<HAM>(S, P, A.h, y, y1, sr);
            ++taken;
            bool accept;
            st = terminate_f64(S, A.r_escape, sr, y1, accept);
            if (accept) copy8(y, y1);
            if (st != kActive) break;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = y[k];
        A.status[i] = st;
        A.steps[i] += taken;
    }
    if (CKPT) {
        // slots up to the end of this launch (inclusive of the call's last slot when
        // this launch ends the call) repeat the current state for stopped lanes and
        // receive the end state otherwise
        const int32_t end = A.k0 + A.n_steps;
        int32_t last = end / A.ck_every;
        if (last * A.ck_every == end && last != A.ck_last) --last;  // next launch writes it
        for (int32_t s = next_slot; s <= last; ++s) put_slot(A, i, s, y);
    }
}

// One lane of the batch as a work item of the persistent driver; the step is the
// same rk4_step_f64 / terminate_f64 sequence as the one-thread-per-lane kernel.
template <bool HAM>
struct F64Prog {
    const IntArgs &A;
    const Spacetime *table;  // LDS copy (mixed batch) or kernel argument
    bool multi;
    int32_t n_st;
    struct Lane {
        double y[8];
        Spacetime S;
        HamConst<double> P;
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
#pragma unroll
        for (int k = 0; k < 8; ++k) L.y[k] = A.state[k * A.n + i];
        L.P = ham_const(L.S.a, L.y[4], L.y[7]);
        L.taken = 0;
        return A.n_steps > 0;
    }
    __device__ __forceinline__ bool step(Lane &L)
    {
        double y1[8], sr[3];
        step_f64<HAM>(L.S, L.P, A.h, L.y, y1, sr);
        ++L.taken;
        bool accept = true;  // the common outcome of the stop rules first, as rk4_f64_kernel
        if (!still_active_f64(L.S, A.r_escape, sr, y1)) L.st = terminate_f64(L.S, A.r_escape, sr, y1, accept);
        if (accept) copy8(L.y, y1);
        return L.st != kActive || L.taken == A.n_steps;
    }
    __device__ __forceinline__ void store(int64_t item, const Lane &L)
    {
        const int64_t i = opaque(item);
#pragma unroll
        for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = L.y[k];
        A.status[i] = L.st;
        A.steps[i] += L.taken;
    }
    __device__ static __forceinline__ void state64(const Lane &L, double y[8]) { copy8(y, L.y); }
};

template <bool MULTI, bool HAM>
__global__ void __launch_bounds__(256) rk4_f64_persistent_kernel(IntArgs A, StTable T,
                                                                 unsigned long long *counter,
                                                                 int32_t chunk)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    F64Prog<HAM> P{A, lds_st, MULTI, T.n_st};
    persistent_loop(P, A.n, counter, chunk);
}

// The FP64 step with the invariant monitor folded in every K steps: one thread per
// lane, or the persistent work queue.
template <bool HAM>
__global__ void __launch_bounds__(256) rk4_f64_monitor_kernel(IntArgs A, StTable T, MonArgs MA,
                                                              int32_t multi)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    __shared__ double lds_mon[8 * kMonLanes];
    MonProg<F64Prog<HAM>, HAM> P{F64Prog<HAM>{A, lds_st, multi != 0, T.n_st}, MA, &lds_mon[threadIdx.x]};
    typename MonProg<F64Prog<HAM>, HAM>::Lane L;
    if (!P.load(i, L)) return;
    while (!P.step(L)) {
    }
    P.store(i, L);
}

template <bool HAM>
__global__ void __launch_bounds__(256) rk4_f64_monitor_persistent_kernel(IntArgs A, StTable T,
                                                                         MonArgs MA, int32_t multi,
                                                                         unsigned long long *counter,
                                                                         int32_t chunk)
{
    __shared__ Spacetime lds_st[kMaxSt];
    for (int k = threadIdx.x; k < T.n_st; k += blockDim.x) lds_st[k] = T.st[k];
    __syncthreads();
    __shared__ double lds_mon[8 * kMonLanes];
    MonProg<F64Prog<HAM>, HAM> P{F64Prog<HAM>{A, lds_st, multi != 0, T.n_st}, MA, &lds_mon[threadIdx.x]};
    persistent_loop(P, A.n, counter, chunk);
}

template <bool HAM>
int launch_monitor(const IntArgs &A, const StTable &T, const MonArgs &MA, bool multi, int block,
                   bool persistent, int32_t sub, unsigned long long *counter, hipStream_t s)
{
    if (persistent) {
        int grid = 0;
        int rc = persistent_grid((const void *)rk4_f64_monitor_persistent_kernel<HAM>, block, A.n, grid);
        if (rc) return rc;
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, counter);
        MALBEC_LAUNCH_CHECK("zero_u64_kernel");
        hipLaunchKernelGGL((rk4_f64_monitor_persistent_kernel<HAM>), dim3(grid), dim3(block), 0, s,
                           A, T, MA, (int32_t)multi, counter, sub);
        MALBEC_LAUNCH_CHECK("rk4_f64_monitor_persistent_kernel");
        return MALBEC_OK;
    }
    hipLaunchKernelGGL((rk4_f64_monitor_kernel<HAM>), dim3(grid_for(A.n, block)), dim3(block), 0, s,
                       A, T, MA, (int32_t)multi);
    MALBEC_LAUNCH_CHECK("rk4_f64_monitor_kernel");
    return MALBEC_OK;
}

template <bool MULTI, bool CKPT, bool HAM>
int launch_kernel(const IntArgs &A, const StTable &T, int block, hipStream_t s)
{
    if (!MULTI && !CKPT && T.st[0].M == 1.0)
        hipLaunchKernelGGL((rk4_f64_kernel<false, false, HAM, true>), dim3(grid_for(A.n, block)),
                           dim3(block), 0, s, A, T);
    else
        hipLaunchKernelGGL((rk4_f64_kernel<MULTI, CKPT, HAM>), dim3(grid_for(A.n, block)), dim3(block),
                           0, s, A, T);
    MALBEC_LAUNCH_CHECK("rk4_f64_kernel");
    return MALBEC_OK;
}

template <bool MULTI, bool HAM>
int launch_persistent(const IntArgs &A, const StTable &T, int block, int32_t sub,
                      unsigned long long *counter, hipStream_t s)
{
    int grid = 0;
    int rc = persistent_grid((const void *)rk4_f64_persistent_kernel<MULTI, HAM>, block, A.n, grid);
    if (rc) return rc;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, counter);
    MALBEC_LAUNCH_CHECK("zero_u64_kernel");
    hipLaunchKernelGGL((rk4_f64_persistent_kernel<MULTI, HAM>), dim3(grid), dim3(block), 0, s, A, T,
                       counter, sub);
    MALBEC_LAUNCH_CHECK("rk4_f64_persistent_kernel");
    return MALBEC_OK;
}

}  // namespace

int launch_integrate_f64(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                         int64_t n, double *state, int32_t *status, int32_t *steps,
                         double *checkpoints, void *ws, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const bool ham = run.formulation == MALBEC_FORM_HAMILTONIAN;
    if (ham && checkpoints && run.checkpoint_every > 0)
        return fail(MALBEC_ENOTSUP, "checkpoints need the Christoffel formulation");
    const int64_t total = run.n_steps;
    const int64_t chunk = run.steps_per_chunk > 0 ? run.steps_per_chunk : total;
    IntArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.ckpt = run.checkpoint_every > 0 ? checkpoints : nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    A.ck_every = run.checkpoint_every;
    A.ck_last = run.checkpoint_every > 0 ? (int32_t)(total / run.checkpoint_every) : 0;
    if (run.persistent) {
        if (A.ckpt) return fail(MALBEC_ENOTSUP, "checkpoints need the non-persistent kernel");
        // one launch runs all steps; steps_per_chunk is the retire/refill interval
        A.k0 = 0;
        A.n_steps = (int32_t)total;
        const int32_t sub = run.steps_per_chunk > 0 ? run.steps_per_chunk : 64;
        unsigned long long *counter = (unsigned long long *)ws;
        if (ham)
            return multi ? launch_persistent<true, true>(A, T, block, sub, counter, s)
                         : launch_persistent<false, true>(A, T, block, sub, counter, s);
        return multi ? launch_persistent<true, false>(A, T, block, sub, counter, s)
                     : launch_persistent<false, false>(A, T, block, sub, counter, s);
    }
    for (int64_t k0 = 0; k0 < total; k0 += chunk) {
        A.k0 = (int32_t)k0;
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        int rc;
        if (A.ckpt)
            rc = multi ? launch_kernel<true, true, false>(A, T, block, s)
                       : launch_kernel<false, true, false>(A, T, block, s);
        else if (ham)
            rc = multi ? launch_kernel<true, false, true>(A, T, block, s)
                       : launch_kernel<false, false, true>(A, T, block, s);
        else
            rc = multi ? launch_kernel<true, false, false>(A, T, block, s)
                       : launch_kernel<false, false, false>(A, T, block, s);
        if (rc) return rc;
    }
    return MALBEC_OK;
}

int launch_monitor_f64(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                       int64_t n, double *state, int32_t *status, int32_t *steps, int32_t every,
                       int32_t reset, double *mon, void *ws, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    const bool ham = run.formulation == MALBEC_FORM_HAMILTONIAN;
    const int64_t total = run.n_steps;
    IntArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.st_of_lane = multi ? st_of_lane : nullptr;
    A.ckpt = nullptr;
    A.h = run.h;
    A.r_escape = run.r_escape;
    A.ck_every = 0;
    A.ck_last = 0;
    A.k0 = 0;
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
        A.k0 = (int32_t)k0;
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        MA.reset = (k0 == 0) ? reset : 0;
        int rc = ham ? launch_monitor<true>(A, T, MA, multi, block, false, 0, counter, s)
                     : launch_monitor<false>(A, T, MA, multi, block, false, 0, counter, s);
        if (rc) return rc;
    }
    return MALBEC_OK;
}

}  // namespace malbec
