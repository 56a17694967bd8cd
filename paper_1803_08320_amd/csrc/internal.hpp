// Internal host-side declarations shared by the translation units of libmalbec.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/malbec.h"
#include "kerr_device.hpp"

namespace malbec {

// Records the error text for malbec_last_error() and returns `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define MALBEC_HIP_CHECK(expr)                                                              \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::malbec::fail(MALBEC_EDEVICE, "%s failed: %s", #expr,                   \
                                  hipGetErrorString(e_));                                   \
    } while (0)

#define MALBEC_LAUNCH_CHECK(name)                                                           \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess)                                                               \
            return ::malbec::fail(MALBEC_EDEVICE, "launch of %s failed: %s", name,          \
                                  hipGetErrorString(e_));                                   \
    } while (0)

constexpr int kMaxSt = MALBEC_MAX_SPACETIMES;

// Spacetime table passed by value in kernel arguments.
struct StTable {
    Spacetime st[kMaxSt];
    int32_t n_st;
};

// Validates a batch and fills the table (r_stop from horizon_factor, r_zone from
// zone_factor).  Returns MALBEC_OK or an error code with the text recorded.
int make_table(const malbec_batch *b, double horizon_factor, double zone_factor, StTable &T);

// Launchers (one per translation unit).  Arguments are validated by the caller.
int launch_init(const malbec_ic_spec &spec, const StTable &T, const int32_t *st_of_lane,
                int64_t n, double *state, double *consts, int64_t *attempts, hipStream_t s);
int launch_integrate_f64(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                         int64_t n, double *state, int32_t *status, int32_t *steps,
                         double *checkpoints, void *ws, hipStream_t s);
int launch_integrate_f32k(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                          int64_t n, double *state, int32_t *status, int32_t *steps, void *ws,
                          hipStream_t s);
// The same integrators with the invariant monitor every `every` steps (mon: 8n).
int launch_monitor_f64(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                       int64_t n, double *state, int32_t *status, int32_t *steps, int32_t every,
                       int32_t reset, double *mon, void *ws, hipStream_t s);
int launch_monitor_f32k(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                        int64_t n, double *state, int32_t *status, int32_t *steps, int32_t every,
                        int32_t reset, double *mon, void *ws, hipStream_t s);
// Grid of a persistent kernel: resident blocks per CU x CUs, capped by the blocks the
// work needs.
int persistent_grid(const void *kernel, int block, int64_t n_items, int &grid);
int launch_camera(const malbec_camera &cam, double r_stop, double disk_r_in, int32_t *status,
                  int32_t *steps, double *hit, double *final_state, void *ws, hipStream_t s);
int launch_adjoint(const malbec_run &run, const StTable &T, const int32_t *st_of_lane, int64_t n,
                   const double *checkpoints, const int32_t *status, const int32_t *steps,
                   const double *g_final, double *g_initial, const double *E_fixed,
                   double *g_named, void *ws, hipStream_t s);
int launch_invariants(const StTable &T, const int32_t *st_of_lane, int64_t n,
                      const double *state, double *out, hipStream_t s);
int launch_convert(const StTable &T, const int32_t *st_of_lane, int64_t n, double *state,
                   int32_t to_momenta, hipStream_t s);
// order: the work order of the persistent kernel (nullptr: index order).
int launch_adaptive(const malbec_adaptive &ad, const StTable &T, const int32_t *st_of_lane,
                    int64_t n, double *state, double *tau, double *h, int32_t *status,
                    int32_t *steps, int32_t *rejects, const uint32_t *order, void *ws,
                    hipStream_t s);
// Byte offsets in the workspace of the periapsis schedule of n lanes: bucket counts and
// running offsets (MALBEC_SCHED_BUCKETS uint32 each), keys and order (n uint32 each,
// 256-byte aligned); `order` is also the size without the order array.
struct SchedLayout {
    size_t count, next, key, order, bytes;
};
SchedLayout sched_layout(int64_t n);
// keys: nullptr = in the workspace.
int launch_adaptive_order(const StTable &T, const int32_t *st_of_lane, int64_t n,
                          const double *state, const double *tau, const int32_t *status,
                          double tau_end, uint32_t *order, uint32_t *keys, void *ws,
                          hipStream_t s);
int launch_grid_fill_kerr(const malbec_grid &g, double M, double a, void *nodes, hipStream_t s);
int launch_integrate_grid(const malbec_run &run, const malbec_grid &g, int64_t n, double *state,
                          int32_t *status, int32_t *steps, hipStream_t s);
int launch_integrate_record(const malbec_run &run, const StTable &T, const int32_t *st_of_lane,
                            int64_t n, double *state, int32_t *status, int32_t *steps,
                            int32_t record_every, double *traj, hipStream_t s);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace malbec
