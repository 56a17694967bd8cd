// C ABI entry points of libmalbec: argument validation, error text, dispatch to
// the kernel launchers of the other translation units.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "internal.hpp"

namespace malbec {

static thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

int persistent_grid(const void *kernel, int block, int64_t n_items, int &grid)
{
    int dev = 0;
    MALBEC_HIP_CHECK(hipGetDevice(&dev));
    int n_cu = 0;
    MALBEC_HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0;
    MALBEC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
    if (per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)n_cu * per_cu;
    const int64_t need = (n_items + block - 1) / block;
    if (g > need) g = need;
    if (g < 1) g = 1;
    grid = (int)g;
    return MALBEC_OK;
}

int make_table(const malbec_batch *b, double horizon_factor, double zone_factor, StTable &T)
{
    if (!b || !b->st) return fail(MALBEC_EINVAL, "batch or batch->st is NULL");
    if (b->n_st < 1 || b->n_st > kMaxSt)
        return fail(MALBEC_EINVAL, "n_st = %d outside [1, %d]", b->n_st, kMaxSt);
    if (!(horizon_factor >= 1.0) || !isfinite(horizon_factor))
        return fail(MALBEC_EINVAL, "horizon_factor = %g must be >= 1", horizon_factor);
    T.n_st = b->n_st;
    for (int k = 0; k < b->n_st; ++k) {
        double M = b->st[k].M, a = b->st[k].a;
        if (!(M > 0.0) || !isfinite(M)) return fail(MALBEC_EINVAL, "spacetime %d: M = %g must be > 0", k, M);
        if (!(a >= 0.0) || !(a <= M))
            return fail(MALBEC_EINVAL, "spacetime %d: a = %g outside [0, M = %g]", k, a, M);
        double rp = M + sqrt(M * M - a * a);
        T.st[k].M = M;
        T.st[k].a = a;
        T.st[k].r_stop = horizon_factor * rp;
        T.st[k].r_zone = zone_factor * rp;
    }
    for (int k = b->n_st; k < kMaxSt; ++k) T.st[k] = T.st[0];
    return MALBEC_OK;
}

}  // namespace malbec

using namespace malbec;

namespace {

// Argument checks shared by malbec_integrate and malbec_integrate_monitored.
int check_run(const malbec_run *run, int64_t n, const double *state, const int32_t *status,
              const int32_t *steps, const double *checkpoints, const void *ws, size_t ws_bytes)
{
    if (!run) return fail(MALBEC_EINVAL, "run is NULL");
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0 && (!state || !status || !steps))
        return fail(MALBEC_EINVAL, "state, status and steps must be non-NULL");
    if (n > ((int64_t)1 << 40)) return fail(MALBEC_EINVAL, "n too large");
    if (!(run->h > 0.0) || !isfinite(run->h)) return fail(MALBEC_EINVAL, "h = %g must be > 0", run->h);
    if (run->n_steps < 0 || run->n_steps > INT32_MAX)
        return fail(MALBEC_EINVAL, "n_steps = %lld outside [0, 2^31)", (long long)run->n_steps);
    if (!(run->r_escape > 0.0)) return fail(MALBEC_EINVAL, "r_escape must be > 0");
    if (run->block < 0 || run->block > 1024 || (run->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block = %d must be a multiple of 64 in [64, 1024] or 0", run->block);
    if (run->steps_per_chunk < 0) return fail(MALBEC_EINVAL, "steps_per_chunk < 0");
    if (run->checkpoint_every < 0) return fail(MALBEC_EINVAL, "checkpoint_every < 0");
    if (run->checkpoint_every > 0 && !checkpoints)
        return fail(MALBEC_EINVAL, "checkpoint_every > 0 needs a checkpoints buffer");
    if (run->persistent != 0 && run->persistent != 1) return fail(MALBEC_EINVAL, "persistent must be 0 or 1");
    if (run->persistent && run->checkpoint_every > 0)
        return fail(MALBEC_ENOTSUP, "checkpoints need persistent = 0");
    if (run->formulation != MALBEC_FORM_CHRISTOFFEL && run->formulation != MALBEC_FORM_HAMILTONIAN)
        return fail(MALBEC_EINVAL, "unknown formulation %d", run->formulation);
    if (run->formulation == MALBEC_FORM_HAMILTONIAN) {
        if (run->checkpoint_every > 0)
            return fail(MALBEC_ENOTSUP, "checkpoints need the Christoffel formulation");
    }
    size_t need = malbec_workspace_bytes(MALBEC_OP_INTEGRATE, n, run->persistent);
    if (ws_bytes < need || (need > 0 && !ws))
        return fail(MALBEC_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    if (run->precision == MALBEC_F32_KAHAN && !(run->fp64_zone_factor >= 1.0))
        return fail(MALBEC_EINVAL, "fp64_zone_factor = %g must be >= 1", run->fp64_zone_factor);
    if (run->precision != MALBEC_F64 && run->precision != MALBEC_F32_KAHAN)
        return fail(MALBEC_EINVAL, "unknown precision %d", run->precision);
    return MALBEC_OK;
}

}  // namespace

extern "C" {

const char *malbec_last_error(void) { return g_err; }

int malbec_version(void) { return 10000 * 0 + 100 * 3 + 0; }

size_t malbec_workspace_bytes(int32_t op, int64_t n, int32_t aux)
{
    if (op == MALBEC_OP_CAMERA && n >= 0)  // work counter (own cache line), then the rays' initial states
        return 256 + (size_t)n * 8 * sizeof(double);
    if (op == MALBEC_OP_ADAPTIVE && aux == 2 && n >= 0)
        return 256 + sched_layout(n).bytes;  // work counter, then the periapsis order
    if ((op == MALBEC_OP_INTEGRATE || op == MALBEC_OP_ADAPTIVE) && aux)
        return 256;  // persistent kernel's work counter
    if (op == MALBEC_OP_ADAPTIVE_ORDER && n > 0) return sched_layout(n).order;
    if (op == MALBEC_OP_ADJOINT && n > 0 && aux > 0) return (size_t)aux * 8 * (size_t)n * sizeof(double);
    return 0;
}

int malbec_init_particles(const malbec_ic_spec *spec, const malbec_batch *b, int64_t n,
                          double *state, double *consts, int64_t *attempts, void *stream)
{
    clear_error();
    if (!spec) return fail(MALBEC_EINVAL, "spec is NULL");
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0 && !state) return fail(MALBEC_EINVAL, "state is NULL");
    StTable T;
    int rc = make_table(b, 1.0, 1.0, T);
    if (rc) return rc;
    switch (spec->mode) {
    case MALBEC_IC_CANONICAL:
        if (n > 0 && !spec->rows) return fail(MALBEC_EINVAL, "CANONICAL mode needs spec->rows");
        break;
    case MALBEC_IC_CIRCULAR:
        if (!(spec->r_lo > 0) || !(spec->r_hi >= spec->r_lo))
            return fail(MALBEC_EINVAL, "CIRCULAR: need 0 < r_lo <= r_hi");
        break;
    case MALBEC_IC_PARAMS:
        if (n > 0 && !spec->rows) return fail(MALBEC_EINVAL, "PARAMS mode needs spec->rows");
        break;
    case MALBEC_IC_CONSTANTS:
        if (spec->max_attempts < 1 || spec->max_attempts >= (1 << 20))
            return fail(MALBEC_EINVAL, "max_attempts = %lld outside [1, 2^20)",
                        (long long)spec->max_attempts);
        if (!(spec->mu2 == 0.0 || spec->mu2 == 1.0))
            return fail(MALBEC_EINVAL, "mu2 = %g must be 0 (null) or 1 (timelike)", spec->mu2);
        {
            const double *rg[5] = {spec->r_range, spec->th_range, spec->E_range, spec->Lz_range,
                                   spec->Q_range};
            for (int k = 0; k < 5; ++k)
                if (!(rg[k][1] >= rg[k][0]) || !isfinite(rg[k][0]) || !isfinite(rg[k][1]))
                    return fail(MALBEC_EINVAL, "range %d is empty or not finite", k);
        }
        break;
    default:
        return fail(MALBEC_EINVAL, "unknown IC mode %d", spec->mode);
    }
    if (spec->lane0 < 0 || spec->lane0 + n > ((int64_t)1 << 39))
        return fail(MALBEC_EINVAL, "lane range exceeds the 2^39 counter space");
    if (n == 0) return MALBEC_OK;
    return launch_init(*spec, T, b->st_of_lane, n, state, consts, attempts, (hipStream_t)stream);
}


int malbec_integrate(const malbec_run *run, const malbec_batch *b, int64_t n, double *state,
                     int32_t *status, int32_t *steps, double *checkpoints, void *ws,
                     size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_run(run, n, state, status, steps, checkpoints, ws, ws_bytes);
    if (rc) return rc;
    double zone = run->precision == MALBEC_F32_KAHAN ? run->fp64_zone_factor : 1.0;
    StTable T;
    rc = make_table(b, run->horizon_factor, zone, T);
    if (rc) return rc;
    if (run->precision == MALBEC_F32_KAHAN && run->checkpoint_every > 0)
        return fail(MALBEC_ENOTSUP, "checkpoints are FP64 only");
    if (n == 0 || run->n_steps == 0) {
        if (run->checkpoint_every > 0 && n > 0)
            return fail(MALBEC_ENOTSUP, "checkpoints with n_steps = 0");
        return MALBEC_OK;
    }
    if (run->precision == MALBEC_F64)
        return launch_integrate_f64(*run, T, b->st_of_lane, n, state, status, steps, checkpoints,
                                    ws, (hipStream_t)stream);
    return launch_integrate_f32k(*run, T, b->st_of_lane, n, state, status, steps, ws,
                                 (hipStream_t)stream);
}

int malbec_integrate_monitored(const malbec_run *run, const malbec_batch *b, int64_t n,
                               double *state, int32_t *status, int32_t *steps,
                               int32_t monitor_every, int32_t reset, double *monitor, void *ws,
                               size_t ws_bytes, void *stream)
{
    clear_error();
    if (run && run->checkpoint_every != 0)
        return fail(MALBEC_ENOTSUP, "the monitored integration writes no checkpoints");
    int rc = check_run(run, n, state, status, steps, nullptr, ws, ws_bytes);
    if (rc) return rc;
    if (monitor_every < 1) return fail(MALBEC_EINVAL, "monitor_every = %d must be >= 1", monitor_every);
    if (reset != 0 && reset != 1) return fail(MALBEC_EINVAL, "reset must be 0 or 1");
    if (n > 0 && !monitor) return fail(MALBEC_EINVAL, "monitor must be non-NULL");
    double zone = run->precision == MALBEC_F32_KAHAN ? run->fp64_zone_factor : 1.0;
    StTable T;
    rc = make_table(b, run->horizon_factor, zone, T);
    if (rc) return rc;
    if (n == 0 || run->n_steps == 0) return MALBEC_OK;
    if (run->precision == MALBEC_F64)
        return launch_monitor_f64(*run, T, b->st_of_lane, n, state, status, steps, monitor_every,
                                  reset, monitor, ws, (hipStream_t)stream);
    return launch_monitor_f32k(*run, T, b->st_of_lane, n, state, status, steps, monitor_every,
                               reset, monitor, ws, (hipStream_t)stream);
}

int malbec_trace_camera(const malbec_camera *cam, int32_t *status, int32_t *steps, double *hit,
                        double *final_state, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!cam) return fail(MALBEC_EINVAL, "cam is NULL");
    if (cam->nx < 1 || cam->ny < 1) return fail(MALBEC_EINVAL, "nx, ny must be >= 1");
    int64_t npix = (int64_t)cam->nx * cam->ny;
    if (npix > ((int64_t)1 << 31) - 1) return fail(MALBEC_EINVAL, "nx * ny too large");
    if (!status || !steps || !hit) return fail(MALBEC_EINVAL, "status, steps and hit must be non-NULL");
    if (!(cam->M > 0.0) || !(cam->a >= 0.0) || !(cam->a <= cam->M))
        return fail(MALBEC_EINVAL, "need M > 0 and 0 <= a <= M");
    if (!(cam->r_obs > 0.0) || !(cam->incl > 0.0) || !(cam->incl < M_PI))
        return fail(MALBEC_EINVAL, "need r_obs > 0 and 0 < incl < pi");
    if (!(cam->half_width > 0.0)) return fail(MALBEC_EINVAL, "half_width must be > 0");
    if (!(cam->h0 > 0.0) || !(cam->h_r0 > 0.0)) return fail(MALBEC_EINVAL, "need h0 > 0 and h_r0 > 0");
    if (!(cam->horizon_factor >= 1.0)) return fail(MALBEC_EINVAL, "horizon_factor must be >= 1");
    if (!(cam->r_escape > cam->r_obs))
        return fail(MALBEC_EINVAL, "r_escape must exceed r_obs");
    if (cam->max_steps < 1 || cam->max_steps > INT32_MAX)
        return fail(MALBEC_EINVAL, "max_steps outside [1, 2^31)");
    if (cam->block < 0 || cam->block > 1024 || (cam->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block must be a multiple of 64 in [64, 1024] or 0");
    if (cam->steps_per_chunk < 0) return fail(MALBEC_EINVAL, "steps_per_chunk < 0");
    size_t need = malbec_workspace_bytes(MALBEC_OP_CAMERA, npix, 0);
    if (ws_bytes < need || !ws)
        return fail(MALBEC_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    double M = cam->M, a = cam->a;
    double rp = M + sqrt(M * M - a * a);
    double r_in = cam->disk_r_in;
    if (r_in <= 0.0) {
        // prograde ISCO (Bardeen, Press & Teukolsky 1972)
        double chi = a / M;
        double Z1 = 1.0 + cbrt(1.0 - chi * chi) * (cbrt(1.0 + chi) + cbrt(1.0 - chi));
        double Z2 = sqrt(3.0 * chi * chi + Z1 * Z1);
        r_in = M * (3.0 + Z2 - sqrt((3.0 - Z1) * (3.0 + Z1 + 2.0 * Z2)));
    }
    return launch_camera(*cam, cam->horizon_factor * rp, r_in, status, steps, hit, final_state, ws,
                         (hipStream_t)stream);
}

int malbec_adjoint(const malbec_run *run, const malbec_batch *b, int64_t n,
                   const double *checkpoints, const int32_t *status, const int32_t *steps,
                   const double *g_final, double *g_initial, const double *E_fixed,
                   double *g_named, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!run) return fail(MALBEC_EINVAL, "run is NULL");
    if (n < 0) return fail(MALBEC_EINVAL, "n < 0");
    if (n > 0 && (!checkpoints || !status || !steps || !g_final || !g_initial))
        return fail(MALBEC_EINVAL, "checkpoints, status, steps, g_final and g_initial must be non-NULL");
    if (!(run->h > 0.0) || !isfinite(run->h)) return fail(MALBEC_EINVAL, "h must be > 0");
    if (run->n_steps < 1 || run->n_steps > INT32_MAX) return fail(MALBEC_EINVAL, "n_steps outside [1, 2^31)");
    if (run->checkpoint_every < 1) return fail(MALBEC_EINVAL, "checkpoint_every must be >= 1");
    if (run->precision != MALBEC_F64) return fail(MALBEC_ENOTSUP, "the adjoint is FP64 only");
    if (run->formulation != MALBEC_FORM_CHRISTOFFEL)
        return fail(MALBEC_ENOTSUP, "the adjoint differentiates the Christoffel formulation only");
    if (run->block < 0 || run->block > 1024 || (run->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block must be a multiple of 64 in [64, 1024] or 0");
    size_t need = malbec_workspace_bytes(MALBEC_OP_ADJOINT, n, run->checkpoint_every);
    if (ws_bytes < need || (need > 0 && !ws))
        return fail(MALBEC_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    StTable T;
    int rc = make_table(b, run->horizon_factor, 1.0, T);
    if (rc) return rc;
    if (n == 0) return MALBEC_OK;
    return launch_adjoint(*run, T, b->st_of_lane, n, checkpoints, status, steps, g_final, g_initial,
                          E_fixed, g_named, ws, (hipStream_t)stream);
}

int malbec_invariants(const malbec_batch *b, int64_t n, const double *state, double *out,
                      void *stream)
{
    clear_error();
    if (n < 0) return fail(MALBEC_EINVAL, "n < 0");
    if (n > 0 && (!state || !out)) return fail(MALBEC_EINVAL, "state and out must be non-NULL");
    StTable T;
    int rc = make_table(b, 1.0, 1.0, T);
    if (rc) return rc;
    if (n == 0) return MALBEC_OK;
    return launch_invariants(T, b->st_of_lane, n, state, out, (hipStream_t)stream);
}

int malbec_integrate_adaptive(const malbec_adaptive *ad, const malbec_batch *b, int64_t n,
                              double *state, double *tau, double *h, int32_t *status,
                              int32_t *steps, int32_t *rejects, void *ws, size_t ws_bytes,
                              void *stream)
{
    clear_error();
    if (!ad) return fail(MALBEC_EINVAL, "ad is NULL");
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0 && (!state || !tau || !h || !status || !steps || !rejects))
        return fail(MALBEC_EINVAL, "state, tau, h, status, steps and rejects must be non-NULL");
    if (n > ((int64_t)1 << 40)) return fail(MALBEC_EINVAL, "n too large");
    if (!isfinite(ad->tau_end)) return fail(MALBEC_EINVAL, "tau_end must be finite");
    if (!(ad->rtol > 0.0) || !(ad->atol > 0.0) || !isfinite(ad->rtol) || !isfinite(ad->atol))
        return fail(MALBEC_EINVAL, "rtol and atol must be finite and > 0");
    if (!(ad->fac > 0.0 && ad->fac <= 1.0)) return fail(MALBEC_EINVAL, "fac must be in (0, 1]");
    if (!(ad->facmin > 0.0 && ad->facmin <= 1.0 && ad->facmax >= 1.0 && isfinite(ad->facmax)))
        return fail(MALBEC_EINVAL, "need 0 < facmin <= 1 <= facmax");
    if (ad->max_attempts < 1) return fail(MALBEC_EINVAL, "max_attempts must be >= 1");
    if (!(ad->r_escape > 0.0)) return fail(MALBEC_EINVAL, "r_escape must be > 0");
    if (ad->block < 0 || ad->block > 1024 || (ad->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block = %d must be a multiple of 64 in [64, 1024] or 0", ad->block);
    if (ad->persistent != 0 && ad->persistent != 1) return fail(MALBEC_EINVAL, "persistent must be 0 or 1");
    if (ad->steps_per_chunk < 0) return fail(MALBEC_EINVAL, "steps_per_chunk < 0");
    if (ad->schedule != MALBEC_SCHED_INDEX && ad->schedule != MALBEC_SCHED_PERIAPSIS)
        return fail(MALBEC_EINVAL, "unknown schedule %d", ad->schedule);
    if (ad->schedule == MALBEC_SCHED_PERIAPSIS && !ad->persistent)
        return fail(MALBEC_EINVAL, "the periapsis schedule needs persistent = 1");
    if (ad->schedule == MALBEC_SCHED_PERIAPSIS && n > (int64_t)UINT32_MAX)
        return fail(MALBEC_EINVAL, "the periapsis schedule needs n < 2^32");
    size_t need = malbec_workspace_bytes(MALBEC_OP_ADAPTIVE, n,
                                         ad->persistent ? 1 + ad->schedule : 0);
    if (ws_bytes < need || (need > 0 && !ws))
        return fail(MALBEC_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    StTable T;
    int rc = make_table(b, ad->horizon_factor, 1.0, T);
    if (rc) return rc;
    if (n == 0) return MALBEC_OK;
    const uint32_t *order = nullptr;
    if (ad->schedule == MALBEC_SCHED_PERIAPSIS) {
        // the order sits after the work counter's 256 bytes
        void *sw = (char *)ws + 256;
        uint32_t *o = (uint32_t *)((char *)sw + sched_layout(n).order);
        rc = launch_adaptive_order(T, b->st_of_lane, n, state, tau, status, ad->tau_end, o,
                                   nullptr, sw, (hipStream_t)stream);
        if (rc) return rc;
        order = o;
    }
    return launch_adaptive(*ad, T, b->st_of_lane, n, state, tau, h, status, steps, rejects, order,
                           ws, (hipStream_t)stream);
}

int malbec_adaptive_order(const malbec_batch *b, int64_t n, const double *state,
                          const double *tau, const int32_t *status, double tau_end,
                          uint32_t *order, uint32_t *keys, void *ws, size_t ws_bytes,
                          void *stream)
{
    clear_error();
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > (int64_t)UINT32_MAX) return fail(MALBEC_EINVAL, "n must be < 2^32");
    if (n > 0 && (!state || !tau || !status || !order))
        return fail(MALBEC_EINVAL, "state, tau, status and order must be non-NULL");
    if (!isfinite(tau_end)) return fail(MALBEC_EINVAL, "tau_end must be finite");
    size_t need = malbec_workspace_bytes(MALBEC_OP_ADAPTIVE_ORDER, n, 0);
    if (ws_bytes < need || (need > 0 && !ws))
        return fail(MALBEC_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    StTable T;
    int rc = make_table(b, 1.0, 1.0, T);
    if (rc) return rc;
    return launch_adaptive_order(T, b->st_of_lane, n, state, tau, status, tau_end, order, keys,
                                 ws, (hipStream_t)stream);
}

static int check_grid(const malbec_grid *g)
{
    if (!g) return fail(MALBEC_EINVAL, "grid is NULL");
    if (g->nr < 4 || g->nth < 4) return fail(MALBEC_EINVAL, "the grid needs >= 4 nodes per axis");
    if ((int64_t)g->nr * g->nth > ((int64_t)1 << 31))
        return fail(MALBEC_EINVAL, "grid too large");
    if (!g->nodes) return fail(MALBEC_EINVAL, "grid nodes are NULL");
    if (g->node_precision != MALBEC_GRID_F64 && g->node_precision != MALBEC_GRID_F32)
        return fail(MALBEC_EINVAL, "unknown node_precision %d", g->node_precision);
    if (!(g->dr > 0.0) || !(g->dth > 0.0) || !isfinite(g->r0) || !isfinite(g->dr) ||
        !isfinite(g->th0) || !isfinite(g->dth))
        return fail(MALBEC_EINVAL, "need finite r0, th0 and dr, dth > 0");
    if (!(g->th0 > 0.0) || !(g->th0 + (double)(g->nth - 1) * g->dth < M_PI))
        return fail(MALBEC_EINVAL, "the theta range must lie inside (0, pi)");
    if (!(g->r0 > 0.0)) return fail(MALBEC_EINVAL, "r0 must be > 0");
    if (!(g->r_stop >= g->r0 + g->dr)) return fail(MALBEC_EINVAL, "r_stop must be >= r0 + dr");
    return MALBEC_OK;
}

int malbec_grid_fill_kerr(const malbec_grid *g, double M, double a, void *nodes, void *stream)
{
    clear_error();
    int rc = check_grid(g);
    if (rc) return rc;
    if (nodes != g->nodes) return fail(MALBEC_EINVAL, "nodes must be g->nodes");
    if (!(M > 0.0) || !(a >= 0.0) || !(a <= M)) return fail(MALBEC_EINVAL, "need M > 0 and 0 <= a <= M");
    if (!(g->r0 > M + sqrt(M * M - a * a)))
        return fail(MALBEC_EINVAL, "the grid must start outside the horizon");
    return launch_grid_fill_kerr(*g, M, a, nodes, (hipStream_t)stream);
}

int malbec_integrate_grid(const malbec_run *run, const malbec_grid *g, int64_t n, double *state,
                          int32_t *status, int32_t *steps, void *stream)
{
    clear_error();
    if (!run) return fail(MALBEC_EINVAL, "run is NULL");
    int rc = check_grid(g);
    if (rc) return rc;
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0 && (!state || !status || !steps))
        return fail(MALBEC_EINVAL, "state, status and steps must be non-NULL");
    if (n > ((int64_t)1 << 40)) return fail(MALBEC_EINVAL, "n too large");
    if (!(run->h > 0.0) || !isfinite(run->h)) return fail(MALBEC_EINVAL, "h = %g must be > 0", run->h);
    if (run->n_steps < 0 || run->n_steps > INT32_MAX)
        return fail(MALBEC_EINVAL, "n_steps = %lld outside [0, 2^31)", (long long)run->n_steps);
    if (run->block < 0 || run->block > 1024 || (run->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block = %d must be a multiple of 64 in [64, 1024] or 0", run->block);
    if (run->steps_per_chunk < 0) return fail(MALBEC_EINVAL, "steps_per_chunk < 0");
    if (run->formulation != MALBEC_FORM_HAMILTONIAN)
        return fail(MALBEC_EINVAL, "the gridded metric integrates (x, p): formulation must be HAMILTONIAN");
    if (run->precision != MALBEC_F64) return fail(MALBEC_ENOTSUP, "the gridded metric is FP64 only");
    if (run->persistent || run->checkpoint_every > 0)
        return fail(MALBEC_ENOTSUP, "the gridded metric runs without persistent kernel or checkpoints");
    if (!(run->r_escape > g->r_stop) || !(run->r_escape <= g->r0 + (double)(g->nr - 2) * g->dr))
        return fail(MALBEC_EINVAL, "r_escape must lie inside the grid, above r_stop");
    if (n == 0 || run->n_steps == 0) return MALBEC_OK;
    return launch_integrate_grid(*run, *g, n, state, status, steps, (hipStream_t)stream);
}

int malbec_integrate_record(const malbec_run *run, const malbec_batch *b, int64_t n, double *state,
                            int32_t *status, int32_t *steps, int32_t record_every, double *traj,
                            void *stream)
{
    clear_error();
    if (!run) return fail(MALBEC_EINVAL, "run is NULL");
    if (n < 0) return fail(MALBEC_EINVAL, "n = %lld < 0", (long long)n);
    if (n > 0 && (!state || !status || !steps || !traj))
        return fail(MALBEC_EINVAL, "state, status, steps and traj must be non-NULL");
    if (n > ((int64_t)1 << 40)) return fail(MALBEC_EINVAL, "n too large");
    if (!(run->h > 0.0) || !isfinite(run->h)) return fail(MALBEC_EINVAL, "h = %g must be > 0", run->h);
    if (run->n_steps < 0 || run->n_steps > INT32_MAX)
        return fail(MALBEC_EINVAL, "n_steps = %lld outside [0, 2^31)", (long long)run->n_steps);
    if (record_every < 1) return fail(MALBEC_EINVAL, "record_every = %d must be >= 1", record_every);
    if (run->n_steps % record_every != 0)
        return fail(MALBEC_EINVAL, "n_steps must be a multiple of record_every");
    if (!(run->r_escape > 0.0)) return fail(MALBEC_EINVAL, "r_escape must be > 0");
    if (run->block < 0 || run->block > 1024 || (run->block % 64) != 0)
        return fail(MALBEC_EINVAL, "block = %d must be a multiple of 64 in [64, 1024] or 0", run->block);
    if (run->formulation != MALBEC_FORM_CHRISTOFFEL && run->formulation != MALBEC_FORM_HAMILTONIAN)
        return fail(MALBEC_EINVAL, "unknown formulation %d", run->formulation);
    if (run->precision != MALBEC_F64) return fail(MALBEC_ENOTSUP, "trajectory recording is FP64 only");
    if (run->persistent || run->checkpoint_every > 0 || run->steps_per_chunk > 0)
        return fail(MALBEC_ENOTSUP, "trajectory recording runs one launch, without checkpoints");
    StTable T;
    int rc = make_table(b, run->horizon_factor, 1.0, T);
    if (rc) return rc;
    if (n == 0 || run->n_steps == 0) return MALBEC_OK;
    return launch_integrate_record(*run, T, b->st_of_lane, n, state, status, steps, record_every,
                                   traj, (hipStream_t)stream);
}

int malbec_convert_state(const malbec_batch *b, int64_t n, double *state, int32_t to_momenta,
                         void *stream)
{
    clear_error();
    if (n < 0) return fail(MALBEC_EINVAL, "n < 0");
    if (n > 0 && !state) return fail(MALBEC_EINVAL, "state must be non-NULL");
    if (to_momenta != 0 && to_momenta != 1) return fail(MALBEC_EINVAL, "to_momenta must be 0 or 1");
    StTable T;
    int rc = make_table(b, 1.0, 1.0, T);
    if (rc) return rc;
    if (n == 0) return MALBEC_OK;
    return launch_convert(T, b->st_of_lane, n, state, to_momenta, (hipStream_t)stream);
}

}  // extern "C"
