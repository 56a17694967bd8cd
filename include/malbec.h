/*
 * malbec.h - C ABI of the MI355X (gfx950) batched geodesic RK4 integrator.
 *
 * The method is that of G. D. Quiroga, "MALBEC: a new CUDA-C ray-tracer in
 * General Relativity" (arXiv:1803.08320): timelike and null geodesics of the
 * Kerr metric in Boyer-Lindquist coordinates (Section 2, eq. kerr; a = 0 is
 * Schwarzschild, Section 4), one independent particle or photon per lane,
 * advanced with the classic fourth-order Runge-Kutta method (Section 5), and
 * stopped per lane at the event horizon (Section 5: r <= 1 + sqrt(1 - a^2) for
 * M = 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units G = c = 1.  Coordinates x = (t, r, theta, phi), affine parameter tau
 *    (proper time for timelike geodesics).
 *  - State layout: double state[8 * n], component-major ("SoA"):
 *      state[k * n + i], k = 0..7 = (t, r, theta, phi, u^t, u^r, u^theta, u^phi),
 *    u^mu = dx^mu / dtau.  The geodesic ODE is dx/dtau = u,
 *    du^mu/dtau = -Gamma^mu_{ab} u^a u^b.
 *  - Pointers: "device" pointers are HIP device memory of the current device
 *    (for example torch tensors' data_ptr()); "host" pointers are CPU memory.
 *    Every buffer is owned by the caller.  The library allocates no device
 *    memory: scratch space, where needed, is the caller's workspace `ws`.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 *    Device work is enqueued asynchronously on it; a return of MALBEC_OK means
 *    the arguments were valid and the launches were enqueued, not that they
 *    finished.  Per-lane physics outcomes are lane status codes, never call
 *    errors.
 *  - Errors: every call returns one of the MALBEC_E* codes below; the text of
 *    the last error on the calling host thread is malbec_last_error().  On an
 *    argument error nothing is enqueued and no buffer is touched.
 *  - Calls on different streams are independent; calls that write the same
 *    buffers must be ordered by the caller.
 */
#ifndef MALBEC_H
#define MALBEC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define MALBEC_API __attribute__((visibility("default")))
#else
#define MALBEC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------------- */
#define MALBEC_OK 0
#define MALBEC_EINVAL (-1)  /* bad argument: null pointer, n < 0, M <= 0, a < 0 or a > M,
                               h <= 0, n_steps < 0, unknown enum, table too large */
#define MALBEC_ENOMEM (-2)  /* caller workspace smaller than malbec_workspace_bytes() */
#define MALBEC_EDEVICE (-3) /* a HIP runtime error (text in malbec_last_error()) */
#define MALBEC_ENOTSUP (-4) /* valid but unsupported combination */
#define MALBEC_ESAMPLE (-5) /* malbec_init_particles with strict = 1: some lanes exhausted
                               max_attempts (their state is NaN, attempts = max_attempts) */

/* ---- lane status (int32 per lane) ------------------------------------------------ */
#define MALBEC_ACTIVE 0    /* still integrating */
#define MALBEC_HORIZON 1   /* reached r <= horizon_factor * r_+ (Section 5 stop rule) */
#define MALBEC_ESCAPE 2    /* reached r >= r_escape */
#define MALBEC_DISK 3      /* crossed the thin equatorial disk (camera) */
#define MALBEC_NONFINITE 4 /* step result non-finite or theta left (0, pi) */
#define MALBEC_BUDGET 5    /* camera ray still active after max_steps */

/* ---- enums ----------------------------------------------------------------------- */
#define MALBEC_F64 0       /* FP64 throughout */
#define MALBEC_F32_KAHAN 1 /* FP32 state with compensated update, FP64 near the horizon */

/* Formulation of the geodesic ODE (malbec_run.formulation) and with it the meaning of
 * state components 4..7. */
#define MALBEC_FORM_CHRISTOFFEL 0 /* y = (x^mu, u^mu), du/dtau = -Gamma u u (default) */
#define MALBEC_FORM_HAMILTONIAN 1 /* z = (x^mu, p_mu), Hamilton's equations (Section 2,
                                     eq. Ham); p_t = -E and p_phi = L_z stay exact */

#define MALBEC_IC_CANONICAL 0 /* the paper's initial-condition rows (Section 5 table) */
#define MALBEC_IC_CIRCULAR 1  /* equatorial near-circular orbits (Sections 3-4) */
#define MALBEC_IC_CONSTANTS 2 /* random (E, L_z, Carter Q) with potential rejection */
#define MALBEC_IC_PARAMS 3    /* rows (r0, theta0, u^r0, u^theta0, L_z, E): the map the
                                 adjoint differentiates */

#define MALBEC_MAX_SPACETIMES 64

#define MALBEC_OP_INTEGRATE 1
#define MALBEC_OP_CAMERA 2
#define MALBEC_OP_ADJOINT 3
#define MALBEC_OP_ADAPTIVE 4
#define MALBEC_OP_ADAPTIVE_ORDER 5

/* Work order of the persistent adaptive kernel (malbec_adaptive.schedule). */
#define MALBEC_SCHED_INDEX 0      /* lanes in index order */
#define MALBEC_SCHED_PERIAPSIS 1  /* smallest periapsis first (malbec_adaptive_order) */
#define MALBEC_SCHED_BUCKETS 1024 /* keys of malbec_adaptive_order: 0 .. 1023 */
#define MALBEC_NOALLOC_MAX_LANES 2097152 /* batch limit of malbec_integrate_adaptive_noalloc */

/* One Kerr spacetime: mass M > 0 and spin a in [0, M] (Section 2; a > M is a naked
 * singularity and is rejected). */
typedef struct {
    double M;
    double a;
} malbec_spacetime;

/* A batch may mix spacetimes: lane i uses st[st_of_lane[i]]. */
typedef struct {
    const malbec_spacetime *st; /* host, n_st entries (copied during the call) */
    int32_t n_st;               /* 1 .. MALBEC_MAX_SPACETIMES */
    int32_t pad_;
    const int32_t *st_of_lane;  /* device, n entries in [0, n_st), or NULL: all lanes use st[0] */
} malbec_batch;

/* Initial-condition recipe (malbec_init_particles). */
typedef struct {
    int32_t mode;   /* MALBEC_IC_* */
    int32_t strict; /* CONSTANTS: 1 = count the lanes that exhaust max_attempts on the device,
                       wait for the stream and return MALBEC_ESAMPLE if there are any (a
                       blocking call); 0 = report them per lane only (asynchronous) */
    uint64_t seed;  /* SplitMix64 seed: draw k of attempt j of lane i is output
                       (i*2^24 + j*2^4 + k + 1) of the SplitMix64 sequence from `seed` */
    int64_t lane0;  /* global index of lane 0 of this call (sub-batches draw the same numbers) */
    double mu2;     /* 1 timelike, 0 null (CONSTANTS mode) */
    /* CIRCULAR: r0 = U[r_lo, r_hi), L = L_circ(r0) (1 + dL (2U - 1)), theta = pi/2,
       u^r = u^theta = 0; E from g(u,u) = -1 if e_from_norm else E_circ(r0). */
    double r_lo, r_hi, dL;
    int32_t prograde, e_from_norm;
    /* CONSTANTS: per attempt draw r0, theta0, E, L_z, Q uniformly in the ranges and the
       signs of u^r, u^theta; accept iff R(r0) >= 0 and Theta(theta0) >= 0. */
    double r_range[2], th_range[2], E_range[2], Lz_range[2], Q_range[2];
    int64_t max_attempts; /* lanes that exhaust it get NaN state and attempts = max_attempts */
    /* CANONICAL: device, n rows of 8 doubles (t, r, theta, phi, p_t, p_r, p_theta, p_phi),
       row-major as in the paper's IC table, with the paper's sign p_t = +E.
       PARAMS: device, n rows of 6 doubles (r0, theta0, u^r0, u^theta0, L_z, E): state
       (0, r0, theta0, 0, u^t, u^r0, u^theta0, u^phi) with (u^t, u^phi) = G^{-1} (-E, L_z),
       G the (t, phi) block of the metric at (r0, theta0). */
    const double *rows;
} malbec_ic_spec;

/* Integration controls (malbec_integrate). */
typedef struct {
    double h;                /* affine step, > 0 */
    int64_t n_steps;         /* RK4 steps per ACTIVE lane in this call, >= 0 */
    int32_t precision;       /* MALBEC_F64 or MALBEC_F32_KAHAN */
    int32_t block;           /* threads per block (multiple of 64, <= 1024), 0 = default */
    double horizon_factor;   /* stop at r <= horizon_factor * r_+ ; >= 1 (1.01 typical) */
    double r_escape;         /* stop at r >= r_escape */
    double fp64_zone_factor; /* F32_KAHAN: steps starting at r < factor * r_+ run in FP64 */
    int32_t steps_per_chunk; /* persistent = 0: steps per kernel launch (0 = all n_steps in
                                one launch); persistent = 1: steps between retire/refill
                                checks (0 = 64) */
    int32_t checkpoint_every;/* K > 0: write the state every K steps (see malbec_integrate) */
    int32_t persistent;      /* 1: persistent kernel refilling lanes that stop early from a
                                work counter in ws (needs persistent = 0 for checkpoints) */
    int32_t formulation;     /* MALBEC_FORM_*; HAMILTONIAN runs with F64 or F32_KAHAN and
                                without checkpoints (MALBEC_ENOTSUP otherwise) */
} malbec_run;

/* Adaptive integration controls (malbec_integrate_adaptive): Dormand-Prince 5(4)
 * with the standard step-size controller. */
typedef struct {
    double tau_end;        /* each lane integrates until its tau reaches tau_end */
    double rtol, atol;     /* weights sc_i = atol + rtol max(|y_i|, |y1_i|), > 0 */
    double fac;            /* safety factor, in (0, 1] (0.9 typical) */
    double facmin, facmax; /* bounds of h_new / h, 0 < facmin <= 1 <= facmax */
    int64_t max_attempts;  /* attempts per lane per call, >= 1; BUDGET when used up */
    double horizon_factor; /* stop at r <= horizon_factor * r_+ ; >= 1 */
    double r_escape;       /* stop at r >= r_escape */
    int32_t block;         /* threads per block, 0 = default */
    int32_t persistent;    /* 1: work-queue kernel (lanes need different attempt counts) */
    int32_t steps_per_chunk; /* persistent: attempts between retire/refill checks, 0 = 8 */
    int32_t schedule;      /* persistent: MALBEC_SCHED_INDEX (0) or MALBEC_SCHED_PERIAPSIS
                              (hand out the lanes in the order of malbec_adaptive_order);
                              the results do not depend on it */
} malbec_adaptive;

/* Storage of the node values of a malbec_grid (the interpolation and every other
 * operation run in FP64 either way). */
#define MALBEC_GRID_F64 0 /* double */
#define MALBEC_GRID_F32 1 /* float: half the bytes gathered per right-hand side, which
                             set the gridded kernel's rate, at a rounding of the stored
                             functions of 2^-24 relative */

/* A stationary, axisymmetric metric in 3+1 form (Section 2, eq. ADM) sampled on a
 * uniform (r, theta) grid: shift beta = (0, 0, beta^phi), diagonal spatial metric.
 * Node (i, j) sits at r = r0 + i dr, theta = th0 + j dth and holds five values,
 * nodes[(i * nth + j) * 5 + k], k = (alpha, beta^phi, gamma_rr, gamma_thth,
 * gamma_phph / sin^2 theta), stored as node_precision says. */
typedef struct {
    int32_t nr, nth;        /* nodes in r and theta, >= 4 each */
    double r0, dr;          /* dr > 0 */
    double th0, dth;        /* dth > 0; th0 > 0 and th0 + (nth - 1) dth < pi */
    double r_stop;          /* lanes stop at r <= r_stop (e.g. 1.01 r_+); >= r0 + dr */
    const void *nodes;      /* device, nr * nth * 5 doubles or floats */
    int32_t node_precision; /* MALBEC_GRID_F64 (0) or MALBEC_GRID_F32 (1) */
    int32_t pad_;
} malbec_grid;

/* Camera (malbec_trace_camera): Bardeen image plane of a static observer at
 * (r_obs, theta = incl, phi = 0); pixel p = j * nx + i, alpha = -w + (i + 1/2) 2w / nx,
 * beta = -w + (j + 1/2) 2w / ny.  Photon: E = 1, L_z = -alpha sin(incl),
 * Q = beta^2 + cos^2(incl) (alpha^2 - a^2), arriving with u^r > 0 and
 * sign(u^theta) = sign(beta); traced backward by negating u.  Step
 * h = h0 * max(1, r_n / h_r0).  Disk: thin, equatorial, disk_r_in <= r <= disk_r_out
 * (disk_r_in <= 0 selects the prograde ISCO). */
typedef struct {
    double M, a;
    double r_obs, incl, half_width;
    int32_t nx, ny;
    double h0, h_r0;
    double r_escape, horizon_factor;
    double disk_r_in, disk_r_out;
    int64_t max_steps;
    int32_t block;           /* threads per block, 0 = default */
    int32_t steps_per_chunk; /* steps between retire/refill checks, 0 = default */
    int32_t persistent;      /* 1: persistent work-queue kernel (default), 0: one lane per pixel */
    int32_t pad_;
} malbec_camera;

/* Text of the last error on this host thread ("" if none).  Valid until the next
 * call on the same thread. */
MALBEC_API const char *malbec_last_error(void);

/* Library version as 10000 * major + 100 * minor + patch. */
MALBEC_API int malbec_version(void);

/* Bytes of caller workspace an operation needs: op = MALBEC_OP_INTEGRATE (n lanes,
 * aux = run->persistent), MALBEC_OP_CAMERA (n = nx * ny pixels: 256 + 64n bytes), MALBEC_OP_ADJOINT
 * (n lanes, aux = the checkpoint interval K: K * 8 * n doubles),
 * MALBEC_OP_ADAPTIVE (n lanes, aux = ad->persistent ? 1 + ad->schedule : 0; about
 * 8n bytes with the periapsis schedule) or MALBEC_OP_ADAPTIVE_ORDER (n lanes, aux
 * unused; about 4n bytes).  Returns 0 for operations that need none. */
MALBEC_API size_t malbec_workspace_bytes(int32_t op, int64_t n, int32_t aux);

/* Build the initial state of n lanes on the device (one GPU thread per lane).
 * spec: host.  b: host (st_of_lane device or NULL).  state: device, 8n doubles (out).
 * consts: device, 4n doubles (out, nullable): (E, L_z, Q, mu2) component-major;
 * attempts: device, n int64 (out, nullable): draws used by the CONSTANTS sampler.
 * Passages: Section 5 IC table (CANONICAL; u^mu = g^{mu nu} p_nu with p_t = -E),
 * Sections 3-4 circular orbits (CIRCULAR), Carter's separated equations (CONSTANTS).
 * Errors: MALBEC_EINVAL on bad arguments; lanes whose sampler is exhausted are
 * reported through attempts == max_attempts and a NaN state; with spec->strict = 1
 * (CONSTANTS mode) the call also counts them on the device, waits for the stream and
 * returns MALBEC_ESAMPLE when there are any (their number in malbec_last_error()).
 * The count lives in a file-scope device variable of the library (one per GPU), so
 * strict calls that overlap on one GPU race; MALBEC_EDEVICE if its lookup fails. */
MALBEC_API int malbec_init_particles(const malbec_ic_spec *spec, const malbec_batch *b, int64_t n,
                          double *state, double *consts, int64_t *attempts, void *stream);

/* Advance every ACTIVE lane by up to run->n_steps classic RK4 steps of size run->h
 * (Section 5).  state: device 8n (in/out); status, steps: device n int32 (in/out;
 * steps accumulates the steps each lane evaluated).  After each step the lane stops,
 * in this order, when: an RK4 stage point lies at r <= horizon_factor r_+ (HORIZON,
 * the step's start state kept); the result is non-finite or has theta outside (0, pi)
 * (NONFINITE, start state kept); r <= horizon_factor r_+ (HORIZON); r >= r_escape
 * (ESCAPE).  Lanes not ACTIVE on entry are not touched.  Calling twice with n_steps/2
 * gives bitwise the same result as one call with n_steps.  With run->formulation =
 * MALBEC_FORM_HAMILTONIAN the state holds (x^mu, p_mu) and the step is the RK4 step
 * of Hamilton's equations (Section 2, eq. Ham), under the same stop rules.
 * checkpoints: device (nullable, F64 only): if run->checkpoint_every = K > 0, slot
 * s = 0 .. n_steps/K receives the state after s*K steps of this call, at
 * checkpoints[s * 8n + k * n + i]; a lane stopped earlier repeats its final state.
 * ws / ws_bytes: caller workspace of malbec_workspace_bytes(MALBEC_OP_INTEGRATE, n,
 * run->persistent) bytes (the persistent kernel's work counter; 0 bytes otherwise).
 * Errors: MALBEC_EINVAL, MALBEC_ENOMEM, MALBEC_EDEVICE. */
MALBEC_API int malbec_integrate(const malbec_run *run, const malbec_batch *b, int64_t n, double *state,
                     int32_t *status, int32_t *steps, double *checkpoints, void *ws,
                     size_t ws_bytes, void *stream);

/* malbec_integrate with the invariant monitor inside the step loop.  The conserved
 * quantities of Kerr geodesics, E = -p_t and L_z = p_phi (Sections 3-4: the metric of
 * Section 2, eq. kerr, depends on neither t nor phi), the norm g(u,u) (the constraint
 * of eq. geo) and Carter's constant Q, are evaluated in FP64 after every step whose
 * index in the lane's life (its step count over all calls, steps[i]) is a multiple of
 * monitor_every, and |I - I_0| is folded into a running maximum per invariant.  For
 * the Hamiltonian formulation E and L_z are read off p_t and p_phi (their drift is
 * exactly 0) and the norm is g^{mu nu} p_mu p_nu.
 * monitor: device, 8 * n doubles, component-major (monitor[k * n + i]): rows 0..3 the
 * reference invariants I_0 = (E, L_z, Q, g(u,u)) of lane i, rows 4..7 the running
 * maxima of |E - E_0|, |L_z - L_z0|, |Q - Q_0|, |g(u,u) - g_0|.  reset = 1: lanes ACTIVE
 * on entry take I_0 from their entry state and start from maxima of 0 (rows 0..7
 * written); reset = 0: rows 0..7 are read and the maxima continue, so that calls of
 * n_steps / 2 each give bitwise the monitor of one call of n_steps.  Rows of lanes
 * not ACTIVE on entry are not touched; with n_steps = 0 the call does nothing.
 * Everything else (precision, formulation, persistent queue, steps_per_chunk, stop
 * rules, ws) is as in malbec_integrate, and state, status and steps end bitwise as
 * malbec_integrate leaves them; run->checkpoint_every must be 0 (MALBEC_ENOTSUP).
 * Errors: MALBEC_EINVAL (also monitor_every < 1, reset not 0/1, monitor NULL with
 * n > 0), MALBEC_ENOMEM, MALBEC_ENOTSUP, MALBEC_EDEVICE. */
MALBEC_API int malbec_integrate_monitored(const malbec_run *run, const malbec_batch *b, int64_t n,
                                          double *state, int32_t *status, int32_t *steps,
                                          int32_t monitor_every, int32_t reset, double *monitor,
                                          void *ws, size_t ws_bytes, void *stream);

/* malbec_integrate (FP64, either formulation, one launch) that also records the
 * paper's trajectory output (Section 5: affine parameter tau, coordinate time t and
 * the Cartesian position of Section 2, eq. coord, x = sqrt(r^2 + a^2) sin(theta)
 * cos(phi), y = sqrt(r^2 + a^2) sin(theta) sin(phi), z = r cos(theta)) every
 * record_every steps.  traj: device, (n_steps / record_every) * 5 * n doubles (out);
 * record s holds the lane after (s + 1) * record_every steps of this call at
 * traj[(s * 5 + k) * n + i], k = (tau, t, x, y, z), tau = h * steps[i] (steps
 * accumulated over calls, so lanes that start at tau = 0 with steps = 0 report their
 * affine parameter).  A lane that has stopped repeats its last record.  n_steps must
 * be a multiple of record_every; run->persistent, checkpoint_every and
 * steps_per_chunk must be 0 (MALBEC_ENOTSUP otherwise).  The state, status and steps
 * end exactly as malbec_integrate leaves them.
 * Errors: MALBEC_EINVAL, MALBEC_ENOTSUP, MALBEC_EDEVICE. */
MALBEC_API int malbec_integrate_record(const malbec_run *run, const malbec_batch *b, int64_t n,
                                       double *state, int32_t *status, int32_t *steps,
                                       int32_t record_every, double *traj, void *stream);

/* Trace the nx * ny pixels of a camera backward until each photon stops (status
 * HORIZON, ESCAPE, DISK, NONFINITE or BUDGET), with the rules of malbec_integrate
 * plus: DISK when the equatorial plane is crossed between y_n and y_{n+1}
 * (signbit of cos theta differs) at r_c = r_n + (r_{n+1} - r_n) c_n / (c_n - c_{n+1})
 * inside [disk_r_in, disk_r_out] (checked after NONFINITE, before HORIZON).
 * status, steps: device nx*ny int32 (out).  hit: device 2*nx*ny doubles (out),
 * component-major (r_c, phi_c), NaN unless DISK.  final_state: device 8*nx*ny
 * (out, nullable).  ws: caller workspace of malbec_workspace_bytes(MALBEC_OP_CAMERA,
 * nx*ny) bytes (the persistent kernel's work counter and the rays' initial states,
 * 256 + 64 nx*ny bytes).
 * Errors: MALBEC_EINVAL, MALBEC_ENOMEM, MALBEC_EDEVICE. */
MALBEC_API int malbec_trace_camera(const malbec_camera *cam, int32_t *status, int32_t *steps, double *hit,
                        double *final_state, void *ws, size_t ws_bytes, void *stream);

/* Invariants of n states: out (device, 4n doubles, component-major) =
 * (E, L_z, Q, g(u,u)) with E = -(g_tt u^t + g_tphi u^phi) and L_z = g_tphi u^t +
 * g_phiphi u^phi (the conserved momenta, dp_t/dtau = dp_phi/dtau = 0 in Sections 3-4),
 * Carter's Q = (rho^2 u^theta)^2 + cos^2 theta [a^2 (mu^2 - E^2) + L_z^2 / sin^2 theta]
 * with mu^2 = -g(u,u), and the norm g(u,u) (= -1 timelike, eq. geo; 0 null).
 * Errors: MALBEC_EINVAL, MALBEC_EDEVICE. */
MALBEC_API int malbec_invariants(const malbec_batch *b, int64_t n, const double *state, double *out,
                      void *stream);

/* Adaptive FP64 integration (Christoffel form) of every ACTIVE lane with tau < tau_end
 * by the embedded Runge-Kutta pair of Dormand and Prince, 5(4) (the paper's Section 5
 * integrates with classic RK4 and announces other members of the family).  An attempt
 * of size h from y gives y1 (5th order) and the difference e to the 4th-order
 * companion; err = sqrt(mean_i (e_i / (atol + rtol max(|y_i|, |y1_i|)))^2); the attempt
 * is accepted iff err <= 1; the next size is h min(F, max(facmin, fac err^(-1/5))),
 * F = 1 right after a rejection and facmax otherwise; an attempt that would pass
 * tau_end is shortened to end on it.  Stops: a stage point at r <= horizon_factor r_+
 * (HORIZON) or a non-finite / off-range (theta outside (0, pi)) result or error
 * (NONFINITE) end the lane with the start state kept; an accepted step reaching
 * r <= horizon_factor r_+ (HORIZON) or r >= r_escape (ESCAPE); max_attempts attempts
 * in this call without reaching tau_end (BUDGET).
 * state: device 8n (in/out); tau, h: device n doubles (in/out: affine parameter and
 * the next step size); status: device n (in/out); steps, rejects: device n int32
 * (accumulate accepted and rejected attempts).  ws: caller workspace of
 * malbec_workspace_bytes(MALBEC_OP_ADAPTIVE, n, ad->persistent ? 1 + ad->schedule : 0)
 * bytes.  ad->schedule = MALBEC_SCHED_PERIAPSIS needs ad->persistent = 1 and n < 2^32;
 * it changes the order in which lanes are handed out, not their results.
 * Errors: MALBEC_EINVAL, MALBEC_ENOMEM, MALBEC_EDEVICE. */
MALBEC_API int malbec_integrate_adaptive(const malbec_adaptive *ad, const malbec_batch *b,
                                         int64_t n, double *state, double *tau, double *h,
                                         int32_t *status, int32_t *steps, int32_t *rejects,
                                         void *ws, size_t ws_bytes, void *stream);

/* Work order for the persistent adaptive kernel (ad->schedule = MALBEC_SCHED_PERIAPSIS
 * computes it in its workspace; this entry point exposes it).  Not an operation of the
 * paper: a schedule.  An adaptive integrator takes most of its attempts near the
 * orbit's closest approach, and a long lane handed out last keeps its wavefront busy
 * after the queue has drained, so the lanes expected to be longest go first.  The
 * expectation is ranked by the periapsis r_p of the lane's geodesic: the first zero,
 * inward from the lane's r, of the radial function of Carter's separation (the
 * constants of motion of Sections 3-4),
 *   R(r) = [E (r^2 + a^2) - a L_z]^2 - Delta [mu^2 r^2 + (L_z - a E)^2 + Q],
 * with (E, L_z, Q, mu^2 = -g(u,u)) as malbec_invariants gives them.  key[i] = the
 * largest j in [1, 1022] with r_j = r_+ 2^(j/32) <= r and R(r_j) < 0, found by a march
 * inward one bucket at a time from j = floor(32 log2(r / r_+)) (capped at 1022); 0 when
 * there is none (R(r_+) >= 0 always: the lane plunges, or its forbidden band is
 * narrower than a bucket; such lanes go first), and MALBEC_SCHED_BUCKETS - 1 = 1023 when
 * r < 2^(1/32) r_+ or the constants are not finite, and for every lane the integrator
 * skips (status not ACTIVE, tau >= tau_end, st_of_lane outside 0 .. n_st - 1).
 * order (device, n uint32, out): a permutation of 0 .. n-1 with key[order[k]]
 * non-decreasing in k; the order among equal keys is not specified (it may differ
 * between calls).  keys (device, n uint32, out, nullable): key[i].  state, tau, status:
 * device, as in malbec_integrate_adaptive (Christoffel form, read only).  ws: caller
 * workspace of malbec_workspace_bytes(MALBEC_OP_ADAPTIVE_ORDER, n, 0) bytes.  n must be
 * below 2^32.
 * Errors: MALBEC_EINVAL, MALBEC_ENOMEM, MALBEC_EDEVICE. */
MALBEC_API int malbec_adaptive_order(const malbec_batch *b, int64_t n, const double *state,
                                     const double *tau, const int32_t *status, double tau_end,
                                     uint32_t *order, uint32_t *keys, void *ws, size_t ws_bytes,
                                     void *stream);

/* malbec_integrate_adaptive without a caller workspace, for callers that cannot
 * allocate device memory around the call (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation).  Arguments, results and errors are those
 * of malbec_integrate_adaptive; the call allocates nothing: the work counter and the
 * periapsis work order use a static device array of the library (16 MiB + 8.4 KiB on
 * every GPU the library runs on, held until the process ends), so n is limited to
 * MALBEC_NOALLOC_MAX_LANES (2^21; larger n: MALBEC_EINVAL).  Every call on one GPU uses
 * that GPU's single array: calls that overlap on one GPU (concurrent streams or host
 * threads) race and give undefined results; calls in one stream order are safe (the
 * call clears what must start at zero). */
MALBEC_API int malbec_integrate_adaptive_noalloc(const malbec_adaptive *ad, const malbec_batch *b,
                                                 int64_t n, double *state, double *tau, double *h,
                                                 int32_t *status, int32_t *steps, int32_t *rejects,
                                                 void *stream);

/* Fill g->nodes (device, written through the pointer passed as `nodes`, which must be
 * g->nodes, in g->node_precision's type: each value computed in FP64, then rounded
 * to nearest) with the 3+1 functions of Kerr given in Section 2: alpha =
 * sqrt(rho^2 Delta / Sigma), beta^phi = -2 M a r / Sigma, gamma_rr = rho^2 / Delta,
 * gamma_thth = rho^2, gamma_phph / sin^2 theta = Sigma / rho^2 (the test metric of the
 * gridded path).  Errors: MALBEC_EINVAL, MALBEC_EDEVICE. */
MALBEC_API int malbec_grid_fill_kerr(const malbec_grid *g, double M, double a, void *nodes,
                                     void *stream);

/* Fixed-step RK4 of Hamilton's equations (Section 2, eq. Ham) in the gridded 3+1
 * metric g: the five functions and their r, theta derivatives are the tensor-product
 * 4-point Lagrange interpolant of the grid (stencil of nodes i-1 .. i+2 around the
 * point's cell, shifted inwards at the edges), the inverse metric is g^tt =
 * -1/alpha^2, g^tphi = beta^phi / alpha^2, g^phph = 1/gamma_phph - (beta^phi)^2 /
 * alpha^2, g^rr = 1/gamma_rr, g^thth = 1/gamma_thth.  state: device 8n, (x^mu, p_mu)
 * (run->formulation must be MALBEC_FORM_HAMILTONIAN); status, steps as in
 * malbec_integrate.  Stops after each step, the first RK4 stage point (in order) that
 * is at r <= g->r_stop (HORIZON) or outside the grid's interior [r0 + dr,
 * r0 + (nr - 2) dr] x [th0 + dth, th0 + (nth - 2) dth] (NONFINITE) deciding, both with
 * the start state kept; a non-finite or off-grid result (NONFINITE, start state kept);
 * r <= r_stop (HORIZON); r >= run->r_escape (ESCAPE), which must lie inside the grid.
 * run: h, n_steps, block, steps_per_chunk, r_escape are used; precision F64,
 * persistent 0, no checkpoints.  Errors: MALBEC_EINVAL, MALBEC_ENOTSUP, MALBEC_EDEVICE. */
MALBEC_API int malbec_integrate_grid(const malbec_run *run, const malbec_grid *g, int64_t n,
                                     double *state, int32_t *status, int32_t *steps,
                                     void *stream);

/* Convert n states in place between the two formulations: to_momenta = 1 lowers
 * the index, (x, u^mu) -> (x, p_mu = g_{mu nu} u^nu); to_momenta = 0 raises it,
 * (x, p_mu) -> (x, u^mu = g^{mu nu} p_nu), with the metric of Section 2, eq. kerr at
 * each lane's (r, theta).  state: device 8n (in/out).  The canonical momenta are the
 * covariant ones (p_t = -E; the paper's printed tables use +E).
 * Errors: MALBEC_EINVAL, MALBEC_EDEVICE. */
MALBEC_API int malbec_convert_state(const malbec_batch *b, int64_t n, double *state,
                                    int32_t to_momenta, void *stream);

/* Discrete adjoint of malbec_integrate (FP64): the exact gradient of the computed RK4
 * map.  Inputs describe a forward call made with run->checkpoint_every = K > 0 that
 * started with all lanes ACTIVE and steps = 0: checkpoints (device, (N/K + 1) * 8n),
 * status and steps (device n, as that call left them), run (same h, n_steps = N, K,
 * horizon_factor, r_escape, block).  g_final (device 8n) = dL/dy_N.
 * Outputs: g_initial (device 8n) = dL/dy_0; g_named (device 5n, nullable) = dL/dp
 * for p = (r0, theta0, u^r0, u^theta0, L_z) through the MALBEC_IC_PARAMS map with E
 * held fixed (E_fixed: device n, nullable: E is then taken from the initial state).
 * Steps a lane did not take (after it stopped, or a terminal step whose result was
 * discarded) contribute the identity.  ws: caller workspace of
 * malbec_workspace_bytes(MALBEC_OP_ADJOINT, n, K) bytes (recomputed segment states).
 * There is no derivative in the paper; this is the transposed tangent of the RK4
 * step of Section 5.  Errors: MALBEC_EINVAL, MALBEC_ENOMEM, MALBEC_EDEVICE. */
MALBEC_API int malbec_adjoint(const malbec_run *run, const malbec_batch *b, int64_t n,
                              const double *checkpoints, const int32_t *status,
                              const int32_t *steps, const double *g_final, double *g_initial,
                              const double *E_fixed, double *g_named, void *ws, size_t ws_bytes,
                              void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MALBEC_H */
