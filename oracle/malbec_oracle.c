/*
 * Plain FP64 CPU oracle for batched RK4 integration of Kerr / Schwarzschild
 * geodesics in Boyer-Lindquist coordinates (G. D. Quiroga, "MALBEC: a new
 * CUDA-C ray-tracer in General Relativity", arXiv:1803.08320).
 *
 * TEST INFRASTRUCTURE.  This library exists to check the GPU product path.  It
 * shares no code with it.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product never calls it.
 *
 * It is deliberately slow and literal: the Christoffel symbols are formed from
 * their definition with index loops (oracle_core.inc), RK4 is the textbook
 * tableau, and every lane is integrated on its own.  Build:
 *     gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 *
 * Readings of points the paper leaves open (each is repeated where used):
 *  - state y = (t, r, theta, phi, u^t, u^r, u^theta, u^phi), affine parameter tau;
 *  - termination after each step, in the order: a stage point inside the
 *    horizon zone (HORIZON, previous state kept) > NONFINITE (previous state
 *    kept) > DISK > HORIZON > ESCAPE > BUDGET (see integrate_lane);
 *  - horizon: r <= horizon_factor * r_+, r_+ = M + sqrt(M^2 - a^2) (Section 5
 *    stops at r <= 1 + sqrt(1 - a^2) with M = 1, i.e. horizon_factor = 1).
 *
 * Parity pins: see tests/test_oracle_*.py.  The gradient functions (complex
 * step) are pinned by finite differences and dot-product tests only: the paper
 * prints no gradient, so gradient parity is unpinned by the paper.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- instantiate the core for double -------------------------------------------- */
#define REAL double
#define FN(name) d_##name
#define RSIN sin
#define RCOS cos
#include "oracle_core.inc"
#undef REAL
#undef FN
#undef RSIN
#undef RCOS

/* ---- and for double complex (complex-step tangents) ------------------------------ */
#define REAL double complex
#define FN(name) z_##name
#define RSIN csin
#define RCOS ccos
#include "oracle_core.inc"
#undef REAL
#undef FN
#undef RSIN
#undef RCOS

/* lane status codes */
enum { ST_ACTIVE = 0, ST_HORIZON = 1, ST_ESCAPE = 2, ST_DISK = 3, ST_NONFINITE = 4, ST_BUDGET = 5 };

/* ================================================================================ */
/* Pointwise access for the tests                                                    */
/* ================================================================================ */

void oracle_metric(double M, double a, double r, double th, double *g16)
{
    double g[4][4];
    d_metric(M, a, r, th, g);
    memcpy(g16, g, sizeof g);
}

void oracle_metric_partials(double M, double a, double r, double th, double *dg64)
{
    double dg[4][4][4];
    d_metric_partials(M, a, r, th, dg);
    memcpy(dg64, dg, sizeof dg);
}

int oracle_inverse_metric(double M, double a, double r, double th, double *gi16)
{
    double g[4][4], gi[4][4];
    d_metric(M, a, r, th, g);
    int rc = d_inverse4(g, gi);
    memcpy(gi16, gi, sizeof gi);
    return rc;
}

void oracle_christoffel(double M, double a, double r, double th, double *G64)
{
    double G[4][4][4];
    d_christoffel(M, a, r, th, G);
    memcpy(G64, G, sizeof G);
}

void oracle_rhs(double M, double a, const double *y, double *f) { d_rhs(M, a, y, f); }
void oracle_rhs_hamiltonian(double M, double a, const double *z, double *f) { d_rhs_hamiltonian(M, a, z, f); }

/* complex-step partials of the metric itself (used to check the analytic ones):
 * d g / d x^l = Im g(x + i eps e_l) / eps. */
void oracle_metric_partials_complex_step(double M, double a, double r, double th, double *dg64)
{
    const double eps = 1e-30;
    double complex g[4][4];
    memset(dg64, 0, 64 * sizeof(double));
    z_metric(M, a, r + I * eps, th, g);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) dg64[1 * 16 + i * 4 + j] = cimag(g[i][j]) / eps;
    z_metric(M, a, r, th + I * eps, g);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) dg64[2 * 16 + i * 4 + j] = cimag(g[i][j]) / eps;
}

/* ================================================================================ */
/* Closed forms                                                                      */
/* ================================================================================ */

/* Outer horizon r_+ = M + sqrt(M^2 - a^2) (Section 3, after eq. (ISCO)). */
double oracle_r_horizon(double M, double a) { return M + sqrt(M * M - a * a); }

/* ISCO radius.  The closed form printed in Section 3 (eq. iscokerr) does not
 * evaluate to a real radius; the paper cites Bardeen, Press & Teukolsky (1972)
 * for the limits, and that reference's formula is used:
 *   chi = a/M, Z1 = 1 + (1-chi^2)^(1/3) [(1+chi)^(1/3) + (1-chi)^(1/3)],
 *   Z2 = sqrt(3 chi^2 + Z1^2),  r = M [3 + Z2 -/+ sqrt((3-Z1)(3+Z1+2 Z2))],
 * upper sign prograde (co-rotating). */
double oracle_r_isco(double M, double a, int prograde)
{
    double chi = a / M;
    double Z1 = 1.0 + cbrt(1.0 - chi * chi) * (cbrt(1.0 + chi) + cbrt(1.0 - chi));
    double Z2 = sqrt(3.0 * chi * chi + Z1 * Z1);
    double root = sqrt((3.0 - Z1) * (3.0 + Z1 + 2.0 * Z2));
    return M * (3.0 + Z2 + (prograde ? -root : root));
}

/* Energy and axial angular momentum of an equatorial circular orbit, in the
 * Bardeen-Press-Teukolsky form (upper sign prograde):
 *   E = (r^{3/2} - 2M r^{1/2} +/- a M^{1/2}) / (r^{3/4} sqrt(r^{3/2} - 3M r^{1/2} +/- 2a M^{1/2}))
 *   L = +/- M^{1/2} (r^2 -/+ 2a M^{1/2} r^{1/2} + a^2) / (same denominator). */
void oracle_circular_EL(double M, double a, double r, int prograde, double *E, double *L)
{
    double sg = prograde ? 1.0 : -1.0;
    double sr = sqrt(r), sM = sqrt(M);
    double den = pow(r, 0.75) * sqrt(r * sr - 3.0 * M * sr + sg * 2.0 * a * sM);
    *E = (r * sr - 2.0 * M * sr + sg * a * sM) / den;
    *L = sg * sM * (r * r - sg * 2.0 * a * sM * sr + a * a) / den;
}

/* The paper's own circular-orbit formulas (Section 3, eqs. energia, momento)
 * with R = r^2(-12M^3 r + 5M^2 a^2 + 16 M^2 r^2 - 3 M a^2 r - 7 M r^3 + r^4).
 * As printed they do not satisfy the paper's eq1/eq2 for a != 0; the reading
 * used here flips the sign in front of the a-term under the root and the sign
 * of the M a (...) term in L (both become -/+ for the +/- orbit), which makes
 * them satisfy eq1/eq2 and agree with the BPT form. */
void oracle_circular_EL_paper(double M, double a, double r, int prograde, double *E, double *L)
{
    double sg = prograde ? 1.0 : -1.0;
    double R = r * r * (-12.0 * M * M * M * r + 5.0 * M * M * a * a + 16.0 * M * M * r * r
                        - 3.0 * M * a * a * r - 7.0 * M * r * r * r + r * r * r * r);
    double D = R - sg * 2.0 * pow(M, 1.5) * pow(r, 1.5) * (2.0 * M * r - a * a - r * r) * a;
    *E = fabs(4.0 * M * M * r - M * a * a - 4.0 * M * r * r + r * r * r) / sqrt(D);
    *L = sg * fabs(-sg * M * a * (4.0 * M * r - a * a - 3.0 * r * r)
                   + pow(r, 1.5) * (2.0 * M * r - a * a - r * r) * sqrt(M)) / sqrt(D);
}

/* Schwarzschild circular orbits (Section 4, eqs. COrbit, COrbit2):
 * E^2 = (4M^2 - 4Mr + r^2) / (r (r - 3M)),  L^2 = M r^2 / (r - 3M). */
void oracle_schwarzschild_circular(double M, double r, double *E, double *L)
{
    *E = sqrt((4.0 * M * M - 4.0 * M * r + r * r) / (r * (r - 3.0 * M)));
    *L = sqrt(M * r * r / (r - 3.0 * M));
}

/* ================================================================================ */
/* Counter-based random numbers (SplitMix64, Steele, Lea & Flood, OOPSLA 2014)       */
/* ================================================================================ */
/* Draw k of attempt `attempt` of lane `lane` is output number (ctr + 1) of the
 * SplitMix64 sequence started at state `seed`, with
 * ctr = lane * 2^24 + attempt * 2^4 + k; i.e. mix(seed + (ctr + 1) * gamma). */
static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t oracle_draw_u64(uint64_t seed, uint64_t lane, uint64_t attempt, uint64_t k)
{
    uint64_t ctr = (lane << 24) | (attempt << 4) | k;
    return sm64_mix(seed + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
}

/* uniform in [0, 1) with 53 random bits */
static double draw_unit(uint64_t seed, uint64_t lane, uint64_t attempt, uint64_t k)
{
    return (double)(oracle_draw_u64(seed, lane, attempt, k) >> 11) * 0x1.0p-53;
}

static double draw_range(uint64_t seed, uint64_t lane, uint64_t attempt, uint64_t k, double lo, double hi)
{
    return lo + (hi - lo) * draw_unit(seed, lane, attempt, k);
}

static double draw_sign(uint64_t seed, uint64_t lane, uint64_t attempt, uint64_t k)
{
    return (oracle_draw_u64(seed, lane, attempt, k) >> 63) ? -1.0 : 1.0;
}

/* ================================================================================ */
/* Constants of motion <-> 4-velocity (Carter 1968; textbook, not in the paper)      */
/* ================================================================================ */
/* E = -(g_tt u^t + g_tphi u^phi) and L_z = g_tphi u^t + g_phiphi u^phi are the
 * conserved momenta -p_t and p_phi (the paper's eqs. show dp_t/dtau = dp_phi/dtau = 0);
 * mu^2 = -g(u,u) (constraint 2L = -1 of eq. (geo) for timelike, 0 for null);
 * Carter's constant Q = (rho^2 u^theta)^2 + cos^2(theta) [a^2 (mu^2 - E^2) + L_z^2 / sin^2(theta)].
 * out = (E, L_z, Q, g(u,u)). */
void oracle_invariants_one(double M, double a, const double *y, double *out)
{
    double g[4][4];
    d_metric(M, a, y[1], y[2], g);
    const double *u = y + 4;
    double norm = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) norm += g[i][j] * u[i] * u[j];
    double E = -(g[0][0] * u[0] + g[0][3] * u[3]);
    double Lz = g[0][3] * u[0] + g[3][3] * u[3];
    double s = sin(y[2]), c = cos(y[2]);
    double rho2 = y[1] * y[1] + a * a * c * c;
    double mu2 = -norm;
    double pth = rho2 * u[2];
    double Q = pth * pth + c * c * (a * a * (mu2 - E * E) + Lz * Lz / (s * s));
    out[0] = E;
    out[1] = Lz;
    out[2] = Q;
    out[3] = norm;
}

/* Radial and polar potentials of the separated Kerr geodesic equations:
 * P = E (r^2 + a^2) - a L_z,  R(r) = P^2 - Delta [mu^2 r^2 + (L_z - a E)^2 + Q],
 * Theta(theta) = Q - cos^2 [a^2 (mu^2 - E^2) + L_z^2 / sin^2]. */
double oracle_potential_R(double M, double a, double E, double Lz, double Q, double mu2, double r)
{
    double P = E * (r * r + a * a) - a * Lz;
    double Delta = r * r - 2.0 * M * r + a * a;
    return P * P - Delta * (mu2 * r * r + (Lz - a * E) * (Lz - a * E) + Q);
}

double oracle_potential_Theta(double a, double E, double Lz, double Q, double mu2, double th)
{
    double s = sin(th), c = cos(th);
    return Q - c * c * (a * a * (mu2 - E * E) + Lz * Lz / (s * s));
}

/* 4-velocity from (E, L_z, Q) at (r, theta) with chosen signs of u^r and u^theta:
 * rho^2 u^r = s_r sqrt(R), rho^2 u^theta = s_th sqrt(Theta),
 * rho^2 u^t = (r^2+a^2) P / Delta + a (L_z - a E sin^2),
 * rho^2 u^phi = a P / Delta + L_z / sin^2 - a E. */
void oracle_velocity_from_constants(double M, double a, double E, double Lz, double Q, double mu2,
                                    double r, double th, double sr, double sth, double *u)
{
    double s = sin(th), c = cos(th);
    double rho2 = r * r + a * a * c * c;
    double Delta = r * r - 2.0 * M * r + a * a;
    double P = E * (r * r + a * a) - a * Lz;
    double R = oracle_potential_R(M, a, E, Lz, Q, mu2, r);
    double Th = oracle_potential_Theta(a, E, Lz, Q, mu2, th);
    if (R < 0.0) R = 0.0;
    if (Th < 0.0) Th = 0.0;
    u[0] = ((r * r + a * a) * P / Delta + a * (Lz - a * E * s * s)) / rho2;
    u[1] = sr * sqrt(R) / rho2;
    u[2] = sth * sqrt(Th) / rho2;
    u[3] = (a * P / Delta + Lz / (s * s) - a * E) / rho2;
}

/* ================================================================================ */
/* Initial-condition builders (the oracle's own; the product has its own)            */
/* ================================================================================ */

static void put_state(double *state, int64_t n, int64_t i, const double y[8])
{
    for (int k = 0; k < 8; ++k) state[k * n + i] = y[k];
}

static void get_state(const double *state, int64_t n, int64_t i, double y[8])
{
    for (int k = 0; k < 8; ++k) y[k] = state[k * n + i];
}

/* Paper canonical rows (Section 5 IC table: t, r, theta, phi, p_t, p_r, p_theta, p_phi,
 * row-major, one row per particle) -> SoA state.  The table's p_t is +E
 * (Section 4: dt/dtau = p_t / (1 - 2M/r)), so the covariant momentum is
 * p = (-p_t, p_r, p_theta, p_phi) and u^mu = g^{mu nu} p_nu. */
int oracle_ic_canonical(double M, double a, int64_t n, const double *rows, double *state)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *z = rows + 8 * i;
        double g[4][4], gi[4][4];
        d_metric(M, a, z[1], z[2], g);
        if (d_inverse4(g, gi)) return -1;
        double p[4] = {-z[4], z[5], z[6], z[7]};
        double y[8] = {z[0], z[1], z[2], z[3], 0, 0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            double acc = 0.0;
            for (int nu = 0; nu < 4; ++nu) acc += gi[mu][nu] * p[nu];
            y[4 + mu] = acc;
        }
        put_state(state, n, i, y);
    }
    return 0;
}

/* Equatorial near-circular orbits.  r0 = U[r_lo, r_hi) (draw 0), delta =
 * dL (2 U - 1) (draw 1), L = L_circ(r0) (1 + delta), theta = pi/2, t = phi = 0,
 * u^r = u^theta = 0.  If e_from_norm, E is re-solved from g^{mu nu} p_mu p_nu = -1
 * with p = (-E, 0, 0, L) so the 4-velocity stays normalised; otherwise
 * E = E_circ(r0).  Then (u^t, u^phi) = g^{-1}(-E, L).  lane0 offsets the lane
 * counter so that sub-batches draw the same numbers as a full batch. */
int oracle_ic_circular(uint64_t seed, double M, double a, int64_t n, int64_t lane0, double r_lo,
                       double r_hi, double dL, int prograde, int e_from_norm, double *state)
{
    for (int64_t i = 0; i < n; ++i) {
        uint64_t lane = (uint64_t)(lane0 + i);
        double r0 = draw_range(seed, lane, 0, 0, r_lo, r_hi);
        double delta = dL * (2.0 * draw_unit(seed, lane, 0, 1) - 1.0);
        double Ec, Lc;
        oracle_circular_EL(M, a, r0, prograde, &Ec, &Lc);
        double L = Lc * (1.0 + delta);
        double th = M_PI / 2.0;
        double g[4][4], gi[4][4];
        d_metric(M, a, r0, th, g);
        d_inverse4(g, gi);
        double E = Ec;
        if (e_from_norm) {
            /* g^tt E^2 - 2 g^tphi L E + (g^phiphi L^2 + 1) = 0, g^tt < 0: take E > 0 */
            double A = gi[0][0], B = -2.0 * gi[0][3] * L, C = gi[3][3] * L * L + 1.0;
            double disc = B * B - 4.0 * A * C;
            E = (-B - sqrt(disc)) / (2.0 * A);
        }
        double y[8] = {0.0, r0, th, 0.0, 0, 0.0, 0.0, 0};
        y[4] = gi[0][0] * (-E) + gi[0][3] * L;
        y[7] = gi[3][0] * (-E) + gi[3][3] * L;
        put_state(state, n, i, y);
    }
    return 0;
}

/* Constants-of-motion sampler: per attempt draw (r0, theta0, E, L_z, Q, s_r, s_theta)
 * as draws 0..6 from their ranges; accept iff R(r0) >= 0 and Theta(theta0) >= 0;
 * then u from (E, L_z, Q).  Ma holds (M, a) per spacetime, st_of_lane (nullable)
 * picks the spacetime of each lane.  consts (4n, nullable) receives (E, L_z, Q, mu2)
 * as drawn; attempts (nullable) the number of attempts used.  Returns -5 if some
 * lane exhausted max_attempts (its state is left NaN). */
int oracle_ic_constants(uint64_t seed, const double *Ma, const int32_t *st_of_lane, int64_t n,
                        int64_t lane0, const double *ranges /* r,th,E,Lz,Q lo/hi pairs */,
                        double mu2, int64_t max_attempts, double *state, double *consts,
                        int64_t *attempts)
{
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t lane = (uint64_t)(lane0 + i);
        int st = st_of_lane ? st_of_lane[i] : 0;
        double M = Ma[2 * st], a = Ma[2 * st + 1];
        double y[8];
        int64_t att;
        int ok = 0;
        double E = 0, Lz = 0, Q = 0;
        for (att = 0; att < max_attempts; ++att) {
            double r0 = draw_range(seed, lane, att, 0, ranges[0], ranges[1]);
            double th0 = draw_range(seed, lane, att, 1, ranges[2], ranges[3]);
            E = draw_range(seed, lane, att, 2, ranges[4], ranges[5]);
            Lz = draw_range(seed, lane, att, 3, ranges[6], ranges[7]);
            Q = draw_range(seed, lane, att, 4, ranges[8], ranges[9]);
            double sr = draw_sign(seed, lane, att, 5);
            double sth = draw_sign(seed, lane, att, 6);
            if (oracle_potential_R(M, a, E, Lz, Q, mu2, r0) >= 0.0 &&
                oracle_potential_Theta(a, E, Lz, Q, mu2, th0) >= 0.0) {
                y[0] = 0.0; y[1] = r0; y[2] = th0; y[3] = 0.0;
                oracle_velocity_from_constants(M, a, E, Lz, Q, mu2, r0, th0, sr, sth, y + 4);
                ok = 1;
                break;
            }
        }
        if (!ok) {
            for (int k = 0; k < 8; ++k) y[k] = NAN;
            rc = -5;
        }
        put_state(state, n, i, y);
        if (consts) {
            consts[0 * n + i] = E;
            consts[1 * n + i] = Lz;
            consts[2 * n + i] = Q;
            consts[3 * n + i] = mu2;
        }
        if (attempts) attempts[i] = ok ? att + 1 : max_attempts;
    }
    return rc;
}

/* ================================================================================ */
/* Integration with termination                                                      */
/* ================================================================================ */

/* A step result is usable when every component is finite and theta stays inside
 * (0, pi): a fixed step that carries theta across a pole has not resolved the
 * 1/sin^2 theta terms of the metric (the coordinates are singular on the axis). */
static int usable(const double y[8])
{
    for (int k = 0; k < 8; ++k)
        if (!isfinite(y[k])) return 0;
    return y[2] > 0.0 && y[2] < M_PI;
}

/* Termination after one step from y_n to y_{n+1} (stage points Y2, Y3, Y4), with
 * r_stop = horizon_factor r_+.  Boyer-Lindquist coordinates are singular at
 * r_+, and a fixed step that probes r <= r_stop can blow up, so:
 *   1. some stage radius <= r_stop       -> HORIZON, y_n kept;
 *   2. y_{n+1} not usable (non-finite, or theta outside (0, pi))
 *                                        -> NONFINITE, y_n kept;
 *   3. (camera only) disk crossing       -> DISK, y_{n+1} stored;
 *   4. r_{n+1} <= r_stop                 -> HORIZON, y_{n+1} stored;
 *   5. r_{n+1} >= r_escape               -> ESCAPE, y_{n+1} stored.
 * Every evaluated step counts in the lane's step total, the terminal one too. */
static int stage_in_zone(const double sr[3], double r_stop)
{
    return sr[0] <= r_stop || sr[1] <= r_stop || sr[2] <= r_stop;
}

/* Fixed-step integration of one lane: up to n_steps RK4 steps while ACTIVE.
 * Returns the number of steps evaluated.  hamiltonian != 0: the state holds
 * (x^mu, p_mu) and the step is the canonical one; the termination rules read r and
 * theta from x and are the same for both formulations. */
static int64_t integrate_lane(double M, double a, double h, int64_t n_steps, double hf, double r_esc,
                              int hamiltonian, double y[8], int32_t *status)
{
    double rh = hf * oracle_r_horizon(M, a);
    int64_t n;
    for (n = 0; n < n_steps && *status == ST_ACTIVE; ++n) {
        double y1[8], sr[3];
        if (hamiltonian)
            d_rk4_step_hamiltonian_stages(M, a, h, y, y1, sr);
        else
            d_rk4_step_stages(M, a, h, y, y1, sr);
        if (stage_in_zone(sr, rh)) { *status = ST_HORIZON; continue; }
        if (!usable(y1)) { *status = ST_NONFINITE; continue; }
        memcpy(y, y1, sizeof y1);
        if (y[1] <= rh) *status = ST_HORIZON;
        else if (y[1] >= r_esc) *status = ST_ESCAPE;
    }
    return n;
}

/* Batch driver over SoA state[8n] (component-major), OpenMP over lanes.
 * status / steps are in/out; only ACTIVE lanes step; steps[i] accumulates. */
int oracle_integrate(const double *Ma, const int32_t *st_of_lane, int64_t n, double *state,
                     int32_t *status, int32_t *steps, double h, int64_t n_steps,
                     double horizon_factor, double r_escape, int hamiltonian, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int st = st_of_lane ? st_of_lane[i] : 0;
        double M = Ma[2 * st], a = Ma[2 * st + 1];
        double y[8];
        get_state(state, n, i, y);
        int64_t taken = integrate_lane(M, a, h, n_steps, horizon_factor, r_escape, hamiltonian, y,
                                       &status[i]);
        steps[i] += (int32_t)taken;
        put_state(state, n, i, y);
    }
    return 0;
}

/* The same four invariants of a canonical state z = (x^mu, p_mu): E = -p_t and
 * L_z = p_phi directly (the conserved momenta of Sections 3-4), the norm
 * g^{mu nu} p_mu p_nu with the inverse metric, p_theta as it stands. */
void oracle_invariants_hamiltonian_one(double M, double a, const double *z, double *out)
{
    double gi[4][4];
    oracle_inverse_metric(M, a, z[1], z[2], &gi[0][0]);
    const double *p = z + 4;
    double norm = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) norm += gi[i][j] * p[i] * p[j];
    double E = -p[0];
    double Lz = p[3];
    double s = sin(z[2]), c = cos(z[2]);
    double mu2 = -norm;
    double Q = p[2] * p[2] + c * c * (a * a * (mu2 - E * E) + Lz * Lz / (s * s));
    out[0] = E;
    out[1] = Lz;
    out[2] = Q;
    out[3] = norm;
}

/* Fixed-step integration with the invariant monitor: after every step whose index
 * in the lane's life (steps[i] after the step) is a multiple of `every`, the
 * invariants In of the lane's state update D_k = max(D_k, |In_k - I0_k|).
 * monitor[8n] (component-major): rows 0..3 I0, rows 4..7 D.  reset != 0: lanes ACTIVE
 * on entry take I0 from their entry state and D = 0; otherwise both are read.  Lanes
 * not ACTIVE on entry, and every lane when n_steps = 0, are left untouched. */
int oracle_integrate_monitored(const double *Ma, const int32_t *st_of_lane, int64_t n,
                               double *state, int32_t *status, int32_t *steps, double h,
                               int64_t n_steps, double horizon_factor, double r_escape,
                               int hamiltonian, int64_t every, int reset, double *monitor,
                               int nthreads)
{
    if (every < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (status[i] != ST_ACTIVE || n_steps == 0) continue;
        int st = st_of_lane ? st_of_lane[i] : 0;
        double M = Ma[2 * st], a = Ma[2 * st + 1];
        double y[8], I0[4], D[4], In[4];
        get_state(state, n, i, y);
        if (reset) {
            if (hamiltonian) oracle_invariants_hamiltonian_one(M, a, y, I0);
            else oracle_invariants_one(M, a, y, I0);
            for (int k = 0; k < 4; ++k) D[k] = 0.0;
        } else {
            for (int k = 0; k < 4; ++k) {
                I0[k] = monitor[k * n + i];
                D[k] = monitor[(4 + k) * n + i];
            }
        }
        for (int64_t k = 0; k < n_steps && status[i] == ST_ACTIVE; ++k) {
            integrate_lane(M, a, h, 1, horizon_factor, r_escape, hamiltonian, y, &status[i]);
            steps[i] += 1;
            if (steps[i] % every == 0) {
                if (hamiltonian) oracle_invariants_hamiltonian_one(M, a, y, In);
                else oracle_invariants_one(M, a, y, In);
                for (int c = 0; c < 4; ++c) D[c] = fmax(D[c], fabs(In[c] - I0[c]));
            }
        }
        put_state(state, n, i, y);
        for (int k = 0; k < 4; ++k) {
            monitor[k * n + i] = I0[k];
            monitor[(4 + k) * n + i] = D[k];
        }
    }
    return 0;
}

/* Invariants of a SoA batch: out[4n] = (E, L_z, Q, g(u,u)) component-major. */
int oracle_invariants(const double *Ma, const int32_t *st_of_lane, int64_t n, const double *state,
                      double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        int st = st_of_lane ? st_of_lane[i] : 0;
        double y[8], v[4];
        get_state(state, n, i, y);
        oracle_invariants_one(Ma[2 * st], Ma[2 * st + 1], y, v);
        for (int k = 0; k < 4; ++k) out[k * n + i] = v[k];
    }
    return 0;
}

/* ================================================================================ */
/* Adaptive integration: Dormand-Prince 5(4) with per-lane step-size control          */
/* ================================================================================ */
/* The paper integrates with the fixed-step classic RK4 and announces other members
 * of the Runge-Kutta family (Section 5).  This is the embedded pair of Dormand and
 * Prince (J. Comput. Appl. Math. 6 (1980) 19-26): seven stages, the last evaluated
 * at the new point (first same as last), a 5th-order solution y1 and a 4th-order
 * companion y1*.  Step-size control (Hairer, Norsett and Wanner, Solving Ordinary
 * Differential Equations I, Section II.4):
 *   sc_i = atol + rtol max(|y_i|, |y1_i|),  err = sqrt(mean_i ((y1_i - y1*_i) / sc_i)^2),
 *   accept iff err <= 1,  h_new = h min(facmax', max(facmin, fac err^(-1/5))),
 * with facmax' = 1 for the attempt right after a rejection, facmax otherwise.  The
 * last attempt of a call is shortened to land on tau_end.  Stop rules as for RK4
 * (R5-R8): a stage point at r <= r_stop ends the lane as HORIZON and a non-finite
 * or off-range result (or error) as NONFINITE, both keeping the start state;
 * after an accepted step r <= r_stop is HORIZON and r >= r_escape ESCAPE; a lane
 * that has used max_attempts attempts in the call without reaching tau_end ends
 * as BUDGET.  Rejected attempts count in `rejects`, accepted ones in `steps`. */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BS[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* One attempt of size h from y with k[0] = f(y): fills k[1..6], y1 (5th order),
 * e = y1 - y1* and the radii of the stage points 2..6. */
static void dp45_attempt(double M, double a, double h, const double y[8], double k[7][8],
                         double y1[8], double e[8], double stage_r[5])
{
    for (int s = 1; s < 7; ++s) {
        double Y[8];
        for (int c = 0; c < 8; ++c) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc += DP_A[s][j] * k[j][c];
            Y[c] = y[c] + h * acc;
        }
        if (s < 6) stage_r[s - 1] = Y[1];
        if (s == 6) memcpy(y1, Y, sizeof Y); /* the 7th row of A is the 5th-order weights */
        d_rhs(M, a, Y, k[s]);
    }
    for (int c = 0; c < 8; ++c) {
        double acc = 0.0;
        for (int j = 0; j < 7; ++j) acc += (DP_B[j] - DP_BS[j]) * k[j][c];
        e[c] = h * acc;
    }
}

/* One attempt from y (test hook): y1 (5th order) and e = y1 - y1* (4th order). */
void oracle_dp45_attempt(double M, double a, double h, const double *y, double *y1, double *e)
{
    double k[7][8], sr[5];
    d_rhs(M, a, y, k[0]);
    dp45_attempt(M, a, h, y, k, y1, e, sr);
}

typedef struct {
    double tau_end, rtol, atol, fac, facmin, facmax;
    int64_t max_attempts;
} dp_ctl;

static void adaptive_lane(double M, double a, const dp_ctl *ctl, double r_stop, double r_esc,
                          double y[8], double *tau, double *h, int32_t *status, int32_t *steps,
                          int32_t *rejects)
{
    double k[7][8];
    d_rhs(M, a, y, k[0]);
    double facmax = ctl->facmax;
    for (int64_t att = 0; *status == ST_ACTIVE && *tau < ctl->tau_end; ++att) {
        if (att == ctl->max_attempts) { *status = ST_BUDGET; break; }
        double hh = *h;
        int last = 0;
        if (*tau + hh >= ctl->tau_end) { hh = ctl->tau_end - *tau; last = 1; }
        double y1[8], e[8], sr[5];
        dp45_attempt(M, a, hh, y, k, y1, e, sr);
        int in_zone = 0;
        for (int j = 0; j < 5; ++j) in_zone |= sr[j] <= r_stop;
        if (in_zone) { *status = ST_HORIZON; break; }
        double sum = 0.0;
        for (int c = 0; c < 8; ++c) {
            double sc = ctl->atol + ctl->rtol * fmax(fabs(y[c]), fabs(y1[c]));
            sum += (e[c] / sc) * (e[c] / sc);
        }
        double err = sqrt(sum / 8.0);
        if (!usable(y1) || !isfinite(err)) { *status = ST_NONFINITE; break; }
        double grow = err > 0.0 ? ctl->fac * pow(err, -0.2) : ctl->facmax;
        if (err <= 1.0) {
            memcpy(y, y1, sizeof y1);
            memcpy(k[0], k[6], sizeof k[6]);
            *tau = last ? ctl->tau_end : *tau + hh;
            ++*steps;
            *h = hh * fmin(facmax, fmax(ctl->facmin, grow));
            facmax = ctl->facmax;
            if (y[1] <= r_stop) *status = ST_HORIZON;
            else if (y[1] >= r_esc) *status = ST_ESCAPE;
        } else {
            ++*rejects;
            *h = hh * fmin(1.0, fmax(ctl->facmin, grow));
            facmax = 1.0;
        }
    }
}

/* Batch driver (OpenMP over lanes): state, tau, h, status, steps, rejects in/out. */
int oracle_integrate_adaptive(const double *Ma, const int32_t *st_of_lane, int64_t n, double *state,
                              double *tau, double *h, int32_t *status, int32_t *steps,
                              int32_t *rejects, double tau_end, double rtol, double atol,
                              double fac, double facmin, double facmax, int64_t max_attempts,
                              double horizon_factor, double r_escape, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    dp_ctl ctl = {tau_end, rtol, atol, fac, facmin, facmax, max_attempts};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int st = st_of_lane ? st_of_lane[i] : 0;
        double M = Ma[2 * st], a = Ma[2 * st + 1];
        double y[8];
        get_state(state, n, i, y);
        adaptive_lane(M, a, &ctl, horizon_factor * oracle_r_horizon(M, a), r_escape, y, &tau[i],
                      &h[i], &status[i], &steps[i], &rejects[i]);
        put_state(state, n, i, y);
    }
    return 0;
}

/* ================================================================================ */
/* Numerical metrics in 3+1 form on an (r, theta) grid                                 */
/* ================================================================================ */
/* Section 2 writes the line element in 3+1 form, ds^2 = -alpha^2 dt^2 +
 * gamma_ij (dx^i + beta^i dt)(dx^j + beta^j dt) (eq. ADM), gives alpha, beta^i and
 * gamma_ij of Kerr, and names the 3+1 form as the way to numerical metrics.  A
 * stationary, axisymmetric metric with beta = (0, 0, beta^phi) and diagonal gamma is
 * given here by five functions of (r, theta) sampled on a uniform grid:
 *   F = (alpha, beta^phi, gamma_rr, gamma_thth, gamma_phph / sin^2 theta),
 * node (i, j) at r_i = r0 + i dr, theta_j = th0 + j dth, stored at
 * nodes[(i nth + j) 5 + k].  Between nodes each function is the tensor product of
 * the 4-point Lagrange interpolants in r and theta (nodes i-1 .. i+2 around the cell
 * holding the point, the stencil shifted inwards at the grid's edges); its
 * derivatives are those of the interpolant.  The inverse metric follows from the
 * 3+1 quantities: g^tt = -1/alpha^2, g^tphi = beta^phi/alpha^2,
 * g^phph = 1/gamma_phph - (beta^phi)^2/alpha^2, g^rr = 1/gamma_rr,
 * g^thth = 1/gamma_thth, and the canonical equations (eq. Ham) are integrated with
 * classic RK4 in (x^mu, p_mu). */

/* Kerr in 3+1 form (Section 2): alpha = sqrt(rho^2 Delta / Sigma),
 * beta^phi = -2 M a r / Sigma, gamma = diag(rho^2/Delta, rho^2, Sigma sin^2 / rho^2). */
void oracle_kerr_3p1(double M, double a, double r, double th, double *F)
{
    double s = sin(th), c = cos(th);
    double rho2 = r * r + a * a * c * c;
    double Delta = r * r - 2.0 * M * r + a * a;
    double Sigma = (r * r + a * a) * (r * r + a * a) - a * a * Delta * s * s;
    F[0] = sqrt(rho2 * Delta / Sigma);
    F[1] = -2.0 * M * a * r / Sigma;
    F[2] = rho2 / Delta;
    F[3] = rho2;
    F[4] = Sigma / rho2;
}

void oracle_grid_fill_kerr(double M, double a, int64_t nr, int64_t nth, double r0, double dr,
                           double th0, double dth, double *nodes)
{
    for (int64_t i = 0; i < nr; ++i)
        for (int64_t j = 0; j < nth; ++j)
            oracle_kerr_3p1(M, a, r0 + (double)i * dr, th0 + (double)j * dth, &nodes[(i * nth + j) * 5]);
}

/* Lagrange basis on the nodes -1, 0, 1, 2 at u, and its derivative in u. */
static void lagrange4(double u, double w[4], double dw[4])
{
    const double x[4] = {-1.0, 0.0, 1.0, 2.0};
    for (int k = 0; k < 4; ++k) {
        double num = 1.0, den = 1.0, d = 0.0;
        for (int m = 0; m < 4; ++m) {
            if (m == k) continue;
            den *= x[k] - x[m];
            /* derivative of the product: sum over the factor left out */
            double prod = 1.0;
            for (int q = 0; q < 4; ++q)
                if (q != k && q != m) prod *= u - x[q];
            d += prod;
            num *= u - x[m];
        }
        w[k] = num / den;
        dw[k] = d / den;
    }
}

/* Cell and offset of coordinate x on a grid of n nodes x0 + i h: the stencil starts
 * at node i - 1 with i = floor((x - x0) / h) clamped to [1, n - 3]. */
static int64_t grid_cell(double x, double x0, double h, int64_t n, double *u)
{
    double q = (x - x0) / h;
    int64_t i = (int64_t)floor(q);
    if (i < 1) i = 1;
    if (i > n - 3) i = n - 3;
    *u = q - (double)i;
    return i;
}

/* F, dF/dr, dF/dtheta (5 functions each) at (r, theta). */
void oracle_grid_eval(int64_t nr, int64_t nth, double r0, double dr, double th0, double dth,
                      const double *nodes, double r, double th, double *F, double *Fr, double *Ft)
{
    double ur, ut, wr[4], dwr[4], wt[4], dwt[4];
    int64_t i = grid_cell(r, r0, dr, nr, &ur);
    int64_t j = grid_cell(th, th0, dth, nth, &ut);
    lagrange4(ur, wr, dwr);
    lagrange4(ut, wt, dwt);
    for (int k = 0; k < 5; ++k) {
        double v = 0.0, vr = 0.0, vt = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double f = nodes[((i - 1 + a) * nth + (j - 1 + b)) * 5 + k];
                v += wr[a] * wt[b] * f;
                vr += dwr[a] * wt[b] * f;
                vt += wr[a] * dwt[b] * f;
            }
        F[k] = v;
        Fr[k] = vr / dr;
        Ft[k] = vt / dth;
    }
}

typedef struct {
    int64_t nr, nth;
    double r0, dr, th0, dth;
    const double *nodes;
} grid_t;

/* Inverse metric g^{mu nu} (4x4) and its r and theta derivatives from the gridded
 * 3+1 functions at (r, theta). */
static void grid_inverse_metric(const grid_t *g, double r, double th, double gi[4][4],
                                double dgi[2][4][4])
{
    double F[5], Fd[2][5];
    oracle_grid_eval(g->nr, g->nth, g->r0, g->dr, g->th0, g->dth, g->nodes, r, th, F, Fd[0], Fd[1]);
    double s = sin(th), c = cos(th);
    double al = F[0], be = F[1], grr = F[2], gtt = F[3], gpp = F[4] * s * s;
    double d_al[2] = {Fd[0][0], Fd[1][0]}, d_be[2] = {Fd[0][1], Fd[1][1]};
    double d_grr[2] = {Fd[0][2], Fd[1][2]}, d_gtt[2] = {Fd[0][3], Fd[1][3]};
    double d_gpp[2] = {Fd[0][4] * s * s, Fd[1][4] * s * s + F[4] * 2.0 * s * c};
    memset(gi, 0, 16 * sizeof(double));
    memset(dgi, 0, 32 * sizeof(double));
    double ia2 = 1.0 / (al * al);
    gi[0][0] = -ia2;
    gi[0][3] = gi[3][0] = be * ia2;
    gi[3][3] = 1.0 / gpp - be * be * ia2;
    gi[1][1] = 1.0 / grr;
    gi[2][2] = 1.0 / gtt;
    for (int l = 0; l < 2; ++l) {
        double d_ia2 = -2.0 * d_al[l] / (al * al * al);
        dgi[l][0][0] = -d_ia2;
        dgi[l][0][3] = dgi[l][3][0] = d_be[l] * ia2 + be * d_ia2;
        dgi[l][3][3] = -d_gpp[l] / (gpp * gpp) - 2.0 * be * d_be[l] * ia2 - be * be * d_ia2;
        dgi[l][1][1] = -d_grr[l] / (grr * grr);
        dgi[l][2][2] = -d_gtt[l] / (gtt * gtt);
    }
}

/* Canonical right-hand side (eq. Ham) with the gridded metric:
 * dx^mu = g^{mu nu} p_nu, dp_mu = -1/2 (d_mu g^{ab}) p_a p_b (mu = r, theta; the
 * metric does not depend on t or phi). */
static void grid_rhs(const grid_t *g, const double z[8], double f[8])
{
    double gi[4][4], dgi[2][4][4];
    grid_inverse_metric(g, z[1], z[2], gi, dgi);
    for (int mu = 0; mu < 4; ++mu) {
        double acc = 0.0;
        for (int nu = 0; nu < 4; ++nu) acc += gi[mu][nu] * z[4 + nu];
        f[mu] = acc;
    }
    f[4] = 0.0;
    f[7] = 0.0;
    for (int l = 0; l < 2; ++l) {
        double acc = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) acc += dgi[l][a][b] * z[4 + a] * z[4 + b];
        f[5 + l] = -0.5 * acc;
    }
}

void oracle_grid_rhs(int64_t nr, int64_t nth, double r0, double dr, double th0, double dth,
                     const double *nodes, const double *z, double *f)
{
    grid_t g = {nr, nth, r0, dr, th0, dth, nodes};
    grid_rhs(&g, z, f);
}

/* Fixed-step RK4 on the gridded metric with the stop rules of the analytic path:
 * stage radius <= r_stop -> HORIZON (start state kept); result non-finite, theta
 * outside (0, pi), or a stage point or the result outside the grid's interior
 * [r0 + dr, r0 + (nr - 2) dr] x [th0 + dth, th0 + (nth - 2) dth] -> NONFINITE (start
 * state kept); then r <= r_stop -> HORIZON, r >= r_escape -> ESCAPE. */
int oracle_integrate_grid(int64_t nr, int64_t nth, double r0, double dr, double th0, double dth,
                          const double *nodes, int64_t n, double *state, int32_t *status,
                          int32_t *steps, double h, int64_t n_steps, double r_stop,
                          double r_escape, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    grid_t g = {nr, nth, r0, dr, th0, dth, nodes};
    const double rlo = r0 + dr, rhi = r0 + (double)(nr - 2) * dr;
    const double tlo = th0 + dth, thi = th0 + (double)(nth - 2) * dth;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double y[8];
        get_state(state, n, i, y);
        int64_t k;
        for (k = 0; k < n_steps && status[i] == ST_ACTIVE; ++k) {
            /* RK4 written out with the inside-the-grid check on every stage point */
            double k1[8], k2[8], k3[8], k4[8], Y[8], y1[8];
            int outside = 0, zone = 0;
            grid_rhs(&g, y, k1);
            for (int c = 0; c < 8; ++c) Y[c] = y[c] + 0.5 * h * k1[c];
            zone |= Y[1] <= r_stop;
            outside |= !(Y[1] >= rlo && Y[1] <= rhi && Y[2] >= tlo && Y[2] <= thi);
            if (!zone && !outside) grid_rhs(&g, Y, k2);
            for (int c = 0; c < 8 && !zone && !outside; ++c) Y[c] = y[c] + 0.5 * h * k2[c];
            if (!zone && !outside) {
                zone |= Y[1] <= r_stop;
                outside |= !(Y[1] >= rlo && Y[1] <= rhi && Y[2] >= tlo && Y[2] <= thi);
            }
            if (!zone && !outside) grid_rhs(&g, Y, k3);
            for (int c = 0; c < 8 && !zone && !outside; ++c) Y[c] = y[c] + h * k3[c];
            if (!zone && !outside) {
                zone |= Y[1] <= r_stop;
                outside |= !(Y[1] >= rlo && Y[1] <= rhi && Y[2] >= tlo && Y[2] <= thi);
            }
            if (zone) { status[i] = ST_HORIZON; continue; }
            if (outside) { status[i] = ST_NONFINITE; continue; }
            grid_rhs(&g, Y, k4);
            for (int c = 0; c < 8; ++c)
                y1[c] = y[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
            if (!usable(y1) || !(y1[1] >= rlo && y1[1] <= rhi && y1[2] >= tlo && y1[2] <= thi)) {
                status[i] = ST_NONFINITE;
                continue;
            }
            memcpy(y, y1, sizeof y1);
            if (y[1] <= r_stop) status[i] = ST_HORIZON;
            else if (y[1] >= r_escape) status[i] = ST_ESCAPE;
        }
        steps[i] += (int32_t)k;
        put_state(state, n, i, y);
    }
    return 0;
}

/* ================================================================================ */
/* Camera: backward-traced null geodesics with a thin equatorial disk                */
/* ================================================================================ */
/* Image plane (Bardeen 1973) of a static observer at (r_obs, theta_obs = incl,
 * phi = 0).  Pixel (i, j), j the row: alpha = -w + (i + 1/2) 2w/nx,
 * beta = -w + (j + 1/2) 2w/ny.  Photon constants: E = 1, L_z = -alpha sin(incl),
 * Q = beta^2 + cos^2(incl) (alpha^2 - a^2).  The photon arriving at the observer
 * has u^r > 0 and sign(u^theta) = sign(beta); it is traced backward by negating
 * its 4-velocity and stepping forward in the affine parameter. */
void oracle_ray_ic(double M, double a, double r_obs, double incl, double alpha, double beta, double *y);

void oracle_camera_ic(double M, double a, double r_obs, double incl, double half_width, int64_t nx,
                      int64_t ny, int64_t i, int64_t j, double *y)
{
    double w = half_width;
    double alpha = -w + ((double)i + 0.5) * 2.0 * w / (double)nx;
    double beta = -w + ((double)j + 0.5) * 2.0 * w / (double)ny;
    oracle_ray_ic(M, a, r_obs, incl, alpha, beta, y);
}

/* Photon state for image-plane coordinates (alpha, beta), see above. */
void oracle_ray_ic(double M, double a, double r_obs, double incl, double alpha, double beta, double *y)
{
    double si = sin(incl), ci = cos(incl);
    double E = 1.0, Lz = -alpha * si, Q = beta * beta + ci * ci * (alpha * alpha - a * a);
    y[0] = 0.0; y[1] = r_obs; y[2] = incl; y[3] = 0.0;
    oracle_velocity_from_constants(M, a, E, Lz, Q, 0.0, r_obs, incl, 1.0, beta >= 0 ? 1.0 : -1.0, y + 4);
    for (int k = 4; k < 8; ++k) y[k] = -y[k];
}

/* Trace one backward ray.  Step size h = h0 max(1, r_n / h_r0) from the state
 * at the start of the step.  Termination as for integrate_lane, with the disk
 * test (rule 3): the equatorial plane is crossed when signbit(cos theta)
 * differs between y_n and y_{n+1}; the crossing radius is the linear
 * interpolation r_c = r_n + (r_{n+1} - r_n) c_n / (c_n - c_{n+1}) (phi_c
 * likewise) and the ray hits the disk iff disk_r_in <= r_c <= disk_r_out.
 * A ray still active after max_steps steps gets BUDGET.  hit = (r_c, phi_c)
 * for DISK, NaN otherwise.  Returns the number of steps evaluated. */
static int64_t trace_ray(double M, double a, double h0, double h_r0, double r_escape, double rh,
                         double disk_r_in, double disk_r_out, int64_t max_steps, double y[8],
                         int32_t *status, double hit[2])
{
    int32_t st = ST_ACTIVE;
    int64_t n = 0;
    double rc = NAN, pc = NAN;
    while (st == ST_ACTIVE) {
        if (n >= max_steps) { st = ST_BUDGET; break; }
        double h = h0 * fmax(1.0, y[1] / h_r0);
        double y1[8], sr[3];
        d_rk4_step_stages(M, a, h, y, y1, sr);
        ++n;
        if (stage_in_zone(sr, rh)) { st = ST_HORIZON; break; }
        if (!usable(y1)) { st = ST_NONFINITE; break; }
        double c0 = cos(y[2]), c1 = cos(y1[2]);
        if (signbit(c0) != signbit(c1)) {
            double f = c0 / (c0 - c1);
            double rcr = y[1] + (y1[1] - y[1]) * f;
            if (rcr >= disk_r_in && rcr <= disk_r_out) {
                rc = rcr;
                pc = y[3] + (y1[3] - y[3]) * f;
                st = ST_DISK;
            }
        }
        memcpy(y, y1, sizeof y1);
        if (st == ST_ACTIVE) {
            if (y[1] <= rh) st = ST_HORIZON;
            else if (y[1] >= r_escape) st = ST_ESCAPE;
        }
    }
    *status = st;
    hit[0] = rc;
    hit[1] = pc;
    return n;
}

/* Trace a list of pixels p (row-major: i = p % nx, j = p / nx). */
int oracle_trace_camera(double M, double a, double r_obs, double incl, double half_width, int64_t nx,
                        int64_t ny, double h0, double h_r0, double r_escape, double horizon_factor,
                        double disk_r_in, double disk_r_out, int64_t max_steps, int64_t npix,
                        const int64_t *pix, int32_t *status, int32_t *steps, double *hit,
                        double *final_state /* 8*npix SoA, nullable */, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double rh = horizon_factor * oracle_r_horizon(M, a);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix[q];
        double y[8];
        oracle_camera_ic(M, a, r_obs, incl, half_width, nx, ny, p % nx, p / nx, y);
        steps[q] = (int32_t)trace_ray(M, a, h0, h_r0, r_escape, rh, disk_r_in, disk_r_out, max_steps,
                                      y, &status[q], hit + 2 * q);
        if (final_state) put_state(final_state, npix, q, y);
    }
    return 0;
}

/* Trace rays given directly by image-plane coordinates (alpha[q], beta[q]). */
int oracle_trace_rays(double M, double a, double r_obs, double incl, int64_t nray, const double *alpha,
                      const double *beta, double h0, double h_r0, double r_escape,
                      double horizon_factor, double disk_r_in, double disk_r_out, int64_t max_steps,
                      int32_t *status, int32_t *steps, double *hit,
                      double *final_state /* 8*nray SoA, nullable */, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double rh = horizon_factor * oracle_r_horizon(M, a);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nray; ++q) {
        double y[8];
        oracle_ray_ic(M, a, r_obs, incl, alpha[q], beta[q], y);
        steps[q] = (int32_t)trace_ray(M, a, h0, h_r0, r_escape, rh, disk_r_in, disk_r_out, max_steps,
                                      y, &status[q], hit + 2 * q);
        if (final_state) put_state(final_state, nray, q, y);
    }
    return 0;
}

/* ================================================================================ */
/* Complex-step tangents of the discrete RK4 map (gradient checks)                   */
/* ================================================================================ */
/* dy_N = d y_N / d y_0 . v for n_steps fixed-size steps (no termination):
 * integrate y_0 + i eps v in complex arithmetic and read Im / eps
 * (Squire & Trapp 1998).  y_out (nullable) receives the real trajectory end. */
void oracle_tangent(double M, double a, double h, int64_t n_steps, const double *y0, const double *v,
                    double *y_out, double *dy_out)
{
    const double eps = 1e-30;
    double complex z[8], z1[8];
    for (int k = 0; k < 8; ++k) z[k] = y0[k] + I * eps * v[k];
    for (int64_t n = 0; n < n_steps; ++n) {
        z_rk4_step(M, a, h, z, z1);
        memcpy(z, z1, sizeof z1);
    }
    for (int k = 0; k < 8; ++k) {
        if (y_out) y_out[k] = creal(z[k]);
        dy_out[k] = cimag(z[k]) / eps;
    }
}

/* Initial-condition map with E held fixed:
 * p = (r0, theta0, u^r0, u^theta0, L_z) -> y0 = (0, r0, theta0, 0, u^t, u^r0, u^theta0, u^phi)
 * with (u^t, u^phi) = G^{-1} (-E, L_z), G the (t, phi) block of g at (r0, theta0). */
static void z_ic_map(double M, double a, double E, const double complex p[5], double complex y[8])
{
    double complex g[4][4];
    z_metric(M, a, p[0], p[1], g);
    double complex det = g[0][0] * g[3][3] - g[0][3] * g[3][0];
    double complex gtt = g[3][3] / det, gtp = -g[0][3] / det, gpp = g[0][0] / det;
    y[0] = 0.0; y[1] = p[0]; y[2] = p[1]; y[3] = 0.0;
    y[4] = gtt * (-E) + gtp * p[4];
    y[5] = p[2];
    y[6] = p[3];
    y[7] = gtp * (-E) + gpp * p[4];
}

void oracle_ic_map(double M, double a, double E, const double *p, double *y)
{
    double complex pz[5], yz[8];
    for (int k = 0; k < 5; ++k) pz[k] = p[k];
    z_ic_map(M, a, E, pz, yz);
    for (int k = 0; k < 8; ++k) y[k] = creal(yz[k]);
}

/* Gradient of loss = sum_{k in r,theta,phi} (y_N[k] - target[k])^2 with respect
 * to p = (r0, theta0, u^r0, u^theta0, L_z), E fixed, by 5 complex-step passes
 * through the IC map and n_steps RK4 steps.  Batch over lanes (p and target SoA
 * 5n / 3n), OpenMP.  loss_out (nullable) per lane. */
int oracle_grad_ic(double M, double a, double h, int64_t n_steps, int64_t n, const double *p_soa,
                   const double *E, const double *target_soa, double *grad_soa, double *loss_out,
                   int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const double eps = 1e-30;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < 5; ++j) {
            double complex p[5], z[8], z1[8];
            for (int k = 0; k < 5; ++k) p[k] = p_soa[k * n + i] + (k == j ? I * eps : 0.0);
            z_ic_map(M, a, E[i], p, z);
            for (int64_t s = 0; s < n_steps; ++s) {
                z_rk4_step(M, a, h, z, z1);
                memcpy(z, z1, sizeof z1);
            }
            double g = 0.0, L = 0.0;
            for (int c = 0; c < 3; ++c) {
                double d = creal(z[1 + c]) - target_soa[c * n + i];
                L += d * d;
                g += 2.0 * d * cimag(z[1 + c]) / eps;
            }
            grad_soa[j * n + i] = g;
            if (j == 0 && loss_out) loss_out[i] = L;
        }
    }
    return 0;
}

/* Loss of one lane (for central finite differences in the tests). */
double oracle_loss_ic(double M, double a, double h, int64_t n_steps, const double *p, double E,
                      const double *target)
{
    double y[8], y1[8];
    oracle_ic_map(M, a, E, p, y);
    for (int64_t s = 0; s < n_steps; ++s) {
        d_rk4_step(M, a, h, y, y1);
        memcpy(y, y1, sizeof y1);
    }
    double L = 0.0;
    for (int c = 0; c < 3; ++c) L += (y[1 + c] - target[c]) * (y[1 + c] - target[c]);
    return L;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
