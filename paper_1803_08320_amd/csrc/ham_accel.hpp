// Canonical (Hamiltonian) form of the geodesic equations for the Kerr metric, shared
// by the FP64 kernel and the host flop counter.
//
// Quiroga, MALBEC, Section 2, eq. Ham: with z = (x^mu, p_mu) and
// H = (1/2) g^{mu nu} p_mu p_nu, dx^mu/dtau = dH/dp_mu and dp_mu/dtau = -dH/dx^mu.
// The metric of eq. kerr does not depend on t or phi, so p_t and p_phi are constants
// of the motion (Sections 3-4 use exactly this); only (r, theta, p_r, p_theta)
// change at the RK4 stage points, and t, phi are accumulated.
//
// H is evaluated in its separated (Carter) form,
//   2 H rho^2 = N = Delta p_r^2 + p_theta^2 + w^2 - P^2 / Delta,
//   w = p_phi / s + a s p_t,  P = (r^2 + a^2) p_t + a p_phi,
// which is g^{mu nu} p_mu p_nu of eq. kerr multiplied out (s = sin theta,
// c = cos theta).  Its derivatives are taken by hand:
//   dt/dtau   = (a s w - (r^2 + a^2) P / Delta) / rho^2
//   dr/dtau   = Delta p_r / rho^2,     dtheta/dtau = p_theta / rho^2
//   dphi/dtau = (w / s - a P / Delta) / rho^2
//   dp_r/dtau = (r N / rho^2 - (1/2) d_r N) / rho^2,
//       (1/2) d_r N = (r - M) p_r^2 - (P / Delta) (2 r p_t - (P / Delta)(r - M))
//   dp_theta/dtau = -(a^2 s c N / rho^2 + (1/2) d_theta N) / rho^2,
//       (1/2) d_theta N = w c (a p_t - p_phi / s^2)
// One reciprocal 1 / (rho^2 Delta s) gives 1/rho^2, 1/Delta and 1/s.
#pragma once

#include "kerr_accel.hpp"

namespace malbec {

// Per-lane constants of the motion: p_t, p_phi and their products with a.
template <typename T>
struct HamConst {
    T pt, pph, apt, apph;
};

template <typename T>
MALBEC_HD inline HamConst<T> ham_const(T a, T pt, T pph)
{
    return HamConst<T>{pt, pph, a * pt, a * pph};
}

// dz/dtau for (r, theta, p_r, p_theta) at s = sin theta, c = cos theta: the
// derivatives of (t, r, theta, phi, p_r, p_theta) (those of p_t, p_phi vanish).
template <typename T>
MALBEC_HD inline void kerr_ham(T M, T a, T r, T s, T c, T pr, T pth, const HamConst<T> &P, T &dt,
                               T &dr, T &dth, T &dph, T &dpr, T &dpth)
{
    const T a2 = a * a;
    const T r2 = r * r;
    const T A = r2 + a2;                     // r^2 + a^2
    const T rho2 = fma(a2, c * c, r2);       // r^2 + a^2 cos^2
    const T Delta = fma(-(M + M), r, A);     // r^2 - 2 M r + a^2
    const T rD = rho2 * Delta;
    const T inv = recip(rD * s);             // 1 / (rho^2 Delta s)
    const T irho2 = inv * (Delta * s);
    const T iDelta = inv * (rho2 * s);
    const T is = inv * rD;                   // 1 / s
    const T Pr = fma(A, P.pt, P.apph);       // P
    const T PD = Pr * iDelta;                // P / Delta
    const T w = fma(P.pph, is, P.apt * s);
    const T prpr = pr * pr;
    const T N = fma(-Pr, PD, fma(w, w, fma(Delta, prpr, pth * pth)));
    const T twoH = N * irho2;                // g^{mu nu} p_mu p_nu
    dr = (Delta * irho2) * pr;
    dth = pth * irho2;
    dt = fma(a * s, w, -A * PD) * irho2;
    dph = fma(w, is, -a * PD) * irho2;
    const T rM = r - M;
    // 2 r p_t as r (2 p_t): the same exact doubling, with 2 p_t constant along the lane
    const T hdrN = fma(rM, prpr, -PD * fma(-PD, rM, r * (P.pt + P.pt)));
    dpr = fma(r, twoH, -hdrN) * irho2;
    const T hdthN = (w * c) * fma(-P.pph, is * is, P.apt);
    dpth = -fma(a2 * (s * c), twoH, hdthN) * irho2;
}

// Stages of one classic RK4 step (b = 1/6, 1/3, 1/3, 1/6; c = 0, 1/2, 1/2, 1) of the
// canonical state z = (t, r, theta, phi, p_t, p_r, p_theta, p_phi).
// f(stage, r, theta, p_r, p_theta, dt, dr, dth, dph, dpr, dpth) evaluates the
// right-hand side at stage point `stage`; acc[] receives the weighted sums
// k1 + 2 k2 + 2 k3 + k4 of (t, r, theta, phi, p_r, p_theta) and sr[] the radii of the
// three intermediate stage points.  p_t and p_phi do not change.
template <typename T, typename F>
MALBEC_HD inline void rk4_ham_stages(F &f, T h, const T z[8], T acc[6], T sr[3])
{
    const T hh = T(0.5) * h;
    T dt, dr, dth, dph, dpr, dpth;
    T s1, s2, s3, s4;  // stage point (r, theta, p_r, p_theta)

    f(0, z[1], z[2], z[5], z[6], dt, dr, dth, dph, dpr, dpth);
    acc[0] = dt; acc[1] = dr; acc[2] = dth; acc[3] = dph; acc[4] = dpr; acc[5] = dpth;
    s1 = fma(hh, dr, z[1]); s2 = fma(hh, dth, z[2]); s3 = fma(hh, dpr, z[5]); s4 = fma(hh, dpth, z[6]);
    sr[0] = s1;

    f(1, s1, s2, s3, s4, dt, dr, dth, dph, dpr, dpth);
    acc[0] = fma(T(2), dt, acc[0]); acc[1] = fma(T(2), dr, acc[1]); acc[2] = fma(T(2), dth, acc[2]);
    acc[3] = fma(T(2), dph, acc[3]); acc[4] = fma(T(2), dpr, acc[4]); acc[5] = fma(T(2), dpth, acc[5]);
    s1 = fma(hh, dr, z[1]); s2 = fma(hh, dth, z[2]); s3 = fma(hh, dpr, z[5]); s4 = fma(hh, dpth, z[6]);
    sr[1] = s1;

    f(2, s1, s2, s3, s4, dt, dr, dth, dph, dpr, dpth);
    acc[0] = fma(T(2), dt, acc[0]); acc[1] = fma(T(2), dr, acc[1]); acc[2] = fma(T(2), dth, acc[2]);
    acc[3] = fma(T(2), dph, acc[3]); acc[4] = fma(T(2), dpr, acc[4]); acc[5] = fma(T(2), dpth, acc[5]);
    s1 = fma(h, dr, z[1]); s2 = fma(h, dth, z[2]); s3 = fma(h, dpr, z[5]); s4 = fma(h, dpth, z[6]);
    sr[2] = s1;

    f(3, s1, s2, s3, s4, dt, dr, dth, dph, dpr, dpth);
    acc[0] += dt; acc[1] += dr; acc[2] += dth; acc[3] += dph; acc[4] += dpr; acc[5] += dpth;
}

// One RK4 step: z1 = z + h/6 (k1 + 2 k2 + 2 k3 + k4), p_t and p_phi copied.
template <typename T, typename F>
MALBEC_HD inline void rk4_ham_step(F &f, T h, const T z[8], T z1[8], T sr[3])
{
    T acc[6];
    rk4_ham_stages(f, h, z, acc, sr);
    const T h6 = h * T(1.0 / 6.0);
    z1[0] = fma(h6, acc[0], z[0]);
    z1[1] = fma(h6, acc[1], z[1]);
    z1[2] = fma(h6, acc[2], z[2]);
    z1[3] = fma(h6, acc[3], z[3]);
    z1[4] = z[4];
    z1[5] = fma(h6, acc[4], z[5]);
    z1[6] = fma(h6, acc[5], z[6]);
    z1[7] = z[7];
}

// The increment d = z1 - z alone (compensated updates); d[4] = d[7] = 0.
template <typename T, typename F>
MALBEC_HD inline void rk4_ham_delta(F &f, T h, const T z[8], T d[8], T sr[3])
{
    T acc[6];
    rk4_ham_stages(f, h, z, acc, sr);
    const T h6 = h * T(1.0 / 6.0);
    d[0] = h6 * acc[0];
    d[1] = h6 * acc[1];
    d[2] = h6 * acc[2];
    d[3] = h6 * acc[3];
    d[4] = T(0);
    d[5] = h6 * acc[4];
    d[6] = h6 * acc[5];
    d[7] = T(0);
}

}  // namespace malbec
