// Geodesic acceleration of the Kerr metric, shared by the FP64 and FP32 kernels.
//
// Kerr metric in Boyer-Lindquist coordinates (Quiroga, MALBEC, Section 2,
// eq. kerr).  The geodesic acceleration du^mu/dtau = -Gamma^mu_ab u^a u^b is
// not formed from the 40 Christoffel symbols.  It uses the identity
//     g_{mu nu} du^nu/dtau = 1/2 (d_mu g_ab) u^a u^b - (d_l g_{mu b}) u^l u^b,
// which is the Christoffel contraction with the metric lowered, and then raises
// the index with the block-diagonal inverse metric ((t, phi) 2x2 block,
// g^rr = Delta / rho^2, g^thth = 1 / rho^2).  Only r and theta partials of the 5
// nonzero metric components enter.  Everything stays in registers.
//
// With q = 2 M r / rho^2:
//   g_tt = q - 1,  g_tphi = -a q s^2,  g_phiphi = (r^2 + a^2 + a^2 q s^2) s^2,
//   g_rr = rho^2 / Delta,  g_thth = rho^2,
// and det of the (t, phi) block = -Delta s^2.  One reciprocal 1 / (rho^2 Delta s^2)
// yields 1/rho^2, 1/Delta and 1/(Delta s^2).
#pragma once

#if defined(__HIPCC__)
#define MALBEC_HD __host__ __device__
#else
#define MALBEC_HD
#include <cmath>
using std::fma;
#endif

namespace malbec {

// Reciprocal used by the acceleration.  On the device: FP64 from the hardware
// estimate r (relative error below 6e-8) refined by one third-order step,
// r (1 + e + e^2) with e = 1 - x r, which leaves a relative error of order e^3 < 3e-22
// before the final rounding (within 0.5 ulp, as two Newton steps, one FMA fewer);
// FP32 the hardware reciprocal (1 ulp).
MALBEC_HD inline double recip(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
#else
    return 1.0 / x;
#endif
}
MALBEC_HD inline float recip(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Position-dependent coefficients of the acceleration at (r, theta), with
// s = sin theta, c = cos theta.  The contraction below works with half the metric
// partials (dg** hold (1/2) d g_**), so that its lowered acceleration needs no
// factor 1/2; the raising coefficients of the (t, phi) block carry the matching
// factor 2: Rtt = 2 g_pp / (Delta s^2), Rtp = 2 g_tp / (Delta s^2),
// Rpp = 2 g_tt / (Delta s^2), the inverse block being
// -(1/2) [[Rtt, -Rtp], [-Rtp, Rpp]].  Also 1/rho^2, Delta/rho^2, and
// c1 = a^2 s c / Delta = -(1/2) d_theta g_rr.
template <typename T>
struct KerrCoef {
    T r, Rtt, Rtp, Rpp, irho2, Dirho2, a2sc;
    T dgtt_r, dgtt_th, dgtp_r, dgtp_th, dgpp_r, dgpp_th, dgrr_r, c1;
};

template <typename T>
MALBEC_HD inline void kerr_coef(T M, T a, T r, T s, T c, KerrCoef<T> &K)
{
    const T a2 = a * a;
    const T s2 = s * s;
    const T sc = s * c;
    const T r2 = r * r;
    const T A = r2 + a2;                    // r^2 + a^2
    const T rho2 = fma(a2, c * c, r2);      // r^2 + a^2 cos^2
    const T M2 = M + M;
    const T Delta = fma(-M2, r, A);         // r^2 - 2 M r + a^2
    const T Ds2 = Delta * s2;
    const T inv = recip(rho2 * Ds2);        // 1 / (rho^2 Delta s^2)
    const T iDs2 = inv * rho2;              // 1 / (Delta s^2)
    const T irho2 = inv * Ds2;              // 1 / rho^2
    const T iDelta = iDs2 * s2;             // 1 / Delta
    const T mi = M * irho2;
    const T ri = r * irho2;                 // r / rho^2
    const T q = M2 * ri;                    // 2 M r / rho^2;  g_tt = q - 1
    const T qs2 = q * s2;                   // g_tp = -a q s^2
    const T gpp_os2 = fma(a2, qs2, A);      // g_pp = (r^2 + a^2 + a^2 q s^2) s^2

    // half partial derivatives of q and of q s^2:
    // (1/2) d_r q = M (rho^2 - 2 r^2) / rho^4 = mi - q r / rho^2
    const T hdq_r = fma(-q, ri, mi);
    const T a2sc = a2 * sc;
    const T hdq_th = (q * irho2) * a2sc;
    const T hdqs2_th = fma(hdq_th, s2, q * sc);
    const T grr = rho2 * iDelta;
    const T iDelta2 = iDelta + iDelta;

    K.r = r;
    K.Rtt = iDelta2 * gpp_os2;
    K.Rtp = (-a * q) * iDelta2;
    K.Rpp = iDs2 * fma(T(2), q, T(-2));
    K.irho2 = irho2;
    K.Dirho2 = Delta * irho2;
    K.a2sc = a2sc;
    K.dgtt_r = hdq_r;
    K.dgtt_th = hdq_th;
    K.dgtp_r = (-a * s2) * hdq_r;
    K.dgtp_th = -a * hdqs2_th;
    K.dgpp_r = fma(-a, K.dgtp_r, r) * s2;                 // (r + a^2 s^2 hdq_r) s^2
    K.dgpp_th = fma(-a * K.dgtp_th, s2, gpp_os2 * sc);    // a^2 hd(q s^2) s^2 + g_pp/s^2 sc
    K.dgrr_r = iDelta * fma(-grr, r - M, r);              // (r - g_rr (r - M)) / Delta
    K.c1 = a2sc * iDelta;
}

// Intermediate products of the contraction (kept for the adjoint).
template <typename T>
struct KerrContr {
    T Pt_r, Pt_th, Pp_r, Pp_th, Wt, Wp, Fr, Fth;
};

// du^mu/dtau from the coefficients and the 4-velocity (ut, ur, uth, uph).
template <typename T>
MALBEC_HD inline void kerr_contract(const KerrCoef<T> &K, T ut, T ur, T uth, T uph, T &at, T &ar,
                                    T &ath, T &aph, KerrContr<T> *keep = nullptr)
{
    // (1/2) (d_l g_{t b}) u^b and (1/2) (d_l g_{phi b}) u^b for l = r, theta
    const T Pt_r = fma(K.dgtt_r, ut, K.dgtp_r * uph);
    const T Pt_th = fma(K.dgtt_th, ut, K.dgtp_th * uph);
    const T Pp_r = fma(K.dgtp_r, ut, K.dgpp_r * uph);
    const T Pp_th = fma(K.dgtp_th, ut, K.dgpp_th * uph);

    // lowered acceleration F_mu = g_{mu nu} du^nu/dtau: F_t = -2 Wt, F_phi = -2 Wp
    const T Wt = fma(ur, Pt_r, uth * Pt_th);
    const T Wp = fma(ur, Pp_r, uth * Pp_th);
    const T Qr = fma(ut, Pt_r, uph * Pp_r);    // (1/2) (t,phi) part of (d_r g_ab) u^a u^b
    const T Qth = fma(ut, Pt_th, uph * Pp_th); // (1/2) (t,phi) part of (d_th g_ab) u^a u^b
    const T urur = ur * ur, uthuth = uth * uth, uruth2 = (ur + ur) * uth;  // 2 ur uth
    // F_r = Qr - (1/2) d_r g_rr ur^2 + r uth^2 - d_th g_rr ur uth
    const T Fr = fma(K.c1, uruth2, fma(K.r, uthuth, fma(-K.dgrr_r, urur, Qr)));
    // F_th = Qth + (1/2) d_th g_rr ur^2 + a^2 s c uth^2 - 2 r ur uth
    const T Fth = fma(-K.r, uruth2, fma(K.a2sc, uthuth, fma(-K.c1, urur, Qth)));

    // raise with the (t, phi) block inverse and g^rr, g^thth
    at = fma(K.Rtt, Wt, -K.Rtp * Wp);
    aph = fma(K.Rpp, Wp, -K.Rtp * Wt);
    ar = Fr * K.Dirho2;
    ath = Fth * K.irho2;
    if (keep) *keep = KerrContr<T>{Pt_r, Pt_th, Pp_r, Pp_th, Wt, Wp, Fr, Fth};
}

// du^mu/dtau for the 4-velocity (ut, ur, uth, uph) at (r, theta) with s = sin theta,
// c = cos theta.  T = double or float.  The same acceleration as kerr_contract with the
// coefficients of kerr_coef (the direct form, which the adjoint differentiates),
// regrouped so that fewer intermediate products are formed.  With V = u^t - a s^2 u^phi
// and A = r^2 + a^2, the half partials of the (t, phi) metric components contracted
// with u^b are
//   (1/2)(d_r g_tb) u^b = (1/2) d_r q V,   (1/2)(d_th g_tb) u^b = (1/2) d_th q V - a q s c u^phi,
//   (1/2)(d_l g_pb) u^b = -a s^2 (1/2)(d_l g_tb) u^b + X_l,
//   X_r = r s^2 u^phi,   X_th = -a q s c V + A s c u^phi,
// so with Wt = u^l (1/2)(d_l g_tb) u^b and Y = u^r X_r + u^theta X_th the lowered
// accelerations are F_t = -2 Wt, F_phi = -2 (-a s^2 Wt + Y), and the block inverse of the
// (t, phi) metric (determinant -Delta s^2) raises them to
//   a^t = (2 / Delta) (A Wt + a q Y),   a^phi = (2 a / Delta) Wt + (2 (q - 1) / (Delta s^2)) Y
// (g_phiphi and g_tphi cancel out of both).  g^rr = Delta / rho^2 and g^thth = 1 / rho^2
// are folded into the r and theta coefficients (with (1/2) d_th g_rr = -a^2 s c / Delta):
//   a^r = (Delta / rho^2)(Qr + r (u^theta)^2) + (a^2 s c / rho^2) 2 u^r u^theta
//         - (r / rho^2 - (r - M) / Delta) (u^r)^2,
//   a^theta = (Qth - 2 r u^r u^theta) / rho^2 + (a^2 s c / rho^2)((u^theta)^2 - (u^r)^2 / Delta),
// Q_l = u^t (1/2)(d_l g_tb) u^b + u^phi (1/2)(d_l g_pb) u^b = (1/2)(d_l g_tb) u^b V + u^phi X_l
// being the (t, phi) part of (1/2)(d_l g_ab) u^a u^b.
template <typename T>
MALBEC_HD inline void kerr_accel(T M, T a, T r, T s, T c, T ut, T ur, T uth, T uph, T &at, T &ar,
                                 T &ath, T &aph)
{
    const T a2 = a * a;
    const T s2 = s * s;
    const T sc = s * c;
    const T r2 = r * r;
    const T A = r2 + a2;                    // r^2 + a^2
    const T rho2 = fma(-a2, s2, A);         // r^2 + a^2 cos^2 = A - a^2 sin^2
    const T M2 = M + M;
    const T Delta = fma(-M2, r, A);         // r^2 - 2 M r + a^2
    const T Ds2 = Delta * s2;
    const T inv = recip(rho2 * Ds2);        // 1 / (rho^2 Delta s^2)
    const T iDs2 = inv * rho2;              // 1 / (Delta s^2)
    const T irho2 = inv * Ds2;              // 1 / rho^2
    const T iDelta = iDs2 * s2;             // 1 / Delta
    const T ri = r * irho2;                 // r / rho^2
    const T q = M2 * ri;                    // 2 M r / rho^2;  g_tt = q - 1
    const T hdq_r = fma(-q, ri, M * irho2); // (1/2) d_r q
    const T k1 = (a2 * sc) * irho2;         // a^2 s c / rho^2
    const T hdq_th = q * k1;                // (1/2) d_th q
    const T aq = -a * q;                    // g_tphi / s^2
    const T as2n = -a * s2;
    const T aqsc = aq * sc;

    const T V = fma(as2n, uph, ut);
    const T Pt_r = hdq_r * V;               // (1/2) (d_r g_tb) u^b
    const T Pt_th = fma(hdq_th, V, aqsc * uph);
    const T X_r = (r * s2) * uph;
    const T X_th = fma(aqsc, V, (A * sc) * uph);
    const T Wt = fma(ur, Pt_r, uth * Pt_th);
    const T Y = fma(ur, X_r, uth * X_th);
    const T Qr = fma(Pt_r, V, uph * X_r);
    const T Qth = fma(Pt_th, V, uph * X_th);
    const T urur = ur * ur, uthuth = uth * uth, uruth2 = (ur + ur) * uth;  // 2 ur uth

    const T iDelta2 = iDelta + iDelta;
    at = iDelta2 * fma(A, Wt, -aq * Y);
    aph = fma(a * iDelta2, Wt, (iDs2 * fma(T(2), q, T(-2))) * Y);
    const T e_rr = fma(-iDelta, r - M, ri);
    ar = fma(k1, uruth2, fma(-e_rr, urur, (Delta * irho2) * fma(r, uthuth, Qr)));
    ath = fma(irho2, fma(-r, uruth2, Qth), k1 * fma(-iDelta, urur, uthuth));
}

// Reverse mode of kerr_accel: given the cotangents (bat, bar, bath, baph) of
// (a^t, a^r, a^theta, a^phi), the cotangents of r, s = sin theta, c = cos theta and
// of the 4-velocity (ub[0..3] for u^t, u^r, u^theta, u^phi), i.e. the transposed
// Jacobian of the computed expression applied to b.  The forward expressions are
// those of kerr_accel, recomputed here; each reverse step below transposes one of them
// (x = f(y, z) adds xb df/dy to yb and xb df/dz to zb).  M and a are constants.
template <typename T>
MALBEC_HD inline void kerr_accel_vjp(T M, T a, T r, T s, T c, T ut, T ur, T uth, T uph, T bat,
                                     T bar, T bath, T baph, T &rb, T &sb, T &cb, T ub[4])
{
    const T a2 = a * a;
    const T s2 = s * s;
    const T sc = s * c;
    const T r2 = r * r;
    const T A = r2 + a2;
    const T rho2 = fma(a2, c * c, r2);
    const T M2 = M + M;
    const T Delta = fma(-M2, r, A);
    const T Ds2 = Delta * s2;
    const T inv = recip(rho2 * Ds2);
    const T iDs2 = inv * rho2;
    const T irho2 = inv * Ds2;
    const T iDelta = iDs2 * s2;
    const T ri = r * irho2;
    const T q = M2 * ri;
    const T hdq_r = fma(-q, ri, M * irho2);
    const T a2sc = a2 * sc;
    const T k1 = a2sc * irho2;
    const T hdq_th = q * k1;
    const T aq = -a * q;
    const T as2n = -a * s2;
    const T aqsc = aq * sc;
    const T V = fma(as2n, uph, ut);
    const T Pt_r = hdq_r * V;
    const T Pt_th = fma(hdq_th, V, aqsc * uph);
    const T rs2 = r * s2;
    const T X_r = rs2 * uph;
    const T Asc = A * sc;
    const T X_th = fma(aqsc, V, Asc * uph);
    const T Wt = fma(ur, Pt_r, uth * Pt_th);
    const T Y = fma(ur, X_r, uth * X_th);
    const T Qr = fma(Pt_r, V, uph * X_r);
    const T Qth = fma(Pt_th, V, uph * X_th);
    const T urur = ur * ur, uthuth = uth * uth, uruth2 = (ur + ur) * uth;
    const T iDelta2 = iDelta + iDelta;
    const T T1 = fma(A, Wt, -aq * Y);           // a^t = iDelta2 T1
    const T aiD2 = a * iDelta2;
    const T q2m2 = fma(T(2), q, T(-2));
    const T C2 = iDs2 * q2m2;                   // a^phi = aiD2 Wt + C2 Y
    const T rmM = r - M;
    const T e_rr = fma(-iDelta, rmM, ri);
    const T DI = Delta * irho2;
    const T G = fma(r, uthuth, Qr);             // a^r = k1 uruth2 - e_rr urur + DI G
    const T H = fma(-r, uruth2, Qth);           // a^theta = irho2 H + k1 Kk
    const T Kk = fma(-iDelta, urur, uthuth);

    // a^theta = irho2 H + k1 Kk
    T irho2b = bath * H;
    const T Hb = bath * irho2;
    T k1b = bath * Kk;
    const T Kkb = bath * k1;
    // Kk = uthuth - iDelta urur
    T iDeltab = -Kkb * urur;
    T ururb = -Kkb * iDelta;
    T uthuthb = Kkb;
    // H = Qth - r uruth2
    T rbar = -Hb * uruth2;
    T uruth2b = -Hb * r;
    const T Qthb = Hb;
    // a^r = k1 uruth2 - e_rr urur + DI G
    k1b = fma(bar, uruth2, k1b);
    uruth2b = fma(bar, k1, uruth2b);
    const T e_rrb = -bar * urur;
    ururb = fma(-bar, e_rr, ururb);
    const T DIb = bar * G;
    const T Gb = bar * DI;
    // G = r uthuth + Qr
    rbar = fma(Gb, uthuth, rbar);
    uthuthb = fma(Gb, r, uthuthb);
    const T Qrb = Gb;
    // DI = Delta irho2
    T Deltab = DIb * irho2;
    irho2b = fma(DIb, Delta, irho2b);
    // e_rr = ri - iDelta (r - M)
    iDeltab = fma(-e_rrb, rmM, iDeltab);
    rbar = fma(-e_rrb, iDelta, rbar);
    T rib = e_rrb;
    // a^phi = aiD2 Wt + C2 Y, aiD2 = a iDelta2
    T iDelta2b = a * (baph * Wt);
    T Wtb = baph * aiD2;
    const T C2b = baph * Y;
    T Yb = baph * C2;
    // C2 = iDs2 (2 q - 2)
    T iDs2b = C2b * q2m2;
    T qb = (C2b + C2b) * iDs2;
    // a^t = iDelta2 T1
    iDelta2b = fma(bat, T1, iDelta2b);
    const T T1b = bat * iDelta2;
    // T1 = A Wt - aq Y
    T Ab = T1b * Wt;
    Wtb = fma(T1b, A, Wtb);
    T aqb = -T1b * Y;
    Yb = fma(-T1b, aq, Yb);
    // iDelta2 = 2 iDelta
    iDeltab = fma(T(2), iDelta2b, iDeltab);
    // Qth = Pt_th V + uph X_th
    T Pt_thb = Qthb * V;
    T Vb = Qthb * Pt_th;
    T uphb = Qthb * X_th;
    T X_thb = Qthb * uph;
    // Qr = Pt_r V + uph X_r
    T Pt_rb = Qrb * V;
    Vb = fma(Qrb, Pt_r, Vb);
    uphb = fma(Qrb, X_r, uphb);
    T X_rb = Qrb * uph;
    // Y = ur X_r + uth X_th
    T urb = Yb * X_r;
    X_rb = fma(Yb, ur, X_rb);
    T uthb = Yb * X_th;
    X_thb = fma(Yb, uth, X_thb);
    // Wt = ur Pt_r + uth Pt_th
    urb = fma(Wtb, Pt_r, urb);
    Pt_rb = fma(Wtb, ur, Pt_rb);
    uthb = fma(Wtb, Pt_th, uthb);
    Pt_thb = fma(Wtb, uth, Pt_thb);
    // X_th = aqsc V + Asc uph, Asc = A sc
    T aqscb = X_thb * V;
    Vb = fma(X_thb, aqsc, Vb);
    const T Ascb = X_thb * uph;
    uphb = fma(X_thb, Asc, uphb);
    Ab = fma(Ascb, sc, Ab);
    T scb = Ascb * A;
    // X_r = rs2 uph, rs2 = r s2
    const T rs2b = X_rb * uph;
    uphb = fma(X_rb, rs2, uphb);
    rbar = fma(rs2b, s2, rbar);
    T s2b = rs2b * r;
    // Pt_th = hdq_th V + aqsc uph
    const T hdq_thb = Pt_thb * V;
    Vb = fma(Pt_thb, hdq_th, Vb);
    aqscb = fma(Pt_thb, uph, aqscb);
    uphb = fma(Pt_thb, aqsc, uphb);
    // Pt_r = hdq_r V
    const T hdq_rb = Pt_rb * V;
    Vb = fma(Pt_rb, hdq_r, Vb);
    // V = ut + as2n uph
    const T as2nb = Vb * uph;
    uphb = fma(Vb, as2n, uphb);
    // aqsc = aq sc, as2n = -a s2, aq = -a q
    aqb = fma(aqscb, sc, aqb);
    scb = fma(aqscb, aq, scb);
    s2b = fma(-a, as2nb, s2b);
    qb = fma(-a, aqb, qb);
    // hdq_th = q k1
    qb = fma(hdq_thb, k1, qb);
    k1b = fma(hdq_thb, q, k1b);
    // k1 = a2sc irho2, a2sc = a^2 sc
    scb = fma(a2 * k1b, irho2, scb);
    irho2b = fma(k1b, a2sc, irho2b);
    // hdq_r = M irho2 - q ri
    qb = fma(-hdq_rb, ri, qb);
    rib = fma(-hdq_rb, q, rib);
    irho2b = fma(hdq_rb, M, irho2b);
    // q = M2 ri, ri = r irho2
    rib = fma(qb, M2, rib);
    rbar = fma(rib, irho2, rbar);
    irho2b = fma(rib, r, irho2b);
    // iDelta = iDs2 s2
    iDs2b = fma(iDeltab, s2, iDs2b);
    s2b = fma(iDeltab, iDs2, s2b);
    // irho2 = inv Ds2, iDs2 = inv rho2, inv = 1 / (rho2 Ds2)
    const T invb = fma(irho2b, Ds2, iDs2b * rho2);
    T Ds2b = irho2b * inv;
    T rho2b = iDs2b * inv;
    const T P0b = -invb * (inv * inv);
    rho2b = fma(P0b, Ds2, rho2b);
    Ds2b = fma(P0b, rho2, Ds2b);
    // Ds2 = Delta s2
    Deltab = fma(Ds2b, s2, Deltab);
    s2b = fma(Ds2b, Delta, s2b);
    // Delta = A - M2 r
    rbar = fma(-M2, Deltab, rbar);
    Ab = Ab + Deltab;
    // rho2 = r2 + a2 c^2, A = r2 + a2, r2 = r r
    rbar = fma(r + r, rho2b + Ab, rbar);
    // s2 = s s, sc = s c, c^2
    sb = fma(scb, c, (s + s) * s2b);
    cb = fma(scb, s, (c + c) * (a2 * rho2b));
    rb = rbar;
    // urur, uthuth, uruth2 = 2 ur uth
    ub[0] = Vb;
    ub[1] = fma(ur + ur, ururb, fma(uth + uth, uruth2b, urb));
    ub[2] = fma(uth + uth, uthuthb, fma(ur + ur, uruth2b, uthb));
    ub[3] = uphb;
}

// The direct form: coefficients, then contraction, as the adjoint differentiates it.
template <typename T>
MALBEC_HD inline void kerr_accel_direct(T M, T a, T r, T s, T c, T ut, T ur, T uth, T uph, T &at,
                                        T &ar, T &ath, T &aph)
{
    KerrCoef<T> K;
    kerr_coef(M, a, r, s, c, K);
    kerr_contract(K, ut, ur, uth, uph, at, ar, ath, aph);
}

// Stages of one classic RK4 step (b = 1/6, 1/3, 1/3, 1/6; c = 0, 1/2, 1/2, 1) of all
// 8 components; accel(stage, r, th, ut, ur, uth, uph, at, ar, ath, aph) evaluates
// du/dtau at stage point `stage` (0 = the step's start).
// The right-hand side does not depend on t or phi, so only (r, theta, u) are formed
// at the stage points; t and phi accumulate the stage values of u^t and u^phi with
// the same weights.  sr[] receives the radii of the three intermediate stage points
// and acc[] the weighted sum k1 + 2 k2 + 2 k3 + k4.
template <typename T, typename Accel>
MALBEC_HD inline void rk4_stages(Accel &accel, T h, const T y[8], T acc[8], T sr[3])
{
    const T hh = T(0.5) * h;
    T at, ar, ath, aph;
    T s1, s2, s3, s4, s5, s6; // stage point (r, th, ut, ur, uth, uph)

    // k1 = f(y)
    accel(0, y[1], y[2], y[4], y[5], y[6], y[7], at, ar, ath, aph);
    acc[0] = y[4]; acc[1] = y[5]; acc[2] = y[6]; acc[3] = y[7];
    acc[4] = at; acc[5] = ar; acc[6] = ath; acc[7] = aph;
    s1 = fma(hh, y[5], y[1]); s2 = fma(hh, y[6], y[2]);
    s3 = fma(hh, at, y[4]); s4 = fma(hh, ar, y[5]); s5 = fma(hh, ath, y[6]); s6 = fma(hh, aph, y[7]);
    sr[0] = s1;

    // k2 = f(y + h/2 k1)
    accel(1, s1, s2, s3, s4, s5, s6, at, ar, ath, aph);
    acc[0] = fma(T(2), s3, acc[0]); acc[1] = fma(T(2), s4, acc[1]);
    acc[2] = fma(T(2), s5, acc[2]); acc[3] = fma(T(2), s6, acc[3]);
    acc[4] = fma(T(2), at, acc[4]); acc[5] = fma(T(2), ar, acc[5]);
    acc[6] = fma(T(2), ath, acc[6]); acc[7] = fma(T(2), aph, acc[7]);
    {
        T n1 = fma(hh, s4, y[1]), n2 = fma(hh, s5, y[2]);
        T n3 = fma(hh, at, y[4]), n4 = fma(hh, ar, y[5]), n5 = fma(hh, ath, y[6]), n6 = fma(hh, aph, y[7]);
        s1 = n1; s2 = n2; s3 = n3; s4 = n4; s5 = n5; s6 = n6;
    }
    sr[1] = s1;

    // k3 = f(y + h/2 k2)
    accel(2, s1, s2, s3, s4, s5, s6, at, ar, ath, aph);
    acc[0] = fma(T(2), s3, acc[0]); acc[1] = fma(T(2), s4, acc[1]);
    acc[2] = fma(T(2), s5, acc[2]); acc[3] = fma(T(2), s6, acc[3]);
    acc[4] = fma(T(2), at, acc[4]); acc[5] = fma(T(2), ar, acc[5]);
    acc[6] = fma(T(2), ath, acc[6]); acc[7] = fma(T(2), aph, acc[7]);
    {
        T n1 = fma(h, s4, y[1]), n2 = fma(h, s5, y[2]);
        T n3 = fma(h, at, y[4]), n4 = fma(h, ar, y[5]), n5 = fma(h, ath, y[6]), n6 = fma(h, aph, y[7]);
        s1 = n1; s2 = n2; s3 = n3; s4 = n4; s5 = n5; s6 = n6;
    }
    sr[2] = s1;

    // k4 = f(y + h k3)
    accel(3, s1, s2, s3, s4, s5, s6, at, ar, ath, aph);
    acc[0] += s3; acc[1] += s4; acc[2] += s5; acc[3] += s6;
    acc[4] += at; acc[5] += ar; acc[6] += ath; acc[7] += aph;
}

// y1 = y + h/6 (k1 + 2 k2 + 2 k3 + k4)
template <typename T, typename Accel>
MALBEC_HD inline void rk4_step(Accel &accel, T h, const T y[8], T y1[8], T sr[3])
{
    T acc[8];
    rk4_stages(accel, h, y, acc, sr);
    const T h6 = h * T(1.0 / 6.0);
    // acc[0..3] hold the weighted sums of (u^t, u^r, u^theta, u^phi) = dx/dtau
#pragma unroll
    for (int k = 0; k < 8; ++k) y1[k] = fma(h6, acc[k], y[k]);
}

// The increment d = h/6 (k1 + 2 k2 + 2 k3 + k4) alone (compensated updates).
template <typename T, typename Accel>
MALBEC_HD inline void rk4_delta(Accel &accel, T h, const T y[8], T d[8], T sr[3])
{
    T acc[8];
    rk4_stages(accel, h, y, acc, sr);
    const T h6 = h * T(1.0 / 6.0);
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = h6 * acc[k];
}

// Transposed RK4 step: lam <- (d y1 / d y)^T lam for the step y -> y1 of rk4_step.
// With k_i = f(Y_i), Y_1 = y, Y_2 = y + h/2 k_1, Y_3 = y + h/2 k_2, Y_4 = y + h k_3 and
// y1 = y + h/6 (k_1 + 2 k_2 + 2 k_3 + k_4), the cotangents of the stage values are
//   lk_4 = h/6 lam,  lk_3 = h/3 lam + h J_4^T lk_4,
//   lk_2 = h/3 lam + h/2 J_3^T lk_3,  lk_1 = h/6 lam + h/2 J_2^T lk_2,
// and lam_y = lam + sum_i J_i^T lk_i, where J_i = df/dy at Y_i.  f = (u, a(r, theta, u)),
// so J^T lk has no t or phi component, (da/d(r, theta))^T lk_a in r and theta, and
// lk_x + (da/du)^T lk_a in u.  F supplies the forward stage accelerations exactly as
// rk4_stages forms them (operator()), the trigonometry of the last stage point
// (prepare(3, theta)), the transposed Jacobian of the acceleration at a stage point
// (vjp(stage, ...), returning the cotangents of r, theta and u), and the storage of the
// stage points between the two passes (Y(stage, k), k = r, theta, u^t, u^r, u^theta,
// u^phi; keep() between the passes, after which they are read back from that storage).
template <typename T, typename F>
MALBEC_HD inline void rk4_vjp(F &f, T h, const T y[8], T lam[8])
{
    const T hh = T(0.5) * h;
    T at, ar, ath, aph;
    {
        T r = y[1], th = y[2], ut = y[4], ur = y[5], uth = y[6], uph = y[7];
        f.Y(0, 0) = r; f.Y(0, 1) = th; f.Y(0, 2) = ut; f.Y(0, 3) = ur; f.Y(0, 4) = uth; f.Y(0, 5) = uph;
        f(0, r, th, ut, ur, uth, uph, at, ar, ath, aph);
        r = fma(hh, y[5], y[1]); th = fma(hh, y[6], y[2]);
        ut = fma(hh, at, y[4]); ur = fma(hh, ar, y[5]); uth = fma(hh, ath, y[6]); uph = fma(hh, aph, y[7]);
        f.Y(1, 0) = r; f.Y(1, 1) = th; f.Y(1, 2) = ut; f.Y(1, 3) = ur; f.Y(1, 4) = uth; f.Y(1, 5) = uph;
        f(1, r, th, ut, ur, uth, uph, at, ar, ath, aph);
        r = fma(hh, ur, y[1]); th = fma(hh, uth, y[2]);
        ut = fma(hh, at, y[4]); ur = fma(hh, ar, y[5]); uth = fma(hh, ath, y[6]); uph = fma(hh, aph, y[7]);
        f.Y(2, 0) = r; f.Y(2, 1) = th; f.Y(2, 2) = ut; f.Y(2, 3) = ur; f.Y(2, 4) = uth; f.Y(2, 5) = uph;
        f(2, r, th, ut, ur, uth, uph, at, ar, ath, aph);
        r = fma(h, ur, y[1]); th = fma(h, uth, y[2]);
        ut = fma(h, at, y[4]); ur = fma(h, ar, y[5]); uth = fma(h, ath, y[6]); uph = fma(h, aph, y[7]);
        f.Y(3, 0) = r; f.Y(3, 1) = th; f.Y(3, 2) = ut; f.Y(3, 3) = ur; f.Y(3, 4) = uth; f.Y(3, 5) = uph;
        f.prepare(3, th);
    }
    f.keep();

    const T h6 = h * T(1.0 / 6.0), h3 = T(2) * h6;
    T ly[8], lk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { ly[k] = lam[k]; lk[k] = h6 * lam[k]; }
#pragma unroll
    for (int st = 3; st >= 0; --st) {
        // mu = J(Y_st)^T lk
        T mr, mth, mu[4];
        f.vjp(st, f.Y(st, 0), f.Y(st, 1), f.Y(st, 2), f.Y(st, 3), f.Y(st, 4), f.Y(st, 5), lk[4],
              lk[5], lk[6], lk[7], mr, mth, mu);
#pragma unroll
        for (int k = 0; k < 4; ++k) mu[k] += lk[k];
        ly[1] += mr;
        ly[2] += mth;
#pragma unroll
        for (int k = 0; k < 4; ++k) ly[4 + k] += mu[k];
        if (st > 0) {
            // lk of the previous stage: its weight times lam plus its offset coefficient times mu
            const T w = st == 1 ? h6 : h3;
            const T o = st == 3 ? h : hh;
            lk[0] = w * lam[0];
            lk[1] = fma(o, mr, w * lam[1]);
            lk[2] = fma(o, mth, w * lam[2]);
            lk[3] = w * lam[3];
#pragma unroll
            for (int k = 0; k < 4; ++k) lk[4 + k] = fma(o, mu[k], w * lam[4 + k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) lam[k] = ly[k];
}

}  // namespace malbec
