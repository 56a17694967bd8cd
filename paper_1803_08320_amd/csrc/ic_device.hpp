// Device helpers that build 4-velocities from constants of motion (Carter's
// separated equations of the Kerr geodesics) and the inverse Kerr metric.
// Used by the initial-condition builder and by the camera.
#pragma once

#include <hip/hip_runtime.h>

namespace malbec {

// Inverse-metric pieces at (r, theta): g^tt, g^tphi, g^phiphi, g^rr, g^thth.
__device__ __forceinline__ void inverse_metric(double M, double a, double r, double s, double c,
                                               double &itt, double &itp, double &ipp, double &irr,
                                               double &ithth)
{
    const double a2 = a * a, s2 = s * s, r2 = r * r;
    const double rho2 = r2 + a2 * c * c;
    const double Delta = r2 - 2.0 * M * r + a2;
    const double Sigma = (r2 + a2) * (r2 + a2) - a2 * Delta * s2;
    const double den = rho2 * Delta;
    itt = -Sigma / den;
    itp = -2.0 * M * a * r / den;
    ipp = (Delta - a2 * s2) / (den * s2);
    irr = Delta / rho2;
    ithth = 1.0 / rho2;
}

// 4-velocity from the constants of motion (Carter): with P = E (r^2 + a^2) - a L_z,
// rho^2 u^r = s_r sqrt(R), rho^2 u^theta = s_th sqrt(Theta),
// rho^2 u^t = (r^2 + a^2) P / Delta + a (L_z - a E sin^2),
// rho^2 u^phi = a P / Delta + L_z / sin^2 - a E.
__device__ __forceinline__ void velocity(double M, double a, double E, double Lz, double Q,
                                         double mu2, double r, double s, double c, double sr,
                                         double sth, double R, double Th, double u[4])
{
    const double a2 = a * a, s2 = s * s, r2 = r * r;
    const double rho2 = r2 + a2 * c * c;
    const double Delta = r2 - 2.0 * M * r + a2;
    const double P = E * (r2 + a2) - a * Lz;
    (void)mu2;
    (void)Q;
    u[0] = ((r2 + a2) * P / Delta + a * (Lz - a * E * s2)) / rho2;
    u[1] = sr * sqrt(fmax(R, 0.0)) / rho2;
    u[2] = sth * sqrt(fmax(Th, 0.0)) / rho2;
    u[3] = (a * P / Delta + Lz / s2 - a * E) / rho2;
}

__device__ __forceinline__ double radial_potential(double M, double a, double E, double Lz, double Q,
                                                   double mu2, double r)
{
    const double a2 = a * a, r2 = r * r;
    const double P = E * (r2 + a2) - a * Lz;
    const double Delta = r2 - 2.0 * M * r + a2;
    const double L = Lz - a * E;
    return P * P - Delta * (mu2 * r2 + L * L + Q);
}

__device__ __forceinline__ double polar_potential(double a, double E, double Lz, double Q, double mu2,
                                                  double s, double c)
{
    return Q - c * c * (a * a * (mu2 - E * E) + Lz * Lz / (s * s));
}

}  // namespace malbec
