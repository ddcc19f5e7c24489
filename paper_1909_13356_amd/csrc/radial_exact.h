// Exact radial functions of the smoothed-indicator kernel and its first two
// derivatives, for the Hessian and target-attached-width sums (device code).
//
// With t = rho^2 s2 = u^2, s2 = 1/(2 sigma^2), and the kernel's normalisation
// c = 1/(4 sqrt2 pi^1.5 sigma^3) factored out (K = c k1, F = K'/rho = c k2,
// G = F'/rho = c k3):
//   t < 9/4:   k1 = S(3), k2 = -2 s2 S(5), k3 = 4 s2^2 S(7),
//              S(m) = sum_k 2 (-t)^k / (k! (2k + m))      (term-wise series)
//   t >= 9/4:  with q = 2/sqrt(pi), e = exp(-t):
//              P3 = erf(u) - q u e,  P5 = P3 - q (2/3) u^3 e,  P7 = P5 - q (4/15) u^5 e
//              (the regularised incomplete gamma functions P(3/2|5/2|7/2, t)),
//              k1 = (sqrt(pi)/2) P3 / u^3, k2 = -(3 sqrt(pi)/2) s2 P5 / u^5,
//              k3 = (15 sqrt(pi)/2) s2^2 P7 / u^7,  and P3 = P5 = P7 = 1 for
//              t >= 50, where the dropped terms are below 1e-18.
#pragma once

#include <hip/hip_runtime.h>

#include "lss_internal.h"

namespace lss {

constexpr double kSqrtPi = 1.7724538509055160273;

// e receives exp(-t) (0 for t >= 50), which the target-attached width needs
__device__ inline void radial3(double t, double s2, double &k1, double &k2, double &k3, double &e) {
    if (t < 2.25) {
        double p = 1.0, a0 = 0.0, a3 = 0.0, a5 = 0.0, a7 = 0.0;
#pragma unroll
        for (int k = 0; k < 30; ++k) {
            a0 += p;
            a3 += p * (2.0 / (2 * k + 3));
            a5 += p * (2.0 / (2 * k + 5));
            a7 += p * (2.0 / (2 * k + 7));
            p *= -t * (1.0 / (k + 1));
        }
        k1 = a3;
        k2 = -2.0 * s2 * a5;
        k3 = 4.0 * s2 * s2 * a7;
        e = a0;
        return;
    }
    // 1/u = t^-1/2: hardware estimate and one third-order correction (to rounding)
    const double iu = rsq64(t);
    double P3 = 1.0, P5 = 1.0, P7 = 1.0;
    e = 0.0;
    if (t < 50.0) {
        const double u = t * iu;
        e = exp(-t);
        const double qe = (2.0 / kSqrtPi) * e;
        const double u3 = u * t;
        P3 = erf(u) - qe * u;
        P5 = P3 - qe * (2.0 / 3.0) * u3;
        P7 = P5 - qe * (4.0 / 15.0) * u3 * t;
    }
    const double iu2 = iu * iu;
    const double iu3 = iu * iu2, iu5 = iu3 * iu2, iu7 = iu5 * iu2;
    k1 = (0.5 * kSqrtPi) * P3 * iu3;
    k2 = -(1.5 * kSqrtPi) * s2 * P5 * iu5;
    k3 = (7.5 * kSqrtPi) * s2 * s2 * P7 * iu7;
}

// Phi, grad Phi and the Hessian (xx, xy, xz, yy, yz, zz) summed over pairs
struct HessAcc {
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    double hxx = 0.0, hxy = 0.0, hxz = 0.0, hyy = 0.0, hyz = 0.0, hzz = 0.0;
};

// one (target, node) pair with the full kernel, node record s (a' = c w J):
//   Phi -= (a'.d) k1,  grad -= a' k1 + (a'.d) k2 d,
//   Hess -= k2 (a' d^T + d a'^T) + (a'.d) k2 I + (a'.d) k3 d d^T
__device__ inline void pair_hess(const Src &s, double px, double py, double pz, HessAcc &A) {
    const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
    const double t = (dx * dx + dy * dy + dz * dz) * s.s2;
    double k1, k2, k3, et;
    radial3(t, s.s2, k1, k2, k3, et);
    const double ad = s.ax * dx + s.ay * dy + s.az * dz;
    A.f -= ad * k1;
    const double adk2 = ad * k2, adk3 = ad * k3;
    A.gx -= s.ax * k1 + adk2 * dx;
    A.gy -= s.ay * k1 + adk2 * dy;
    A.gz -= s.az * k1 + adk2 * dz;
    const double ex = adk3 * dx, ey = adk3 * dy, ez = adk3 * dz;
    A.hxx -= 2.0 * k2 * s.ax * dx + adk2 + ex * dx;
    A.hyy -= 2.0 * k2 * s.ay * dy + adk2 + ey * dy;
    A.hzz -= 2.0 * k2 * s.az * dz + adk2 + ez * dz;
    A.hxy -= k2 * (s.ax * dy + s.ay * dx) + ex * dy;
    A.hxz -= k2 * (s.ax * dz + s.az * dx) + ex * dz;
    A.hyz -= k2 * (s.ay * dz + s.az * dy) + ey * dz;
}

// Phi, grad Phi and dPhi/dsigma-sum with a target-attached width: the node
// record's a' carries the normalisation c(sigma_k) of its own width (s2 =
// 1/(2 sigma_k^2)), the target's s2x = 1/(2 sigma(x)^2) sets the kernel, and
// each pair is rescaled by c(sigma(x)) / c(sigma_k) = (s2x / s2)^(3/2), so the
// sums carry c(sigma(x)) a.
struct MsAcc {
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, e = 0.0;
};

__device__ inline void pair_ms(const Src &s, double px, double py, double pz, double s2x, MsAcc &A) {
    const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
    const double t = (dx * dx + dy * dy + dz * dz) * s2x;
    double k1, k2, k3, et;
    radial3(t, s2x, k1, k2, k3, et);
    const double q = s2x / s.s2, fr = q * sqrt(q);
    const double ax = fr * s.ax, ay = fr * s.ay, az = fr * s.az;
    const double ad = ax * dx + ay * dy + az * dz;
    A.f += ad * k1;
    const double adk2 = ad * k2;
    A.gx += ax * k1 + adk2 * dx;
    A.gy += ay * k1 + adk2 * dy;
    A.gz += az * k1 + adk2 * dz;
    A.e += ad * et;
}

}  // namespace lss
