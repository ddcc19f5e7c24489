// Chart frames (section 3, the chart parametrisation; the quadratic-skeleton
// section for curved patches): base point T(u, v) and direction H(u, v) of
// chart j and their derivatives, shared by the projection, chart-geometry
// and chart-curvature kernels.  Device-only; fp64.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace lss {

// Monomial coefficients of a quadratic patch t6 (corners P1, P2, P3, then the
// edge points of P1P2, P2P3, P3P1): the Lagrange interpolant through the six
// points is y = P1 + u (A + u C + v E) + v (B + v D).
__device__ inline void patch_coef(const double *__restrict__ verts, const int32_t *__restrict__ t6, double P1[3],
                                  double A[3], double B[3], double C[3], double D[3], double E[3]) {
    for (int c = 0; c < 3; ++c) {
        P1[c] = verts[3 * (int64_t)t6[0] + c];
        const double d2 = verts[3 * (int64_t)t6[1] + c] - P1[c];
        const double d3 = verts[3 * (int64_t)t6[2] + c] - P1[c];
        const double d4 = verts[3 * (int64_t)t6[3] + c] - P1[c];
        const double d5 = verts[3 * (int64_t)t6[4] + c] - P1[c];
        const double d6 = verts[3 * (int64_t)t6[5] + c] - P1[c];
        A[c] = 4.0 * d4 - d2;
        B[c] = 4.0 * d6 - d3;
        C[c] = 2.0 * (d2 - 2.0 * d4);
        D[c] = 2.0 * (d3 - 2.0 * d6);
        E[c] = 4.0 * (d5 - d4 - d6);
    }
}

// Chart frame of chart node idx = j * np + i: base point T (eq. tparam) and
// direction H (eq. mkpseudovec) and their derivatives in (u, v).  H is linear
// in the vertex pseudonormals (H_uu = 0); T is linear on the corner triangle,
// or with tris6 the quadratic patch (constant second derivatives).
struct ChartFrame {
    double T[3], Tu[3], Tv[3], Tuu[3], Tuv[3], Tvv[3];
    double H[3], Hu[3], Hv[3];
};

__device__ inline void chart_frame(const double *__restrict__ verts, const int32_t *__restrict__ tris,
                                   const int32_t *__restrict__ tris6, const double *__restrict__ vH,
                                   const double *__restrict__ uv, int32_t np, int64_t idx, ChartFrame &f,
                                   int64_t &j) {
    j = idx / np;
    const int i = (int)(idx - j * np);
    const double u = uv[2 * i], v = uv[2 * i + 1];
    const int32_t *t = tris + 3 * j;
    for (int c = 0; c < 3; ++c) {
        const double p1 = verts[3 * (int64_t)t[0] + c], p2 = verts[3 * (int64_t)t[1] + c],
                     p3 = verts[3 * (int64_t)t[2] + c];
        const double h1 = vH[3 * (int64_t)t[0] + c], h2 = vH[3 * (int64_t)t[1] + c], h3 = vH[3 * (int64_t)t[2] + c];
        f.T[c] = p1 + u * (p2 - p1) + v * (p3 - p1);
        f.Tu[c] = p2 - p1;
        f.Tv[c] = p3 - p1;
        f.Tuu[c] = f.Tuv[c] = f.Tvv[c] = 0.0;
        f.Hu[c] = h2 - h1;
        f.Hv[c] = h3 - h1;
        f.H[c] = h1 + u * f.Hu[c] + v * f.Hv[c];
    }
    if (tris6) {
        double P1[3], A[3], B[3], C[3], D[3], E[3];
        patch_coef(verts, tris6 + 6 * j, P1, A, B, C, D, E);
        for (int c = 0; c < 3; ++c) {
            f.T[c] = P1[c] + (u * (A[c] + u * C[c] + v * E[c]) + v * (B[c] + v * D[c]));
            f.Tu[c] = A[c] + 2.0 * u * C[c] + v * E[c];
            f.Tv[c] = B[c] + 2.0 * v * D[c] + u * E[c];
            f.Tuu[c] = 2.0 * C[c];
            f.Tuv[c] = E[c];
            f.Tvv[c] = 2.0 * D[c];
        }
    }
}

}  // namespace lss
