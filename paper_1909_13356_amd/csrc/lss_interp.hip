// Polynomial interpolation of chart data between the chart nodes (section
// 3.3: each chart is approximated on the standard simplex T0 by a polynomial
// of total degree p, through an orthogonal basis of Koornwinder polynomials
// sampled at the p-th order nodes).  The interpolation matrix from the np
// nodes to the ne evaluation points is the same for every triangle: it is
// formed on the host, I = E V^-1 with V_ik = K_k(node i), E_ek = K_k(point e),
// and a kernel applies it to every triangle's node values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "lss_internal.h"

namespace lss {

namespace {

// Koornwinder (Dubiner) basis on T0 = {u, v >= 0, u + v <= 1}, ordered by
// (m, n) with m + n <= p:  K_mn = L_m(s, t) P_n^(2m+1,0)(2v - 1), where
// s = 2u + v - 1, t = 1 - v and L_m(s, t) = t^m P_m(s / t) is the Legendre
// polynomial made homogeneous (a polynomial in u, v also at v = 1).
void koornwinder(double u, double v, int p, double *out) {
    const double s = 2.0 * u + v - 1.0, t = 1.0 - v, x = 2.0 * v - 1.0;
    std::vector<double> L(p + 1);
    L[0] = 1.0;
    if (p >= 1) L[1] = s;
    for (int m = 1; m < p; ++m) L[m + 1] = ((2.0 * m + 1.0) * s * L[m] - m * t * t * L[m - 1]) / (m + 1.0);
    int k = 0;
    for (int m = 0; m <= p; ++m) {
        const double a = 2.0 * m + 1.0;           // Jacobi P_n^(a, 0)
        double pm2 = 0.0, pm1 = 1.0;
        for (int n = 0; m + n <= p; ++n) {
            double pn;
            if (n == 0) pn = 1.0;
            else if (n == 1) pn = 0.5 * ((a + 2.0) * x + a);
            else {
                const double c = 2.0 * n + a;
                pn = ((c - 1.0) * (c * (c - 2.0) * x + a * a) * pm1 - 2.0 * (n + a - 1.0) * (n - 1.0) * c * pm2) /
                     (2.0 * n * (n + a) * (c - 2.0));
            }
            if (n >= 1) { pm2 = pm1; pm1 = pn; }
            out[k++] = L[m] * pn;
        }
    }
}

// one thread per (triangle j, point e); IT is the interpolation matrix
// stored node-major (IT[i * ne + e]), so the threads of a wave, which hold
// consecutive points, read consecutive entries
__global__ void k_chart_interp(int64_t ntris, int32_t np, int32_t ne, int32_t ncomp, const double *__restrict__ IT,
                               const double *__restrict__ f, double *out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ntris * ne) return;
    const int64_t j = q / ne;
    const int32_t e = (int32_t)(q - j * ne);
    const double *fj = f + j * np * ncomp;
    for (int32_t c = 0; c < ncomp; ++c) {
        double acc = 0.0;
        for (int32_t i = 0; i < np; ++i) acc = fma(IT[(int64_t)i * ne + e], fj[(int64_t)i * ncomp + c], acc);
        out[q * ncomp + c] = acc;
    }
}

// Same product with the interpolation matrix staged once per workgroup in
// LDS, and with the node values of the (at most tpb) triangles that a
// workgroup's 256 consecutive outputs touch staged in LDS per pass of the
// grid-stride loop (when both fit); three independent sums for
// three-component data.
__global__ __launch_bounds__(256) void k_chart_interp_lds(int64_t ntris, int32_t np, int32_t ne, int32_t ncomp,
                                                          int32_t tpb, const double *__restrict__ IT,
                                                          const double *__restrict__ f, double *out) {
    extern __shared__ double sm[];
    double *sIT = sm, *sF = sm + (int64_t)np * ne;
    for (int k = threadIdx.x; k < np * ne; k += blockDim.x) sIT[k] = IT[k];
    const int64_t n = ntris * ne, per = (int64_t)np * ncomp;
    for (int64_t qb = (int64_t)blockIdx.x * blockDim.x; qb < n; qb += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jb = qb / ne;                           // first triangle of this pass
        const int64_t je = ((qb + blockDim.x < n ? qb + blockDim.x : n) - 1) / ne;   // last one
        __syncthreads();                                      // previous pass is done with sF
        const int64_t cnt = (je - jb + 1) * per;              // <= tpb * per by the host's choice of tpb
        for (int64_t k = threadIdx.x; k < cnt; k += blockDim.x) sF[k] = f[jb * per + k];
        __syncthreads();
        const int64_t q = qb + threadIdx.x;
        if (q >= n) continue;
        const int64_t j = q / ne;
        const int32_t e = (int32_t)(q - j * ne);
        const double *fj = sF + (j - jb) * per;
        if (ncomp == 3) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 5
            for (int32_t i = 0; i < np; ++i) {
                const double w = sIT[i * ne + e];
                a0 = fma(w, fj[3 * i], a0);
                a1 = fma(w, fj[3 * i + 1], a1);
                a2 = fma(w, fj[3 * i + 2], a2);
            }
            out[3 * q] = a0;
            out[3 * q + 1] = a1;
            out[3 * q + 2] = a2;
        } else {
            for (int32_t c = 0; c < ncomp; ++c) {
                double acc = 0.0;
                for (int32_t i = 0; i < np; ++i) acc = fma(sIT[i * ne + e], fj[(int64_t)i * ncomp + c], acc);
                out[q * ncomp + c] = acc;
            }
        }
    }
}

}  // namespace

void chart_interp(Ctx &c, const double *chart_uv, int32_t np, const double *f, int32_t ncomp, const double *eval_uv,
                  int32_t ne, double *out, unsigned flags) {
    if (!c.have_sources) throw Error{LSS_ESTATE, "lss_chart_interp: no sources set"};
    if (np <= 0 || ne <= 0 || ncomp <= 0) throw Error{LSS_EINVAL, "lss_chart_interp: np, ne and ncomp must be >= 1"};
    if (!chart_uv || !f || !eval_uv || !out) throw Error{LSS_EINVAL, "lss_chart_interp: null argument"};
    int p = 0;
    while ((p + 1) * (p + 2) / 2 < np) ++p;
    if ((p + 1) * (p + 2) / 2 != np) throw Error{LSS_EINVAL, "lss_chart_interp: np is not (p+1)(p+2)/2"};
    if ((int64_t)c.ntris * ne > (int64_t)INT32_MAX * 64) throw Error{LSS_EINVAL, "lss_chart_interp: too many outputs"};
    const bool dev = flags & LSS_PTR_DEVICE;
    std::vector<double> nuv(2 * (size_t)np), euv(2 * (size_t)ne);
    LSS_HIP(hipMemcpy(nuv.data(), chart_uv, sizeof(double) * nuv.size(), dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    LSS_HIP(hipMemcpy(euv.data(), eval_uv, sizeof(double) * euv.size(), dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    // V^T I^T = E^T: LU with partial pivoting of V^T (np x np), ne right-hand sides
    std::vector<double> A((size_t)np * np), B((size_t)np * ne), row(np);
    for (int i = 0; i < np; ++i) {
        koornwinder(nuv[2 * i], nuv[2 * i + 1], p, row.data());
        for (int k = 0; k < np; ++k) A[(size_t)k * np + i] = row[k];          // A = V^T
    }
    for (int e = 0; e < ne; ++e) {
        koornwinder(euv[2 * e], euv[2 * e + 1], p, row.data());
        for (int k = 0; k < np; ++k) B[(size_t)k * ne + e] = row[k];          // B = E^T
    }
    double amax = 0.0;
    for (double a : A) amax = std::fmax(amax, std::fabs(a));
    for (int col = 0; col < np; ++col) {
        int piv = col;
        for (int r = col + 1; r < np; ++r)
            if (std::fabs(A[(size_t)r * np + col]) > std::fabs(A[(size_t)piv * np + col])) piv = r;
        if (!(std::fabs(A[(size_t)piv * np + col]) > 1e-13 * amax))
            throw Error{LSS_EINVAL, "lss_chart_interp: the chart nodes are not unisolvent for degree p"};
        if (piv != col) {
            for (int k = 0; k < np; ++k) std::swap(A[(size_t)col * np + k], A[(size_t)piv * np + k]);
            for (int e = 0; e < ne; ++e) std::swap(B[(size_t)col * ne + e], B[(size_t)piv * ne + e]);
        }
        for (int r = col + 1; r < np; ++r) {
            const double m = A[(size_t)r * np + col] / A[(size_t)col * np + col];
            if (m == 0.0) continue;
            for (int k = col; k < np; ++k) A[(size_t)r * np + k] -= m * A[(size_t)col * np + k];
            for (int e = 0; e < ne; ++e) B[(size_t)r * ne + e] -= m * B[(size_t)col * ne + e];
        }
    }
    std::vector<double> I((size_t)np * ne);                                    // I^T, node-major: I[i][e]
    for (int e = 0; e < ne; ++e)
        for (int r = np - 1; r >= 0; --r) {
            double s = B[(size_t)r * ne + e];
            for (int k = r + 1; k < np; ++k) s -= A[(size_t)r * np + k] * I[(size_t)k * ne + e];
            I[(size_t)r * ne + e] = s / A[(size_t)r * np + r];
        }
    const int64_t nin = c.ntris * (int64_t)np * ncomp, nout = c.ntris * (int64_t)ne * ncomp;
    DBuf dI, df, dout;
    dI.ensure(sizeof(double) * I.size());
    LSS_HIP(hipMemcpyAsync(dI.p, I.data(), sizeof(double) * I.size(), hipMemcpyHostToDevice, c.stream));
    const double *pf = f;
    double *po = out;
    if (!dev) {
        df.ensure(sizeof(double) * nin);
        LSS_HIP(hipMemcpyAsync(df.p, f, sizeof(double) * nin, hipMemcpyHostToDevice, c.stream));
        pf = df.as<double>();
        dout.ensure(sizeof(double) * nout);
        po = dout.as<double>();
    }
    const int64_t nthr = c.ntris * (int64_t)ne;
    const int32_t tpb = 256 / ne + 2;                         // triangles touched by 256 consecutive outputs
    const size_t lds = sizeof(double) * (I.size() + (size_t)tpb * np * ncomp);
    if (nthr > 0 && lds <= 60 * 1024) {
        const int64_t blocks = ceil_div(nthr, 256);
        hipLaunchKernelGGL(k_chart_interp_lds, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), lds,
                           c.stream, c.ntris, np, ne, ncomp, tpb, dI.as<double>(), pf, po);
        LSS_CHECK_LAUNCH("k_chart_interp_lds");
    } else if (nthr > 0) {
        hipLaunchKernelGGL(k_chart_interp, dim3((unsigned)ceil_div(nthr, 256)), dim3(256), 0, c.stream, c.ntris, np, ne,
                           ncomp, dI.as<double>(), pf, po);
        LSS_CHECK_LAUNCH("k_chart_interp");
    }
    if (!dev) LSS_HIP(hipMemcpyAsync(out, po, sizeof(double) * nout, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));                // the temporaries are freed on return
}

}  // namespace lss
