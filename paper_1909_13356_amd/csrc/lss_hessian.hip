// Direct-sum kernels beyond Phi / grad Phi with per-source widths: the
// Hessian of the smoothed indicator and the second derivatives of the charts
// (section 3.1, eq. uu_vector, uu_vector_aux1, uu_vector_aux2 and their uv,
// vv analogues), and Phi / grad Phi with the target-attached width sigma(x)
// (section 2, eq. basemodelk, convkernel, sigma2).
//
// Per source node (y, a' = c w J, s2 = 1/(2 sigma^2), c = 1/(4 sqrt2 pi^1.5
// sigma^3)) and target x, d = x - y, t = |d|^2 s2, the radial functions
// k1 = K/c, k2 = F/c, k3 = G/c come from radial3 (radial_exact.h).
// Each pair is accumulated by pair_hess (radial_exact.h).
// Every pair uses the full kernel (no cut, no far-field expansion).
#include <climits>

#include "lss_internal.h"
#include "radial_exact.h"
#include "chart_frame.h"

namespace lss {
namespace {

inline unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

// One thread per target.  The block walks the union of its targets' node
// ranges in tiles of 256 records staged in LDS (every lane then reads the
// same record: a broadcast); each thread sums the part of a tile that lies
// in its own mesh's range.  Targets grouped by mesh keep the union to one
// mesh (two at a boundary block).
__global__ void __launch_bounds__(256) k_hessian_direct(int64_t n, const double *__restrict__ x,
                                                        const int32_t *__restrict__ xm,
                                                        const int64_t *__restrict__ node_off,
                                                        const Src *__restrict__ src, double *phi, double *grad,
                                                        double *hess) {
    __shared__ Src tile[256];
    __shared__ long long blo, bhi;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    int64_t j0 = 0, j1 = 0;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (act) {
        const int32_t m = xm ? xm[i] : 0;
        j0 = node_off[m];
        j1 = node_off[m + 1];
        px = x[3 * i];
        py = x[3 * i + 1];
        pz = x[3 * i + 2];
    }
    if (threadIdx.x == 0) {
        blo = LLONG_MAX;
        bhi = 0;
    }
    __syncthreads();
    if (act && j1 > j0) {
        atomicMin(&blo, (long long)j0);
        atomicMax(&bhi, (long long)j1);
    }
    __syncthreads();
    const int64_t lo = blo, hi = bhi;
    HessAcc A;
    for (int64_t base = lo; base < hi; base += 256) {
        __syncthreads();
        if (base + threadIdx.x < hi) tile[threadIdx.x] = src[base + threadIdx.x];
        __syncthreads();
        const int64_t k0 = j0 > base ? j0 - base : 0;
        const int64_t k1 = (j1 - base < 256) ? j1 - base : 256;
        for (int64_t k = k0; k < k1; ++k) pair_hess(tile[k], px, py, pz, A);
    }
    if (!act) return;
    if (phi) phi[i] = A.f;
    if (grad) {
        grad[3 * i] = A.gx;
        grad[3 * i + 1] = A.gy;
        grad[3 * i + 2] = A.gz;
    }
    double *o = hess + 6 * i;
    o[0] = A.hxx;
    o[1] = A.hxy;
    o[2] = A.hxz;
    o[3] = A.hyy;
    o[4] = A.hyz;
    o[5] = A.hzz;
}

// Bounding box (lo xyz, hi xyz) of every run of 256 consecutive centroids.
__global__ void k_cen_boxes(int64_t ntris, const Cen *__restrict__ cen, double *__restrict__ box) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t * 256 >= ntris) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t e = (t + 1) * 256 < ntris ? (t + 1) * 256 : ntris;
    for (int64_t j = t * 256; j < e; ++j) {
        const double p[3] = {cen[j].cx, cen[j].cy, cen[j].cz};
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], p[d]);
            hi[d] = fmax(hi[d], p[d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        box[6 * t + d] = lo[d];
        box[6 * t + 3 + d] = hi[d];
    }
}

// sigma(x) and grad sigma of one target (phase 1 of the multiscale sums).
// The centroids come in runs of 256 (run r = [256 r, 256 r + 256)) with
// bounding boxes.  A first pass bounds the nearest centroid's squared
// distance from above by the farthest corner distance of each run that
// meets the target's range [j0, j1); a run whose nearest box distance exceeds
// that bound by 100 sigma0^2 carries weights below e^-50 of the largest and
// is skipped, and so is any single centroid that far.  The workgroup stages a run in LDS when any of its targets
// needs it; the sums are taken relative to the nearest centroid seen so far
// (rescaled when it changes).  Returns false (sigma = 0.5, grad = 0) for an
// empty range.  Every thread of the workgroup must call it.
__device__ bool sigma_phase(const Cen *__restrict__ cen, const double *__restrict__ box, Cen *ctile, long long *blo,
                            long long *bhi, int64_t j0, int64_t j1, double px, double py, double pz, double s0,
                            double &sg, double gs[3]) {
    if (threadIdx.x == 0) {
        *blo = LLONG_MAX;
        *bhi = 0;
    }
    __syncthreads();
    if (j1 > j0) {
        atomicMin(blo, (long long)j0);
        atomicMax(bhi, (long long)j1);
    }
    __syncthreads();
    const int64_t lo = *blo, hi = *bhi;
    const double inv2s0 = 0.5 / (s0 * s0);
    const double p[3] = {px, py, pz};
    const int64_t r0 = lo / 256, r1 = hi > lo ? (hi + 255) / 256 : r0;
    double dref = INFINITY;                       // >= squared distance of the nearest centroid
    for (int64_t r = r0; r < r1; ++r) {
        if (!(j0 < (r + 1) * 256 && j1 > r * 256)) continue;
        double far2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double a = fmax(fabs(p[d] - box[6 * r + d]), fabs(p[d] - box[6 * r + 3 + d]));
            far2 += a * a;
        }
        dref = fmin(dref, far2);
    }
    double dmin = INFINITY, S0 = 0.0, S1 = 0.0, V0x = 0.0, V0y = 0.0, V0z = 0.0, V1x = 0.0, V1y = 0.0, V1z = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        bool need = j0 < (r + 1) * 256 && j1 > r * 256;
        if (need) {
            double near2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double a = fmax(fmax(box[6 * r + d] - p[d], p[d] - box[6 * r + 3 + d]), 0.0);
                near2 += a * a;
            }
            need = (near2 - dref) * inv2s0 <= 50.0;
        }
        if (!__syncthreads_or(need)) continue;      // uniform: no target of the workgroup needs the run
        const int64_t b = r * 256;
        const int64_t j = b + threadIdx.x;
        if (j >= lo && j < hi) ctile[threadIdx.x] = cen[j];
        __syncthreads();
        if (need) {
            const int64_t k0 = j0 > b ? j0 - b : 0;
            const int64_t k1 = (j1 - b < 256) ? j1 - b : 256;
            for (int64_t k = k0; k < k1; ++k) {
                const Cen c = ctile[k];
                const double dx = px - c.cx, dy = py - c.cy, dz = pz - c.cz;
                const double d2 = dx * dx + dy * dy + dz * dz;
                if ((d2 - dref) * inv2s0 > 50.0) continue;   // weight below e^-50 of the nearest
                if (d2 < dmin) {          // new nearest centroid: rescale the sums to it
                    const double f = exp((d2 - dmin) * inv2s0);
                    S0 *= f;
                    S1 *= f;
                    V0x *= f;
                    V0y *= f;
                    V0z *= f;
                    V1x *= f;
                    V1y *= f;
                    V1z *= f;
                    dmin = d2;
                }
                const double w = exp((dmin - d2) * inv2s0);
                const double sw = c.sj * w;
                S0 += w;
                S1 += sw;
                V0x += w * dx;
                V0y += w * dy;
                V0z += w * dz;
                V1x += sw * dx;
                V1y += sw * dy;
                V1z += sw * dz;
            }
        }
        __syncthreads();                  // the run's LDS copy is consumed
    }
    const bool have = S0 > 0.0;
    sg = have ? S1 / S0 : 0.5;
    const double gsc = have ? -1.0 / (s0 * s0 * S0) : 0.0;
    gs[0] = gsc * (V1x - sg * V0x);
    gs[1] = gsc * (V1y - sg * V0y);
    gs[2] = gsc * (V1z - sg * V0z);
    return have;
}

// sigma(x) and grad sigma alone (the octree path of the multiscale sums)
__global__ void __launch_bounds__(256) k_sigma_field(int64_t n, const double *__restrict__ x,
                                                     const int32_t *__restrict__ xm,
                                                     const int64_t *__restrict__ tri_off,
                                                     const Cen *__restrict__ cen,
                                                     const double *__restrict__ cbox,
                                                     const double *__restrict__ sigma0, double *sig,
                                                     double *gsig) {
    __shared__ Cen ctile[256];
    __shared__ long long blo, bhi;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    int32_t m = 0;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (act) {
        m = xm ? xm[i] : 0;
        px = x[3 * i];
        py = x[3 * i + 1];
        pz = x[3 * i + 2];
    }
    const int64_t j0 = act ? tri_off[m] : 0, j1 = act ? tri_off[m + 1] : 0;
    double sg, gs[3];
    const bool have = sigma_phase(cen, cbox, ctile, &blo, &bhi, j0, j1, px, py, pz, act ? sigma0[m] : 1.0, sg, gs);
    if (!act) return;
    sig[i] = have ? sg : NAN;
    gsig[3 * i] = gs[0];
    gsig[3 * i + 1] = gs[1];
    gsig[3 * i + 2] = gs[2];
}

// Target-attached width (section 2, eq. basemodelk, convkernel, sigma2).
// Phase 1: sigma(x) = sum_j sigma_j w_j / sum_j w_j over the centroids of the
// target's mesh, w_j = exp(-|x - c_j|^2 / (2 sigma0^2)), accumulated relative
// to the nearest centroid seen so far (the sums are rescaled when it
// changes), and grad sigma = -(V1 - sigma V0) / (sigma0^2 S0) with
// S0 = sum w_j, V0 = sum w_j (x - c_j), V1 = sum sigma_j w_j (x - c_j).
// Phase 2: every node of the mesh with the raw normal a = w J and the
// target's width, c = 1/(4 sqrt2 pi^1.5 sigma^3), s2 = 1/(2 sigma^2):
//   Phi = -c sum (a.d) k1,  grad Phi = -c sum (a k1 + (a.d) k2 d)
//         + (dPhi/dsigma) grad sigma,  dPhi/dsigma = (2c/sigma) sum (a.d) exp(-t),
// k1, k2 as in radial3 (K = c k1, F = c k2).  A target whose mesh has no
// triangles gets sigma = NaN and Phi = grad Phi = 0.
__global__ void __launch_bounds__(256) k_eval_multiscale(int64_t n, const double *__restrict__ x,
                                                         const int32_t *__restrict__ xm,
                                                         const int64_t *__restrict__ tri_off,
                                                         const int64_t *__restrict__ node_off,
                                                         const Cen *__restrict__ cen,
                                                         const double *__restrict__ cbox,
                                                         const RawNode *__restrict__ nodes,
                                                         const double *__restrict__ sigma0, double *phi,
                                                         double *grad, double *sig_out) {
    __shared__ RawNode tile[256];
    __shared__ long long blo, bhi;
    Cen *ctile = reinterpret_cast<Cen *>(tile);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n;
    int32_t m = 0;
    double px = 0.0, py = 0.0, pz = 0.0;
    if (act) {
        m = xm ? xm[i] : 0;
        px = x[3 * i];
        py = x[3 * i + 1];
        pz = x[3 * i + 2];
    }
    // ---- phase 1: sigma(x) and its gradient
    int64_t j0 = act ? tri_off[m] : 0, j1 = act ? tri_off[m + 1] : 0;
    double sg, gs[3];
    const bool have = sigma_phase(cen, cbox, ctile, &blo, &bhi, j0, j1, px, py, pz, act ? sigma0[m] : 1.0, sg, gs);
    const double gsx = gs[0], gsy = gs[1], gsz = gs[2];
    int64_t lo, hi;
    // ---- phase 2: Phi, grad Phi with width sigma(x)
    j0 = act ? node_off[m] : 0;
    j1 = act ? node_off[m + 1] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        blo = LLONG_MAX;
        bhi = 0;
    }
    __syncthreads();
    if (j1 > j0) {
        atomicMin(&blo, (long long)j0);
        atomicMax(&bhi, (long long)j1);
    }
    __syncthreads();
    lo = blo;
    hi = bhi;
    const double s2 = 0.5 / (sg * sg);
    double P = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0, E = 0.0;
    for (int64_t base = lo; base < hi; base += 256) {
        __syncthreads();
        if (base + threadIdx.x < hi) tile[threadIdx.x] = nodes[base + threadIdx.x];
        __syncthreads();
        const int64_t k0 = j0 > base ? j0 - base : 0;
        const int64_t k1 = (j1 - base < 256) ? j1 - base : 256;
        for (int64_t k = k0; k < k1; ++k) {
            const RawNode s = tile[k];
            const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
            const double t = (dx * dx + dy * dy + dz * dz) * s2;
            double r1, r2, r3, et;
            radial3(t, s2, r1, r2, r3, et);
            const double ad = s.ax * dx + s.ay * dy + s.az * dz;
            P += ad * r1;
            const double adr2 = ad * r2;
            Gx += s.ax * r1 + adr2 * dx;
            Gy += s.ay * r1 + adr2 * dy;
            Gz += s.az * r1 + adr2 * dz;
            E += ad * et;
        }
    }
    if (!act) return;
    if (!have) {
        phi[i] = 0.0;
        if (grad) grad[3 * i] = grad[3 * i + 1] = grad[3 * i + 2] = 0.0;
        if (sig_out) sig_out[i] = NAN;
        return;
    }
    const double c = 1.0 / (4.0 * 1.4142135623730951 * 5.568327996831708 * sg * sg * sg);   // pi^1.5
    const double dps = 2.0 * c / sg * E;
    phi[i] = -c * P;
    if (grad) {
        grad[3 * i] = -c * Gx + dps * gsx;
        grad[3 * i + 1] = -c * Gy + dps * gsy;
        grad[3 * i + 2] = -c * Gz + dps * gsz;
    }
    if (sig_out) sig_out[i] = sg;
}

// Second derivatives and curvatures of chart j at node i (index q = j np + i).
// H is linear on the corner triangle (H_uu = 0); T is linear too, or with
// curved charts the quadratic patch with constant T_uu, T_uv, T_vv.  With
// w_u = x_u, w_v = x_v, g = grad Phi, B = the Hessian, D = g . H:
//   h_uu = -(w_u B w_u + 2 h_u g.H_u + g.T_uu) / D,
//   h_uv = -(w_u B w_v + g.(h_u H_v + h_v H_u) + g.T_uv) / D,
//   h_vv = -(w_v B w_v + 2 h_v g.H_v + g.T_vv) / D,
//   x_uu = T_uu + 2 h_u H_u + h_uu H,  x_uv = T_uv + h_u H_v + h_v H_u + h_uv H,
//   x_vv = T_vv + 2 h_v H_v + h_vv H.
// Curvatures from the fundamental forms with the outward normal n = -g/|g|:
//   Gaussian (LN - M^2)/(EG - F^2), mean -(EN - 2FM + GL)/(2(EG - F^2)).
__global__ void k_chart_curvature(int64_t N, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                                  const int32_t *__restrict__ tris6, const double *__restrict__ vH,
                                  const double *__restrict__ uv, int32_t np, const double *__restrict__ h,
                                  const double *__restrict__ grad, const double *__restrict__ hess, double *xuu,
                                  double *xuv, double *xvv, double *gauss, double *mean) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    ChartFrame f;
    int64_t j;
    chart_frame(verts, tris, tris6, vH, uv, np, q, f, j);
    const double *H = f.H, *Tu = f.Tu, *Tv = f.Tv, *Hu = f.Hu, *Hv = f.Hv;
    double g[3];
    for (int c = 0; c < 3; ++c) g[c] = grad[3 * q + c];
    const double *b = hess + 6 * q;
    const double B[3][3] = {{b[0], b[1], b[2]}, {b[1], b[3], b[4]}, {b[2], b[4], b[5]}};
    const double hq = h[q];
    const double D = H[0] * g[0] + H[1] * g[1] + H[2] * g[2];
    double au[3], av[3];
    for (int c = 0; c < 3; ++c) {
        au[c] = Tu[c] + hq * Hu[c];
        av[c] = Tv[c] + hq * Hv[c];
    }
    const double hu = -(au[0] * g[0] + au[1] * g[1] + au[2] * g[2]) / D;
    const double hv = -(av[0] * g[0] + av[1] * g[1] + av[2] * g[2]) / D;
    double wu[3], wv[3], Bwu[3], Bwv[3];
    for (int c = 0; c < 3; ++c) {
        wu[c] = au[c] + hu * H[c];
        wv[c] = av[c] + hv * H[c];
    }
    for (int r = 0; r < 3; ++r) {
        Bwu[r] = B[r][0] * wu[0] + B[r][1] * wu[1] + B[r][2] * wu[2];
        Bwv[r] = B[r][0] * wv[0] + B[r][1] * wv[1] + B[r][2] * wv[2];
    }
    const double uBu = wu[0] * Bwu[0] + wu[1] * Bwu[1] + wu[2] * Bwu[2];
    const double uBv = wu[0] * Bwv[0] + wu[1] * Bwv[1] + wu[2] * Bwv[2];
    const double vBv = wv[0] * Bwv[0] + wv[1] * Bwv[1] + wv[2] * Bwv[2];
    const double gHu = g[0] * Hu[0] + g[1] * Hu[1] + g[2] * Hu[2];
    const double gHv = g[0] * Hv[0] + g[1] * Hv[1] + g[2] * Hv[2];
    const double gTuu = g[0] * f.Tuu[0] + g[1] * f.Tuu[1] + g[2] * f.Tuu[2];
    const double gTuv = g[0] * f.Tuv[0] + g[1] * f.Tuv[1] + g[2] * f.Tuv[2];
    const double gTvv = g[0] * f.Tvv[0] + g[1] * f.Tvv[1] + g[2] * f.Tvv[2];
    const double huu = -(uBu + 2.0 * hu * gHu + gTuu) / D;
    const double huv = -(uBv + hu * gHv + hv * gHu + gTuv) / D;
    const double hvv = -(vBv + 2.0 * hv * gHv + gTvv) / D;
    double a[3], m[3], e[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = f.Tuu[c] + 2.0 * hu * Hu[c] + huu * H[c];
        m[c] = f.Tuv[c] + hu * Hv[c] + hv * Hu[c] + huv * H[c];
        e[c] = f.Tvv[c] + 2.0 * hv * Hv[c] + hvv * H[c];
    }
    if (xuu)
        for (int c = 0; c < 3; ++c) xuu[3 * q + c] = a[c];
    if (xuv)
        for (int c = 0; c < 3; ++c) xuv[3 * q + c] = m[c];
    if (xvv)
        for (int c = 0; c < 3; ++c) xvv[3 * q + c] = e[c];
    if (gauss || mean) {
        const double ig = -1.0 / sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double nn[3];
        for (int c = 0; c < 3; ++c) nn[c] = g[c] * ig;
        const double E = wu[0] * wu[0] + wu[1] * wu[1] + wu[2] * wu[2];
        const double F = wu[0] * wv[0] + wu[1] * wv[1] + wu[2] * wv[2];
        const double G = wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2];
        const double L = a[0] * nn[0] + a[1] * nn[1] + a[2] * nn[2];
        const double M = m[0] * nn[0] + m[1] * nn[1] + m[2] * nn[2];
        const double Nn = e[0] * nn[0] + e[1] * nn[1] + e[2] * nn[2];
        const double det = E * G - F * F;
        if (gauss) gauss[q] = (L * Nn - M * M) / det;
        if (mean) mean[q] = -(E * Nn - 2.0 * F * M + G * L) / (2.0 * det);
    }
}

}  // namespace

void launch_hessian_direct(Ctx &c, int64_t n, const double *x, const int32_t *xm, double *phi, double *grad,
                           double *hess) {
    hipLaunchKernelGGL(k_hessian_direct, dim3(blocks256(n)), dim3(256), 0, c.stream, n, x, xm,
                       c.node_off.as<int64_t>(), c.src.as<Src>(), phi, grad, hess);
    LSS_CHECK_LAUNCH("k_hessian_direct");
}

void launch_cen_boxes(Ctx &c, const Cen *cen, double *box) {
    const int64_t runs = (c.ntris + 255) / 256;
    hipLaunchKernelGGL(k_cen_boxes, dim3(blocks256(runs)), dim3(256), 0, c.stream, c.ntris, cen, box);
    LSS_CHECK_LAUNCH("k_cen_boxes");
}

void launch_sigma_field(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen, const double *cbox,
                        const double *sigma0, double *sig, double *gsig) {
    hipLaunchKernelGGL(k_sigma_field, dim3(blocks256(n)), dim3(256), 0, c.stream, n, x, xm, c.tri_off.as<int64_t>(),
                       cen, cbox, sigma0, sig, gsig);
    LSS_CHECK_LAUNCH("k_sigma_field");
}

void launch_eval_multiscale(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen,
                            const double *cbox, const RawNode *nodes, const double *sigma0, double *phi,
                            double *grad, double *sig) {
    hipLaunchKernelGGL(k_eval_multiscale, dim3(blocks256(n)), dim3(256), 0, c.stream, n, x, xm,
                       c.tri_off.as<int64_t>(), c.node_off.as<int64_t>(), cen, cbox, nodes, sigma0, phi, grad, sig);
    LSS_CHECK_LAUNCH("k_eval_multiscale");
}

void launch_chart_curvature(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, const double *grad,
                            const double *hess, double *xuu, double *xuv, double *xvv, double *gauss,
                            double *mean) {
    hipLaunchKernelGGL(k_chart_curvature, dim3(blocks256(N)), dim3(256), 0, c.stream, N, c.verts.as<double>(),
                       c.tris.as<int32_t>(), chart_tris6(c), c.vH.as<double>(), uv, np, h, grad, hess, xuu, xuv, xvv, gauss,
                       mean);
    LSS_CHECK_LAUNCH("k_chart_curvature");
}

}  // namespace lss
