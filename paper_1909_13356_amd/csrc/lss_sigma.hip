// Target-attached width sigma(x) by interpolation (section 2, eq. sigma2).
//
// For the points of mesh m, sigma(x) = S1 / S0 and grad sigma =
// -(V1 - sigma V0) / (sigma0^2 S0) with the weight sums
//   S0 = sum_j w_j,  S1 = sum_j sigma_j w_j,  V0 = sum_j w_j (x - c_j),
//   V1 = sum_j sigma_j w_j (x - c_j),  w_j = exp(-|x - c_j|^2 / (2 sigma0^2))
// over the centroids c_j of the mesh.  Every sum is a Gaussian convolution of
// width sigma0, hence entire in x: on a cube of side 1.5 sigma0 its tensor
// Chebyshev interpolant with 17 points per axis is exact to below the
// rounding of the sum itself.  The points are binned into such cells on a
// per-mesh grid (origin 3 sigma0 below the centroids' bounding box); the
// eight sums are formed by the direct FP64 sum at the 17^3 Chebyshev points of
// each occupied cell, scaled by exp(d_ref / (2 sigma0^2)) with d_ref the
// squared distance from the cell centre to the nearest centroid (so that
// neither overflow nor underflow occurs), and interpolated at the points by
// the barycentric formula.  Points outside the grid, in cells farther than 3
// sigma0 from every centroid, or of a mesh whose grid would exceed 1024 cells
// per axis take the direct sum.
#include <cmath>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "lss_internal.h"

namespace lss {

namespace {

constexpr int kQ = 17;                          // Chebyshev points per axis
constexpr int kQ2 = kQ * kQ;
constexpr int kQ3 = kQ * kQ * kQ;
constexpr int kNv = 8;                          // S0, S1, V0 (3), V1 (3)
constexpr double kSide = 1.5;                   // cell side / sigma0
constexpr double kPad = 3.0;                    // grid margin / sigma0
constexpr double kRefMax = 3.0;                 // cells beyond this / sigma0: direct sum
constexpr int kAxisMax = 1024;                  // cells per axis (10-bit coordinates)
constexpr int64_t kMaxNodes = int64_t(1) << 24; // node storage cap (1 GiB)

struct SigGrid {
    double o[3];      // grid origin
    double h;         // cell side
    double s0;        // sigma0 of the mesh
    int32_t nc[3];    // cells per axis
    int32_t ok;       // 0: the mesh takes the direct sum
};

// Chebyshev point k of the second kind on [-1, 1]
__device__ inline double cheb_z(int k) { return cos(k * (M_PI / (kQ - 1))); }

// barycentric weight of point k (alternating signs, halved at the ends)
__device__ inline double cheb_w(int k) {
    const double s = (k & 1) ? -1.0 : 1.0;
    return (k == 0 || k == kQ - 1) ? 0.5 * s : s;
}

// Lagrange basis values at t in [-1, 1] by the second barycentric formula;
// exact point hits give the unit vector.
__device__ inline void cheb_basis(double t, double L[kQ]) {
    int hit = -1;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const double d = t - cheb_z(k);
        if (d == 0.0) hit = k;
        L[k] = cheb_w(k) / d;
        s += L[k];
    }
    const double is = 1.0 / s;
#pragma unroll
    for (int k = 0; k < kQ; ++k) L[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : L[k] * is;
}

__device__ inline void decode_cell(uint64_t key, int32_t &m, int &ix, int &iy, int &iz) {
    m = (int32_t)(key >> 30);
    ix = (int)((key >> 20) & 1023);
    iy = (int)((key >> 10) & 1023);
    iz = (int)(key & 1023);
}

// per-mesh bounding box of the centroids: lo (3), hi (3); empty: +inf / -inf
__global__ void __launch_bounds__(256) k_mesh_cbox(const int64_t *__restrict__ tri_off,
                                                   const Cen *__restrict__ cen, double *out) {
    __shared__ double red[6][256];
    const int32_t m = blockIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = tri_off[m] + threadIdx.x; j < tri_off[m + 1]; j += 256) {
        const Cen c = cen[j];
        lo[0] = fmin(lo[0], c.cx);
        lo[1] = fmin(lo[1], c.cy);
        lo[2] = fmin(lo[2], c.cz);
        hi[0] = fmax(hi[0], c.cx);
        hi[1] = fmax(hi[1], c.cy);
        hi[2] = fmax(hi[2], c.cz);
    }
    for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = lo[d];
        red[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[6 * m + threadIdx.x] = red[threadIdx.x][0];
}

// cell key of each point: (mesh << 30) | (ix << 20) | (iy << 10) | iz, or
// `none` (sorts last) for points that take the direct sum
__global__ void k_sig_keys(int64_t n, const double *__restrict__ x, const int32_t *__restrict__ xm,
                           const SigGrid *__restrict__ grids, uint64_t none, uint64_t *key, int32_t *perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t m = xm ? xm[i] : 0;
    const SigGrid g = grids[m];
    uint64_t k = none;
    if (g.ok) {
        int ic[3];
        bool in = true;
        for (int d = 0; d < 3; ++d) {
            const double f = (x[3 * i + d] - g.o[d]) / g.h;
            in = in && f >= 0.0 && f < (double)g.nc[d];      // false for NaN
            ic[d] = in ? (int)floor(f) : 0;
            if (ic[d] >= g.nc[d]) ic[d] = g.nc[d] - 1;
        }
        if (in)
            k = ((uint64_t)m << 30) | ((uint64_t)ic[0] << 20) | ((uint64_t)ic[1] << 10) | (uint64_t)ic[2];
    }
    key[i] = k;
    perm[i] = (int32_t)i;
}

// cell heads of the sorted keys, positions, and the count of points with a
// cell (the first `none` position, or n)
__global__ void k_sig_heads(int64_t n, const uint64_t *__restrict__ key, uint64_t none, int32_t *flag,
                            int32_t *iota, int32_t *nvalid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = key[i];
    const uint64_t kp = i > 0 ? key[i - 1] : ~k;
    flag[i] = (k != none && k != kp) ? 1 : 0;
    iota[i] = (int32_t)i;
    if (k == none && (i == 0 || kp != none)) *nvalid = (int32_t)i;
    if (i == n - 1 && k != none) *nvalid = (int32_t)n;
}

// squared distance from each cell's centre to the nearest centroid of its mesh
__global__ void __launch_bounds__(256) k_cell_ref(const int32_t *__restrict__ heads, const uint64_t *__restrict__ key,
                                                  const SigGrid *__restrict__ grids,
                                                  const int64_t *__restrict__ tri_off, const Cen *__restrict__ cen,
                                                  double *cref) {
    __shared__ double red[256];
    const int32_t cell = blockIdx.x;
    int32_t m;
    int ic[3];
    decode_cell(key[heads[cell]], m, ic[0], ic[1], ic[2]);
    const SigGrid g = grids[m];
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = g.o[d] + (ic[d] + 0.5) * g.h;
    double best = INFINITY;
    for (int64_t j = tri_off[m] + threadIdx.x; j < tri_off[m + 1]; j += 256) {
        const Cen c = cen[j];
        const double dx = p[0] - c.cx, dy = p[1] - c.cy, dz = p[2] - c.cz;
        best = fmin(best, dx * dx + dy * dy + dz * dz);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) cref[cell] = red[0];
}

__device__ inline bool cell_far(double cref, double s0) { return !(cref <= kRefMax * kRefMax * s0 * s0); }

// the eight scaled sums at the Chebyshev points of each cell: block (x, y) =
// points [256 x, 256 x + 256) of cell y.  The weight factorises over the
// axes, exp((d_ref - |p - c|^2) / (2 sigma0^2)) = E_x[a] E_y[b] E_z[e] with
// E_x[a] = exp((d_ref - (x_a - c_x)^2) / (2 sigma0^2)) and E_y, E_z without
// d_ref, so a chunk of 64 centroids needs 64 x 3 x 17 exponentials, shared
// by the block's points, and each (point, centroid) term two products.
// Runs of 256 centroids whose box is so far from the cell that every weight
// is below e^-50 of the largest at any point of the cell are skipped.
constexpr int kCenChunk = 64;

__global__ void __launch_bounds__(256) k_cell_nodes(const int32_t *__restrict__ heads,
                                                    const uint64_t *__restrict__ key,
                                                    const SigGrid *__restrict__ grids,
                                                    const int64_t *__restrict__ tri_off,
                                                    const Cen *__restrict__ cen, const double *__restrict__ cbox,
                                                    const double *__restrict__ cref, double *nodes) {
    __shared__ Cen ctile[kCenChunk];
    __shared__ double E[kCenChunk][3 * kQ];
    const int32_t cell = blockIdx.y;
    int32_t m;
    int ic[3];
    decode_cell(key[heads[cell]], m, ic[0], ic[1], ic[2]);
    const SigGrid g = grids[m];
    const double dref = cref[cell];
    if (cell_far(dref, g.s0)) return;                     // uniform over the block
    const int node = blockIdx.x * 256 + threadIdx.x;
    const bool act = node < kQ3;
    const int a = act ? node / kQ2 : 0, b = act ? (node / kQ) % kQ : 0, e = act ? node % kQ : 0;
    double lo[3], p[3];
    for (int d = 0; d < 3; ++d) lo[d] = g.o[d] + ic[d] * g.h;
    p[0] = lo[0] + 0.5 * g.h * (1.0 + cheb_z(a));
    p[1] = lo[1] + 0.5 * g.h * (1.0 + cheb_z(b));
    p[2] = lo[2] + 0.5 * g.h * (1.0 + cheb_z(e));
    const double inv2s0 = 0.5 / (g.s0 * g.s0);
    const double R = sqrt(dref) + 0.8660254037844386 * g.h;   // every point has a centroid within R
    const double R2 = R * R;
    double S0 = 0.0, S1 = 0.0, V0x = 0.0, V0y = 0.0, V0z = 0.0, V1x = 0.0, V1y = 0.0, V1z = 0.0;
    const int64_t j0 = tri_off[m], j1 = tri_off[m + 1];
    for (int64_t r = j0 / 256; r * 256 < j1; ++r) {
        double near2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double gap = fmax(fmax(cbox[6 * r + d] - (lo[d] + g.h), lo[d] - cbox[6 * r + 3 + d]), 0.0);
            near2 += gap * gap;
        }
        if ((near2 - R2) * inv2s0 > 50.0) continue;          // uniform over the block
        for (int64_t base = r * 256; base < r * 256 + 256 && base < j1; base += kCenChunk) {
            const int64_t c0 = base > j0 ? base : j0;
            const int64_t c1 = base + kCenChunk < j1 ? base + kCenChunk : j1;
            if (c1 <= c0) continue;                          // uniform
            const int cnt = (int)(c1 - c0);
            __syncthreads();                                 // the previous chunk is consumed
            if ((int)threadIdx.x < cnt) ctile[threadIdx.x] = cen[c0 + threadIdx.x];
            __syncthreads();
            for (int it = threadIdx.x; it < cnt * 3 * kQ; it += 256) {
                const int c = it / (3 * kQ), q = it - c * 3 * kQ, ax = q / kQ, k = q - ax * kQ;
                const double pc = lo[ax] + 0.5 * g.h * (1.0 + cheb_z(k));
                const double cc = ax == 0 ? ctile[c].cx : (ax == 1 ? ctile[c].cy : ctile[c].cz);
                const double dd = pc - cc;
                E[c][q] = exp(((ax == 0 ? dref : 0.0) - dd * dd) * inv2s0);
            }
            __syncthreads();
            if (act) {
                for (int c = 0; c < cnt; ++c) {
                    const Cen cc = ctile[c];
                    const double w = E[c][a] * E[c][kQ + b] * E[c][2 * kQ + e];
                    const double sw = cc.sj * w;
                    const double dx = p[0] - cc.cx, dy = p[1] - cc.cy, dz = p[2] - cc.cz;
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
        }
    }
    if (!act) return;
    double *o = nodes + ((int64_t)cell * kQ3 + node) * kNv;
    o[0] = S0;
    o[1] = S1;
    o[2] = V0x;
    o[3] = V0y;
    o[4] = V0z;
    o[5] = V1x;
    o[6] = V1y;
    o[7] = V1z;
}

// index of the cell holding sorted position i (heads ascending)
__device__ inline int32_t cell_of(const int32_t *__restrict__ heads, int32_t ncell, int64_t i) {
    int32_t lo = 0, hi = ncell - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (heads[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// points that take the direct sum: no cell, or a cell far from every centroid
__global__ void k_sig_exflags(int64_t n, const int32_t *__restrict__ nvalid, const int32_t *__restrict__ heads,
                              int32_t ncell, const uint64_t *__restrict__ key, const SigGrid *__restrict__ grids,
                              const double *__restrict__ cref, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = 1;
    if (i < *nvalid) {
        const int32_t c = cell_of(heads, ncell, i);
        f = cell_far(cref[c], grids[(int32_t)(key[i] >> 30)].s0) ? 1 : 0;
    }
    flag[i] = f;
}

// interpolation at the sorted points [0, nvalid): the block walks the cells
// its points fall in, staging each cell's node values in LDS one x-slab
// (17 x 17 points x 8 sums) at a time
__global__ void __launch_bounds__(256) k_sig_eval(const int32_t *__restrict__ nvalid,
                                                  const uint64_t *__restrict__ key,
                                                  const int32_t *__restrict__ perm,
                                                  const int32_t *__restrict__ heads, int32_t ncell,
                                                  const double *__restrict__ x, const SigGrid *__restrict__ grids,
                                                  const double *__restrict__ cref,
                                                  const double *__restrict__ nodes, double *sig, double *gsig) {
    __shared__ __align__(16) double slab[kQ2 * kNv];
    __shared__ int32_t crange[2];
    const int64_t nv = *nvalid;
    const int64_t b0 = (int64_t)blockIdx.x * 256;
    if (b0 >= nv) return;                                 // uniform
    const int64_t i = b0 + threadIdx.x;
    const bool act = i < nv;
    const int32_t mycell = act ? cell_of(heads, ncell, i) : -1;
    if (threadIdx.x == 0) crange[0] = mycell;
    const int64_t last = (b0 + 255 < nv ? b0 + 255 : nv - 1);
    if (i == last) crange[1] = mycell;
    __syncthreads();
    const int32_t c0 = crange[0], c1 = crange[1];
    double Ly[kQ], Lz[kQ], tx = 0.0, sx = 0.0;
    int hx = -1;
    double acc[kNv];
#pragma unroll
    for (int q = 0; q < kNv; ++q) acc[q] = 0.0;
    SigGrid g{};
    int32_t m = 0;
    double px[3] = {0.0, 0.0, 0.0};
    bool use = false;
    if (act) {
        int ic[3];
        decode_cell(key[i], m, ic[0], ic[1], ic[2]);
        g = grids[m];
        use = !cell_far(cref[mycell], g.s0);
        const int64_t oi = perm[i];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            px[d] = x[3 * oi + d];
            const double f = (px[d] - g.o[d]) / g.h - ic[d];
            t[d] = fmin(fmax(2.0 * f - 1.0, -1.0), 1.0);
        }
        tx = t[0];
        cheb_basis(t[1], Ly);
        cheb_basis(t[2], Lz);
        // x-axis basis: the sum of the barycentric terms (or an exact hit)
        for (int k = 0; k < kQ; ++k) {
            const double d = tx - cheb_z(k);
            if (d == 0.0) hx = k;
            sx += cheb_w(k) / d;
        }
    }
    for (int32_t c = c0; c <= c1; ++c) {
        const bool far = cell_far(cref[c], grids[(int32_t)(key[heads[c]] >> 30)].s0);
        if (far) continue;                                 // uniform
        const double *src = nodes + (int64_t)c * kQ3 * kNv;
        for (int a = 0; a < kQ; ++a) {
            __syncthreads();
            for (int k = threadIdx.x; k < kQ2 * kNv; k += 256) slab[k] = src[(int64_t)a * kQ2 * kNv + k];
            __syncthreads();
            if (mycell != c || !use) continue;
            double la;
            if (hx >= 0) la = (a == hx) ? 1.0 : 0.0;
            else la = cheb_w(a) / (tx - cheb_z(a)) / sx;
            double ai[kNv];
#pragma unroll
            for (int q = 0; q < kNv; ++q) ai[q] = 0.0;
            for (int b = 0; b < kQ; ++b) {
                double aj[kNv];
#pragma unroll
                for (int q = 0; q < kNv; ++q) aj[q] = 0.0;
                const double2 *row = reinterpret_cast<const double2 *>(slab + b * kQ * kNv);
#pragma unroll
                for (int e = 0; e < kQ; ++e) {
                    const double2 v0 = row[4 * e], v1 = row[4 * e + 1], v2 = row[4 * e + 2], v3 = row[4 * e + 3];
                    aj[0] += Lz[e] * v0.x;
                    aj[1] += Lz[e] * v0.y;
                    aj[2] += Lz[e] * v1.x;
                    aj[3] += Lz[e] * v1.y;
                    aj[4] += Lz[e] * v2.x;
                    aj[5] += Lz[e] * v2.y;
                    aj[6] += Lz[e] * v3.x;
                    aj[7] += Lz[e] * v3.y;
                }
#pragma unroll
                for (int q = 0; q < kNv; ++q) ai[q] += Ly[b] * aj[q];
            }
#pragma unroll
            for (int q = 0; q < kNv; ++q) acc[q] += la * ai[q];
        }
    }
    if (!act || !use) return;
    const int64_t oi = perm[i];
    const double sg = acc[1] / acc[0];
    const double gsc = -1.0 / (g.s0 * g.s0 * acc[0]);
    sig[oi] = sg;
    gsig[3 * oi] = gsc * (acc[5] - sg * acc[2]);
    gsig[3 * oi + 1] = gsc * (acc[6] - sg * acc[3]);
    gsig[3 * oi + 2] = gsc * (acc[7] - sg * acc[4]);
}

__global__ void k_sig_gather(int64_t n, const int32_t *__restrict__ idx, const double *__restrict__ x,
                             const int32_t *__restrict__ xm, double *xo, int32_t *xmo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = idx[i];
    for (int d = 0; d < 3; ++d) xo[3 * i + d] = x[3 * s + d];
    if (xm) xmo[i] = xm[s];
}

__global__ void k_sig_scatter(int64_t n, const int32_t *__restrict__ idx, const double *__restrict__ s,
                              const double *__restrict__ gs, double *sig, double *gsig) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = idx[i];
    sig[o] = s[i];
    for (int d = 0; d < 3; ++d) gsig[3 * o + d] = gs[3 * i + d];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

bool sigma_field_interp(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen, const double *cbox,
                        const double *s0_dev, const double *s0_host, double *sig, double *gsig, bool force) {
    if (n <= 0) return true;
    const int32_t nm = c.nmesh;
    // per-mesh grids
    DBuf mb, grid;
    mb.ensure(sizeof(double) * 6 * nm);
    hipLaunchKernelGGL(k_mesh_cbox, dim3(nm), dim3(256), 0, c.stream, c.tri_off.as<int64_t>(), cen,
                       mb.as<double>());
    LSS_CHECK_LAUNCH("k_mesh_cbox");
    std::vector<double> hb(6 * (size_t)nm);
    LSS_HIP(hipMemcpyAsync(hb.data(), mb.p, sizeof(double) * 6 * nm, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    std::vector<SigGrid> hg(nm);
    bool any = false;
    for (int32_t m = 0; m < nm; ++m) {
        SigGrid &g = hg[m];
        std::memset(&g, 0, sizeof(g));
        const double s0 = s0_host[m];
        g.s0 = s0 > 0.0 ? s0 : 1.0;
        g.h = kSide * g.s0;
        bool ok = s0 > 0.0 && std::isfinite(s0);
        for (int d = 0; d < 3 && ok; ++d) {
            const double lo = hb[6 * m + d], hi = hb[6 * m + 3 + d];
            if (!(hi >= lo) || !std::isfinite(lo) || !std::isfinite(hi)) { ok = false; break; }
            g.o[d] = lo - kPad * s0;
            const double cells = std::ceil((hi - lo + 2.0 * kPad * s0) / g.h);
            if (!(cells >= 1.0 && cells <= kAxisMax)) { ok = false; break; }
            g.nc[d] = (int32_t)cells;
        }
        g.ok = ok ? 1 : 0;
        any = any || ok;
    }
    if (!any) return false;
    grid.ensure(sizeof(SigGrid) * nm);
    LSS_HIP(hipMemcpyAsync(grid.p, hg.data(), sizeof(SigGrid) * nm, hipMemcpyHostToDevice, c.stream));
    // bin the points by cell
    int bits = 1;
    while ((int64_t(1) << bits) <= nm) ++bits;
    const uint64_t none = (uint64_t)nm << 30;
    DBuf key, key2, perm, perm2, flag, iota, heads, cnt;
    key.ensure(sizeof(uint64_t) * n);
    key2.ensure(sizeof(uint64_t) * n);
    perm.ensure(sizeof(int32_t) * n);
    perm2.ensure(sizeof(int32_t) * n);
    flag.ensure(sizeof(int32_t) * (n + 1));
    iota.ensure(sizeof(int32_t) * n);
    heads.ensure(sizeof(int32_t) * n);
    cnt.ensure(sizeof(int32_t) * 4);
    hipLaunchKernelGGL(k_sig_keys, dim3(blocks_for(n)), dim3(256), 0, c.stream, n, x, xm, grid.as<SigGrid>(), none,
                       key.as<uint64_t>(), perm.as<int32_t>());
    LSS_CHECK_LAUNCH("k_sig_keys");
    sort_pairs(c, key.as<uint64_t>(), key2.as<uint64_t>(), perm.as<int32_t>(), perm2.as<int32_t>(), n, 30 + bits);
    int32_t *nvalid = cnt.as<int32_t>(), *ncell_dev = cnt.as<int32_t>() + 1, *nex_dev = cnt.as<int32_t>() + 2;
    hipLaunchKernelGGL(k_sig_heads, dim3(blocks_for(n)), dim3(256), 0, c.stream, n, key2.as<uint64_t>(), none,
                       flag.as<int32_t>(), iota.as<int32_t>(), nvalid);
    LSS_CHECK_LAUNCH("k_sig_heads");
    compact_flags(c, n, nullptr, flag.as<int32_t>(), iota.as<int32_t>(), heads.as<int32_t>(), ncell_dev);
    int32_t hc[2] = {0, 0};
    LSS_HIP(hipMemcpyAsync(hc, cnt.p, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    const int32_t ncell = hc[1];
    const int64_t nnodes = (int64_t)ncell * kQ3;
    if (nnodes > kMaxNodes) return false;
    if (!force && nnodes * 4 > n) return false;
    DBuf cref, nodes;
    if (ncell > 0) {
        cref.ensure(sizeof(double) * ncell);
        nodes.ensure(sizeof(double) * kNv * nnodes);
        hipLaunchKernelGGL(k_cell_ref, dim3(ncell), dim3(256), 0, c.stream, heads.as<int32_t>(),
                           key2.as<uint64_t>(), grid.as<SigGrid>(), c.tri_off.as<int64_t>(), cen, cref.as<double>());
        LSS_CHECK_LAUNCH("k_cell_ref");
        hipLaunchKernelGGL(k_cell_nodes, dim3((kQ3 + 255) / 256, ncell), dim3(256), 0, c.stream,
                           heads.as<int32_t>(), key2.as<uint64_t>(), grid.as<SigGrid>(), c.tri_off.as<int64_t>(),
                           cen, cbox, cref.as<double>(), nodes.as<double>());
        LSS_CHECK_LAUNCH("k_cell_nodes");
        hipLaunchKernelGGL(k_sig_eval, dim3(blocks_for(hc[0])), dim3(256), 0, c.stream, nvalid,
                           key2.as<uint64_t>(), perm2.as<int32_t>(), heads.as<int32_t>(), ncell, x,
                           grid.as<SigGrid>(), cref.as<double>(), nodes.as<double>(), sig, gsig);
        LSS_CHECK_LAUNCH("k_sig_eval");
    }
    // the rest by the direct sum
    hipLaunchKernelGGL(k_sig_exflags, dim3(blocks_for(n)), dim3(256), 0, c.stream, n, nvalid, heads.as<int32_t>(),
                       ncell, key2.as<uint64_t>(), grid.as<SigGrid>(), ncell > 0 ? cref.as<double>() : nullptr,
                       flag.as<int32_t>());
    LSS_CHECK_LAUNCH("k_sig_exflags");
    compact_flags(c, n, nullptr, flag.as<int32_t>(), perm2.as<int32_t>(), iota.as<int32_t>(), nex_dev);
    int32_t nex = 0;
    LSS_HIP(hipMemcpyAsync(&nex, nex_dev, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    if (nex > 0) {
        DBuf xg, xmg, sg, gs;
        xg.ensure(sizeof(double) * 3 * nex);
        if (xm) xmg.ensure(sizeof(int32_t) * nex);
        sg.ensure(sizeof(double) * nex);
        gs.ensure(sizeof(double) * 3 * nex);
        hipLaunchKernelGGL(k_sig_gather, dim3(blocks_for(nex)), dim3(256), 0, c.stream, (int64_t)nex,
                           iota.as<int32_t>(), x, xm, xg.as<double>(), xm ? xmg.as<int32_t>() : nullptr);
        LSS_CHECK_LAUNCH("k_sig_gather");
        launch_sigma_field(c, nex, xg.as<double>(), xm ? xmg.as<int32_t>() : nullptr, cen, cbox, s0_dev,
                           sg.as<double>(), gs.as<double>());
        hipLaunchKernelGGL(k_sig_scatter, dim3(blocks_for(nex)), dim3(256), 0, c.stream, (int64_t)nex,
                           iota.as<int32_t>(), sg.as<double>(), gs.as<double>(), sig, gsig);
        LSS_CHECK_LAUNCH("k_sig_scatter");
    }
    LSS_HIP(hipStreamSynchronize(c.stream));    // the local buffers must outlive the kernels
    return true;
}

}  // namespace lss
