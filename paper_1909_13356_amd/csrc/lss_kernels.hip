// Source preparation, pseudonormals, target ordering and the Newton chart
// projection kernels of liblss (gfx950).
#include <cstring>
#include <hip/hip_runtime.h>

#include <cmath>

#include "lss_internal.h"
#include "chart_frame.h"

namespace lss {

namespace {

constexpr int kBlk = 256;

__device__ inline void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------------------ source prep
// Node k = j * nq + m of triangle j (section 4.3, eq. discrete_int with the
// parametrisation eq. tparam): y = P1 + u (P2-P1) + v (P3-P1); the
// area-weighted normal J = (P2-P1) x (P3-P1) carries N_hat da; the dipole
// vector is folded with the kernel normalisation c = 1/(4 sqrt2 pi^1.5 sigma^3)
// so that the pair kernel needs only S(x), T(x) of x = rho^2/(2 sigma^2).
// Quadrature node k = j * nq + m.  Flat triangle (eq. tparam): y = P1 + u tu
// + v tv, J = tu x tv.  Quadratic triangle (tris6 != nullptr; corners, then
// the edge points of P1P2, P2P3, P3P1): the Lagrange interpolant through the
// six points written in monomials about P1,
//   y = P1 + u (A + u C + v E) + v (B + v D),
//   A = 4 P4 - 3 P1 - P2,  B = 4 P6 - 3 P1 - P3,  C = 2 (P1 + P2 - 2 P4),
//   D = 2 (P1 + P3 - 2 P6),  E = 4 (P1 - P4 + P5 - P6),
// and J = y_u x y_v with y_u = A + 2u C + v E, y_v = B + 2v D + u E.
__device__ inline void node_yJ(const double *__restrict__ verts, const int32_t *__restrict__ tris,
                               const int32_t *__restrict__ tris6, const double *__restrict__ rule, int32_t nq,
                               int64_t k, int64_t &j, double y[3], double J[3], double &w) {
    j = k / nq;
    const int m = (int)(k - j * nq);
    const double u = rule[3 * m], v = rule[3 * m + 1];
    w = rule[3 * m + 2];
    double P1[3];
    if (tris6) {
        const int32_t *t = tris6 + 6 * j;
        double yu[3], yv[3];
        for (int c = 0; c < 3; ++c) {
            P1[c] = verts[3 * (int64_t)t[0] + c];
            const double d2 = verts[3 * (int64_t)t[1] + c] - P1[c];
            const double d3 = verts[3 * (int64_t)t[2] + c] - P1[c];
            const double d4 = verts[3 * (int64_t)t[3] + c] - P1[c];
            const double d5 = verts[3 * (int64_t)t[4] + c] - P1[c];
            const double d6 = verts[3 * (int64_t)t[5] + c] - P1[c];
            const double A = 4.0 * d4 - d2, B = 4.0 * d6 - d3;
            const double C = 2.0 * (d2 - 2.0 * d4), D = 2.0 * (d3 - 2.0 * d6);
            const double E = 4.0 * (d5 - d4 - d6);
            y[c] = P1[c] + (u * (A + u * C + v * E) + v * (B + v * D));
            yu[c] = A + 2.0 * u * C + v * E;
            yv[c] = B + 2.0 * v * D + u * E;
        }
        cross3(yu, yv, J);
    } else {
        const int32_t *t = tris + 3 * j;
        double tu[3], tv[3];
        for (int c = 0; c < 3; ++c) {
            P1[c] = verts[3 * (int64_t)t[0] + c];
            tu[c] = verts[3 * (int64_t)t[1] + c] - P1[c];
            tv[c] = verts[3 * (int64_t)t[2] + c] - P1[c];
            y[c] = P1[c] + u * tu[c] + v * tv[c];
        }
        cross3(tu, tv, J);
    }
}

__global__ void k_prep_sources(int64_t nnodes, int32_t nq, const double *__restrict__ verts,
                               const int32_t *__restrict__ tris, const int32_t *__restrict__ tris6,
                               const double *__restrict__ rule, const double *__restrict__ sigma,
                               Src *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnodes) return;
    int64_t j;
    double y[3], J[3], w;
    node_yJ(verts, tris, tris6, rule, nq, k, j, y, J, w);
    const double s = sigma[j];
    const double cnorm = 1.0 / (4.0 * 1.4142135623730951 * 5.568327996831708 * s * s * s);  // pi^1.5
    Src r;
    r.yx = y[0];
    r.yy = y[1];
    r.yz = y[2];
    r.s2 = 0.5 / (s * s);
    r.ax = cnorm * w * J[0];
    r.ay = cnorm * w * J[1];
    r.az = cnorm * w * J[2];
    r.s2x2 = 2.0 * r.s2;
    out[k] = r;
}

// the same nodes without a width: y and a = w J (for a target-attached sigma)
__global__ void k_prep_raw(int64_t nnodes, int32_t nq, const double *__restrict__ verts,
                           const int32_t *__restrict__ tris, const int32_t *__restrict__ tris6,
                           const double *__restrict__ rule, RawNode *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnodes) return;
    int64_t j;
    double y[3], J[3], w;
    node_yJ(verts, tris, tris6, rule, nq, k, j, y, J, w);
    out[k] = RawNode{y[0], y[1], y[2], w * J[0], w * J[1], w * J[2]};
}

// Centroid c_j of corner triangle j and D_j, the diameter of its smallest
// enclosing ball (section 2): the longest edge if the largest angle is at
// least 90 degrees, else the circumdiameter |AB| |BC| |CA| / |AB x AC|.
// Writes {c_j, D_j / lambda} and D_j.
__global__ void k_centroids(int64_t ntris, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                            double lambda, Cen *__restrict__ out, double *__restrict__ D) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntris) return;
    const int32_t *t = tris + 3 * j;
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) P[a][c] = verts[3 * (int64_t)t[a] + c];
    double e[3][3], l2[3];
    for (int a = 0; a < 3; ++a) {
        const int b = a == 2 ? 0 : a + 1;
        for (int c = 0; c < 3; ++c) e[a][c] = P[b][c] - P[a][c];
        l2[a] = e[a][0] * e[a][0] + e[a][1] * e[a][1] + e[a][2] * e[a][2];
    }
    const double mx = fmax(l2[0], fmax(l2[1], l2[2]));
    double d;
    if (2.0 * mx >= l2[0] + l2[1] + l2[2]) {
        d = sqrt(mx);
    } else {
        double n[3];
        cross3(e[0], e[2], n);
        d = sqrt(l2[0] * l2[1] * l2[2]) / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    }
    D[j] = d;
    out[j] = Cen{(P[0][0] + P[1][0] + P[2][0]) / 3.0, (P[0][1] + P[1][1] + P[2][1]) / 3.0,
                 (P[0][2] + P[1][2] + P[2][2]) / 3.0, d / lambda};
}

// signed volume per mesh (sum P1 . (P2 x P3) / 6) and zero-area count
__global__ void k_orientation(int64_t ntris, int32_t nmesh, const int64_t *__restrict__ tri_off,
                              const double *__restrict__ verts, const int32_t *__restrict__ tris,
                              double *vol, unsigned long long *ndegen) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntris) return;
    const int32_t *t = tris + 3 * j;
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) P[a][c] = verts[3 * (int64_t)t[a] + c];
    double x[3], e1[3], e2[3], J[3];
    cross3(P[1], P[2], x);
    double v6 = P[0][0] * x[0] + P[0][1] * x[1] + P[0][2] * x[2];
    for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
    cross3(e1, e2, J);
    if (J[0] == 0.0 && J[1] == 0.0 && J[2] == 0.0) atomicAdd(ndegen, 1ull);
    int lo = 0, hi = nmesh;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tri_off[mid] <= j) lo = mid; else hi = mid;
    }
    atomicAdd(&vol[lo], v6 / 6.0);
}

// bounding box of the nodes: block partial min/max, then one block folds
__global__ void k_bbox_partial(int64_t n, const Src *__restrict__ src, double *part) {
    __shared__ double sh[6][kBlk];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        double p[3] = {src[k].yx, src[k].yy, src[k].yz};
        for (int c = 0; c < 3; ++c) { lo[c] = fmin(lo[c], p[c]); hi[c] = fmax(hi[c], p[c]); }
    }
    for (int c = 0; c < 3; ++c) { sh[c][threadIdx.x] = lo[c]; sh[3 + c][threadIdx.x] = hi[c]; }
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; ++c) {
                sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
                sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_bbox_final(int nb, double *part) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int b = 1; b < nb; ++b)
        for (int c = 0; c < 3; ++c) {
            part[c] = fmin(part[c], part[6 * b + c]);
            part[3 + c] = fmax(part[3 + c], part[6 * b + 3 + c]);
        }
}

// ----------------------------------------------------------- pseudonormals
// Vertex pseudonormal (section 3, eq. mkvertexpn): angle-weighted mean of the
// unit normals of the incident triangles, not renormalised.  Deterministic:
// each vertex sums its incident corners in increasing corner order.
__global__ void k_corner_count(int64_t ncorner, const int32_t *__restrict__ tris, int32_t *cnt) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ncorner) atomicAdd(&cnt[tris[q]], 1);
}

__global__ void k_corner_fill(int64_t ncorner, const int32_t *__restrict__ tris,
                              const int32_t *__restrict__ off, int32_t *fill, int64_t *list) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ncorner) return;
    int32_t v = tris[q];
    int32_t slot = atomicAdd(&fill[v], 1);
    list[off[v] + slot] = q;
}

// Corner k of triangle q / 3 on a curved patch (tris6): unit normal y_u x y_v
// at the corner and the angle between the patch's two edges there (their
// tangents: y_u, y_v at P1; y_v - y_u, -y_u at P2; -y_v, y_u - y_v at P3).
__device__ void corner_contrib_curved(const double *__restrict__ verts, const int32_t *__restrict__ tris6, int64_t q,
                                      double &theta, double nh[3]) {
    const int64_t j = q / 3;
    const int k = (int)(q - 3 * j);
    double P1[3], A[3], B[3], C[3], D[3], E[3], yu[3], yv[3], p[3], r[3], N[3], cr[3];
    patch_coef(verts, tris6 + 6 * j, P1, A, B, C, D, E);
    for (int c = 0; c < 3; ++c) {
        yu[c] = A[c] + (k == 1 ? 2.0 * C[c] : (k == 2 ? E[c] : 0.0));
        yv[c] = B[c] + (k == 1 ? E[c] : (k == 2 ? 2.0 * D[c] : 0.0));
        p[c] = k == 0 ? yu[c] : (k == 1 ? yv[c] - yu[c] : -yv[c]);
        r[c] = k == 0 ? yv[c] : (k == 1 ? -yu[c] : yu[c] - yv[c]);
    }
    cross3(yu, yv, N);
    const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    if (nn == 0.0) { theta = 0.0; nh[0] = nh[1] = nh[2] = 0.0; return; }
    cross3(p, r, cr);
    theta = atan2(sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]), p[0] * r[0] + p[1] * r[1] + p[2] * r[2]);
    for (int c = 0; c < 3; ++c) nh[c] = N[c] / nn;
}

__device__ void corner_contrib(const double *__restrict__ verts, const int32_t *__restrict__ tris,
                               int64_t q, double &theta, double nh[3]) {
    int64_t j = q / 3;
    int k = (int)(q - 3 * j);
    const int32_t *t = tris + 3 * j;
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) P[a][c] = verts[3 * (int64_t)t[a] + c];
    double e1[3], e2[3], N[3], p[3], r[3], cr[3];
    for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
    cross3(e1, e2, N);
    double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    if (nn == 0.0) { theta = 0.0; nh[0] = nh[1] = nh[2] = 0.0; return; }
    for (int c = 0; c < 3; ++c) {
        p[c] = P[(k + 1) % 3][c] - P[k][c];
        r[c] = P[(k + 2) % 3][c] - P[k][c];
    }
    cross3(p, r, cr);
    theta = atan2(sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]), p[0] * r[0] + p[1] * r[1] + p[2] * r[2]);
    for (int c = 0; c < 3; ++c) nh[c] = N[c] / nn;
}

__global__ void k_vertex_H(int64_t nverts, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                           const int32_t *__restrict__ tris6, const int32_t *__restrict__ off,
                           const int32_t *__restrict__ cnt, int64_t *list, double *H) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nverts) return;
    int64_t *L = list + off[v];
    int n = cnt[v];
    for (int a = 1; a < n; ++a) {           // insertion sort: corner order fixes the sum order
        int64_t key = L[a];
        int b = a - 1;
        while (b >= 0 && L[b] > key) { L[b + 1] = L[b]; --b; }
        L[b + 1] = key;
    }
    double sx = 0, sy = 0, sz = 0, sa = 0;
    for (int a = 0; a < n; ++a) {
        double th, nh[3];
        if (tris6) corner_contrib_curved(verts, tris6, L[a], th, nh);
        else corner_contrib(verts, tris, L[a], th, nh);
        sx += th * nh[0]; sy += th * nh[1]; sz += th * nh[2]; sa += th;
    }
    double inv = sa > 0.0 ? 1.0 / sa : 0.0;
    H[3 * v] = sx * inv; H[3 * v + 1] = sy * inv; H[3 * v + 2] = sz * inv;
}

// ---------------------------------------------------------- target ordering
__device__ inline uint64_t spread16(uint64_t x) {     // 16 bits -> every third bit
    x &= 0xffffull;
    x = (x | (x << 16)) & 0x0000ff0000ffull;
    x = (x | (x << 8)) & 0x00f00f00f00full;
    x = (x | (x << 4)) & 0x0c30c30c30c3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

__device__ inline uint64_t morton_key(double x, double y, double z, const double lo[3], double inv) {
    double q[3] = {(x - lo[0]) * inv, (y - lo[1]) * inv, (z - lo[2]) * inv};
    uint64_t b[3];
    for (int c = 0; c < 3; ++c) {
        double t = q[c] * 65536.0;
        t = t != t ? 0.0 : fmin(fmax(t, 0.0), 65535.0);
        b[c] = (uint64_t)t;
    }
    return spread16(b[0]) | (spread16(b[1]) << 1) | (spread16(b[2]) << 2);
}

struct Box {
    double lo[3];
    double inv;
};

__global__ void k_target_keys(int64_t n, const double *__restrict__ x, const int32_t *__restrict__ xm,
                              int32_t nmesh, Box box, uint64_t *keys, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t m = 0;
    if (xm) {
        int32_t mm = xm[i];
        mm = mm < 0 ? 0 : (mm >= nmesh ? nmesh - 1 : mm);
        m = (uint64_t)mm;
    }
    keys[i] = (m << 48) | morton_key(x[3 * i], x[3 * i + 1], x[3 * i + 2], box.lo, box.inv);
    idx[i] = (int32_t)i;
}

__global__ void k_gather_targets(int64_t n, const double *__restrict__ x, const int32_t *__restrict__ xm,
                                 int32_t nmesh, const int32_t *__restrict__ perm, double *tx, double *ty,
                                 double *tz, int32_t *tmesh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t s = perm[i];
    tx[i] = x[3 * s];
    ty[i] = x[3 * s + 1];
    tz[i] = x[3 * s + 2];
    int32_t m = xm ? xm[s] : 0;
    tmesh[i] = m < 0 ? 0 : (m >= nmesh ? nmesh - 1 : m);
}

// -------------------------------------------------------------- Newton
__device__ inline int32_t mesh_of_tri(const int64_t *tri_off, int32_t nmesh, int64_t j) {
    int lo = 0, hi = nmesh;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tri_off[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

// chart base point T and direction H of chart node idx = j * np + i
__device__ inline void chart_TH(const double *__restrict__ verts, const int32_t *__restrict__ tris,
                                const int32_t *__restrict__ tris6, const double *__restrict__ vH,
                                const double *__restrict__ uv, int32_t np, int64_t idx, double T[3], double H[3],
                                int64_t &j) {
    ChartFrame f;
    chart_frame(verts, tris, tris6, vH, uv, np, idx, f, j);
    for (int c = 0; c < 3; ++c) {
        T[c] = f.T[c];
        H[c] = f.H[c];
    }
}

__global__ void k_chart_keys(int64_t N, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                             const int32_t *__restrict__ tris6, const double *__restrict__ vH, const double *__restrict__ uv, int32_t np,
                             const int64_t *__restrict__ tri_off, int32_t nmesh, Box box,
                             const double *__restrict__ troot, int tbits, uint64_t *keys, int32_t *idx) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    double T[3], H[3];
    int64_t j;
    chart_TH(verts, tris, tris6, vH, uv, np, q, T, H, j);
    uint64_t m = nmesh > 1 ? (uint64_t)mesh_of_tri(tri_off, nmesh, j) : 0;
    if (troot) {        // octree order: the nodes of a leaf are contiguous
        bool inside;
        keys[q] = tree_point_key(T[0], T[1], T[2], (int32_t)m, troot, tbits, inside);
    } else {
        keys[q] = (m << 48) | morton_key(T[0], T[1], T[2], box.lo, box.inv);
    }
    idx[q] = (int32_t)q;
}

enum { ST_ACTIVE = -1 };

__global__ void k_chart_init(int64_t N, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                             const int32_t *__restrict__ tris6, const double *__restrict__ vH, const double *__restrict__ uv, int32_t np,
                             const int64_t *__restrict__ tri_off, int32_t nmesh,
                             const double *__restrict__ sigma, const int32_t *__restrict__ perm,
                             double *Tout, double *Hout, double *h, double *lo, double *hi, double *sig,
                             int32_t *mesh, int32_t *orig, int8_t *status, int8_t *iters, int8_t *seen,
                             int32_t *flag) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    int64_t q = perm[s];
    double T[3], H[3];
    int64_t j;
    chart_TH(verts, tris, tris6, vH, uv, np, q, T, H, j);
    for (int c = 0; c < 3; ++c) { Tout[3 * s + c] = T[c]; Hout[3 * s + c] = H[c]; }
    double sj = sigma[j];
    double nH = sqrt(H[0] * H[0] + H[1] * H[1] + H[2] * H[2]);
    double hmax = 16.0 * sj / nH;
    h[s] = 0.0;
    lo[s] = -hmax;
    hi[s] = hmax;
    sig[s] = sj;
    mesh[s] = nmesh > 1 ? mesh_of_tri(tri_off, nmesh, j) : 0;
    orig[s] = (int32_t)q;
    iters[s] = 0;
    seen[s] = 0;
    bool degenerate = !(nH >= 1e-3);
    status[s] = degenerate ? (int8_t)LSS_NODE_DEGENERATE_H : (int8_t)ST_ACTIVE;
    flag[s] = degenerate ? 0 : 1;
}

// active node a -> evaluation point x = T + h H (eq. h)
__global__ void k_newton_targets(const int32_t *__restrict__ nact, const int32_t *__restrict__ active,
                                 const double *__restrict__ T, const double *__restrict__ H,
                                 const double *__restrict__ h, const int32_t *__restrict__ mesh,
                                 double *tx, double *ty, double *tz, int32_t *tmesh) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= *nact) return;
    int64_t s = active[a];
    double hs = h[s];
    tx[a] = T[3 * s] + hs * H[3 * s];
    ty[a] = T[3 * s + 1] + hs * H[3 * s + 1];
    tz[a] = T[3 * s + 2] + hs * H[3 * s + 2];
    tmesh[a] = mesh[s];
}

// Safeguarded Newton step (eq. newtoneq with derivative eq. newtonderiv):
// g = Phi - 1/2, g' = H . grad Phi; g > 0 raises the bracket's lower end,
// g < 0 lowers its upper end; a step outside (lo, hi), or with g' >= 0, is
// replaced by the bracket midpoint.  Converged when |dh| <= tau sigma_j.
__global__ void k_newton_update(const int32_t *__restrict__ nact, const int32_t *__restrict__ active,
                                const double *__restrict__ phi, const double *__restrict__ grad,
                                const double *__restrict__ H, double *h, double *lo, double *hi,
                                const double *__restrict__ sig, int8_t *status, int8_t *iters, int8_t *seen,
                                int32_t *flag, double tau, int32_t max_iter) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= *nact) return;
    int64_t s = active[a];
    double hs = h[s], l = lo[s], u = hi[s];
    double g = phi[a] - 0.5;
    double gp = H[3 * s] * grad[3 * a] + H[3 * s + 1] * grad[3 * a + 1] + H[3 * s + 2] * grad[3 * a + 2];
    int it = iters[s] + 1;
    int sn = seen[s];               // bit 1: g > 0 seen, bit 2: g < 0 seen
    int st = ST_ACTIVE;
    if (g > 0.0) { l = hs; sn |= 1; }
    else if (g < 0.0) { u = hs; sn |= 2; }
    else st = LSS_NODE_CONVERGED;
    if (st == ST_ACTIVE) {
        double hn = gp < 0.0 ? hs - g / gp : (double)NAN;
        const bool newton = hn > l && hn < u;
        if (!newton) hn = 0.5 * (l + u);
        double dh = hn - hs;
        hs = hn;
        const double hmax = 16.0 * sig[s] / sqrt(H[3 * s] * H[3 * s] + H[3 * s + 1] * H[3 * s + 1] + H[3 * s + 2] * H[3 * s + 2]);
        // a bisection step into the outer quarter of the search range without
        // a sign change of g: no root near the skeleton
        if (!newton && sn != 3 && fabs(hs) > 0.75 * hmax) st = LSS_NODE_NOBRACKET;
        else if (fabs(dh) <= tau * sig[s]) st = LSS_NODE_CONVERGED;
        else if (it >= max_iter) st = fabs(hs) > 0.5 * hmax ? LSS_NODE_NOBRACKET : LSS_NODE_MAXITER;
    }
    h[s] = hs;
    lo[s] = l;
    hi[s] = u;
    iters[s] = (int8_t)it;
    seen[s] = (int8_t)sn;
    status[s] = (int8_t)st;
    flag[a] = st == ST_ACTIVE ? 1 : 0;
}

// Order-preserving compaction of list[0..n) by flag (n on the device):
// per-block counts, one-block scan of the counts, per-block scatter.
constexpr int kCompBlk = 1024;

__global__ void k_block_count(const int32_t *__restrict__ n_dev, const int32_t *__restrict__ flag, int32_t *bsum) {
    __shared__ int32_t sh[kCompBlk / 64];
    int64_t n = *n_dev;
    int64_t i = (int64_t)blockIdx.x * kCompBlk + threadIdx.x;
    int f = (i < n) ? flag[i] : 0;
    unsigned long long b = __ballot(f);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kCompBlk / 64; ++w) t += sh[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ void k_scan_blocks(int32_t nb, int32_t *bsum, int32_t *n_out) {
    // single block: exclusive scan in place, total to *n_out
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nb; base += kCompBlk) {
        __shared__ int32_t sh[kCompBlk];
        int32_t i = base + threadIdx.x;
        int32_t v = i < nb ? bsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kCompBlk; off <<= 1) {
            int32_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kCompBlk - 1) carry += sh[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = carry;
}

__global__ void k_block_scatter(const int32_t *__restrict__ n_dev, const int32_t *__restrict__ flag,
                                const int32_t *__restrict__ bsum, const int32_t *__restrict__ in,
                                int32_t *out) {
    __shared__ int32_t sh[kCompBlk / 64];
    int64_t n = *n_dev;
    int64_t i = (int64_t)blockIdx.x * kCompBlk + threadIdx.x;
    int f = (i < n) ? flag[i] : 0;
    unsigned long long b = __ballot(f);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = __popcll(b);
    __syncthreads();
    int32_t pre = bsum[blockIdx.x];
    for (int q = 0; q < w; ++q) pre += sh[q];
    pre += __popcll(b & ((1ull << lane) - 1ull));
    if (f) out[pre] = in[i];
}

// start of a Newton iteration: the active count becomes the input count of
// this iteration's compaction; a non-empty iteration is counted (nact[3]) and
// its count recorded in hist (capacity cap)
__global__ void k_iter_mark(int32_t *nact, int32_t *hist, int32_t cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int32_t n = nact[0];
        nact[1] = n;
        if (n > 0 && nact[3] < cap) {
            hist[nact[3]] = n;
            nact[3] += 1;
        }
    }
}

__global__ void k_copy_active(const int32_t *__restrict__ n_dev, const int32_t *__restrict__ in, int32_t *out) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < *n_dev) out[a] = in[a];
}

__global__ void k_iota(int64_t n, int32_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)i;
}

__global__ void k_newton_output(int64_t N, const int32_t *__restrict__ orig, const double *__restrict__ T,
                                const double *__restrict__ H, const double *__restrict__ h,
                                const int8_t *__restrict__ status, const int8_t *__restrict__ iters,
                                double *h_out, double *x_out, int8_t *st_out, int8_t *it_out) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    int64_t q = orig[s];
    double hs = h[s];
    if (h_out) h_out[q] = hs;
    if (x_out)
        for (int c = 0; c < 3; ++c) x_out[3 * q + c] = T[3 * s + c] + hs * H[3 * s + c];
    int8_t st = status[s];
    if (st_out) st_out[q] = st < 0 ? (int8_t)LSS_NODE_MAXITER : st;
    if (it_out) it_out[q] = iters[s];
}

inline unsigned grid_for(int64_t n, int blk = kBlk) { return (unsigned)ceil_div(n > 0 ? n : 1, blk); }

Box make_box(const Ctx &c) {
    Box b;
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = fmax(ext, c.bbox_hi[k] - c.bbox_lo[k]);
    ext = ext > 0 ? ext * 1.5 : 1.0;
    for (int k = 0; k < 3; ++k) b.lo[k] = 0.5 * (c.bbox_lo[k] + c.bbox_hi[k]) - 0.5 * ext;
    b.inv = 1.0 / ext;
    return b;
}

}  // namespace

// ============================================================== wrappers
void launch_prep_sources(Ctx &c) {
    hipLaunchKernelGGL(k_prep_sources, dim3(grid_for(c.nnodes)), dim3(kBlk), 0, c.stream, c.nnodes, c.nq,
                       c.verts.as<double>(), c.tris.as<int32_t>(), c.quadratic ? c.tris6.as<int32_t>() : nullptr,
                       c.rule.as<double>(), c.sigma.as<double>(), c.src.as<Src>());
    LSS_CHECK_LAUNCH("k_prep_sources");
}

void launch_prep_raw(Ctx &c, RawNode *out) {
    const int64_t nn = c.ntris * (int64_t)c.nq;
    hipLaunchKernelGGL(k_prep_raw, dim3(grid_for(nn)), dim3(kBlk), 0, c.stream, nn, c.nq,
                       c.verts.as<double>(), c.tris.as<int32_t>(), c.quadratic ? c.tris6.as<int32_t>() : nullptr,
                       c.rule.as<double>(), out);
    LSS_CHECK_LAUNCH("k_prep_raw");
}

void launch_centroids(Ctx &c, double lambda, Cen *out, double *D) {
    hipLaunchKernelGGL(k_centroids, dim3(grid_for(c.ntris)), dim3(kBlk), 0, c.stream, c.ntris,
                       c.verts.as<double>(), c.tris.as<int32_t>(), lambda, out, D);
    LSS_CHECK_LAUNCH("k_centroids");
}

double launch_check_orientation(Ctx &c, std::vector<double> &vol, int64_t &ndegen) {
    DBuf tmp;
    tmp.ensure(sizeof(double) * (c.nmesh + 1) + 64);
    double *dv = tmp.as<double>();
    unsigned long long *dn = reinterpret_cast<unsigned long long *>(dv + c.nmesh);
    LSS_HIP(hipMemsetAsync(tmp.p, 0, sizeof(double) * (c.nmesh + 1), c.stream));
    hipLaunchKernelGGL(k_orientation, dim3(grid_for(c.ntris)), dim3(kBlk), 0, c.stream, c.ntris, c.nmesh,
                       c.tri_off.as<int64_t>(), c.verts.as<double>(), c.tris.as<int32_t>(), dv, dn);
    LSS_CHECK_LAUNCH("k_orientation");
    vol.resize(c.nmesh);
    unsigned long long nd = 0;
    LSS_HIP(hipMemcpyAsync(vol.data(), dv, sizeof(double) * c.nmesh, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipMemcpyAsync(&nd, dn, sizeof(nd), hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    tmp.release();
    ndegen = (int64_t)nd;
    double mn = vol.empty() ? 0.0 : vol[0];
    for (double v : vol) mn = fmin(mn, v);
    return mn;
}

void launch_bbox(Ctx &c) {
    const int nb = 240;
    DBuf part;
    part.ensure(sizeof(double) * 6 * nb);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kBlk), 0, c.stream, c.nnodes, c.src.as<Src>(),
                       part.as<double>());
    LSS_CHECK_LAUNCH("k_bbox_partial");
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, c.stream, nb, part.as<double>());
    LSS_CHECK_LAUNCH("k_bbox_final");
    double h[6];
    LSS_HIP(hipMemcpyAsync(h, part.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    part.release();
    for (int k = 0; k < 3; ++k) { c.bbox_lo[k] = h[k]; c.bbox_hi[k] = h[3 + k]; }
}

void launch_pseudonormals(Ctx &c) {
    int64_t ncorner = 3 * c.ntris;
    DBuf cnt, off, fill, list, tmp;
    cnt.ensure(sizeof(int32_t) * (c.nverts + 1));
    off.ensure(sizeof(int32_t) * (c.nverts + 1));
    fill.ensure(sizeof(int32_t) * (c.nverts + 1));
    list.ensure(sizeof(int64_t) * ncorner);
    LSS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (c.nverts + 1), c.stream));
    LSS_HIP(hipMemsetAsync(fill.p, 0, sizeof(int32_t) * (c.nverts + 1), c.stream));
    hipLaunchKernelGGL(k_corner_count, dim3(grid_for(ncorner)), dim3(kBlk), 0, c.stream, ncorner,
                       c.tris.as<int32_t>(), cnt.as<int32_t>());
    LSS_CHECK_LAUNCH("k_corner_count");
    // exclusive scan of per-vertex counts (reuse the block-count scan kernels)
    {
        // blocks of kCompBlk vertices: per-block sums then scan, then local offsets
        int64_t nv = c.nverts;
        std::vector<int32_t> hc(nv);
        LSS_HIP(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int32_t) * nv, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        std::vector<int32_t> ho(nv + 1);
        int64_t acc = 0;
        for (int64_t v = 0; v < nv; ++v) { ho[v] = (int32_t)acc; acc += hc[v]; }
        ho[nv] = (int32_t)acc;
        LSS_HIP(hipMemcpyAsync(off.p, ho.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
    }
    hipLaunchKernelGGL(k_corner_fill, dim3(grid_for(ncorner)), dim3(kBlk), 0, c.stream, ncorner,
                       c.tris.as<int32_t>(), off.as<int32_t>(), fill.as<int32_t>(), list.as<int64_t>());
    LSS_CHECK_LAUNCH("k_corner_fill");
    c.vH.ensure(sizeof(double) * 3 * c.nverts);
    hipLaunchKernelGGL(k_vertex_H, dim3(grid_for(c.nverts)), dim3(kBlk), 0, c.stream, c.nverts,
                       c.verts.as<double>(), c.tris.as<int32_t>(), chart_tris6(c), off.as<int32_t>(),
                       cnt.as<int32_t>(), list.as<int64_t>(), c.vH.as<double>());
    LSS_CHECK_LAUNCH("k_vertex_H");
    LSS_HIP(hipStreamSynchronize(c.stream));
    cnt.release(); off.release(); fill.release(); list.release();
}

void launch_target_keys(Ctx &c, const double *x, const int32_t *x_mesh, int64_t n, uint64_t *keys,
                        int32_t *idx) {
    hipLaunchKernelGGL(k_target_keys, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, x, x_mesh, c.nmesh,
                       make_box(c), keys, idx);
    LSS_CHECK_LAUNCH("k_target_keys");
}

void launch_gather_targets(Ctx &c, const double *x, const int32_t *x_mesh, const int32_t *perm, int64_t n,
                           double *tx, double *ty, double *tz, int32_t *tmesh) {
    hipLaunchKernelGGL(k_gather_targets, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, x, x_mesh, c.nmesh,
                       perm, tx, ty, tz, tmesh);
    LSS_CHECK_LAUNCH("k_gather_targets");
}

void launch_chart_init(Ctx &c, const double *uv, int32_t np, int64_t N) {
    NewtonState &s = c.ns;
    const bool fmm = c.opt.far_field == LSS_FAR_FMM && c.tree.root.p != nullptr;
    c.tkey.ensure(sizeof(uint64_t) * N);
    c.tkey2.ensure(sizeof(uint64_t) * N);
    c.tperm.ensure(sizeof(int32_t) * N);
    c.tperm2.ensure(sizeof(int32_t) * N);
    hipLaunchKernelGGL(k_chart_keys, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, c.verts.as<double>(),
                       c.tris.as<int32_t>(), chart_tris6(c), c.vH.as<double>(), uv, np, c.tri_off.as<int64_t>(), c.nmesh,
                       make_box(c), fmm ? c.tree.root.as<double>() : nullptr, c.tree.bits, c.tkey.as<uint64_t>(),
                       c.tperm.as<int32_t>());
    LSS_CHECK_LAUNCH("k_chart_keys");
    size_t tb = sort_pairs_u64_tmp_bytes(N);
    c.sort_tmp.ensure(tb);
    sort_pairs_u64(c.sort_tmp.p, tb, c.tkey.as<uint64_t>(), c.tkey2.as<uint64_t>(), c.tperm.as<int32_t>(),
                   c.tperm2.as<int32_t>(), N, 0, 64, c.stream);
    s.T.ensure(sizeof(double) * 3 * N);
    s.H.ensure(sizeof(double) * 3 * N);
    s.h.ensure(sizeof(double) * N);
    s.lo.ensure(sizeof(double) * N);
    s.hi.ensure(sizeof(double) * N);
    s.sig.ensure(sizeof(double) * N);
    s.mesh.ensure(sizeof(int32_t) * N);
    s.orig.ensure(sizeof(int32_t) * N);
    s.status.ensure(N);
    s.iters.ensure(N);
    s.seen.ensure(N);
    s.active.ensure(sizeof(int32_t) * N);
    s.active2.ensure(sizeof(int32_t) * N);
    s.flag.ensure(sizeof(int32_t) * N);
    s.blocksum.ensure(sizeof(int32_t) * (ceil_div(N, kCompBlk) + 4));
    s.nact.ensure(sizeof(int32_t) * 4);
    s.hist.ensure(sizeof(int32_t) * kHistCap);
    hipLaunchKernelGGL(k_chart_init, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, c.verts.as<double>(),
                       c.tris.as<int32_t>(), chart_tris6(c), c.vH.as<double>(), uv, np, c.tri_off.as<int64_t>(), c.nmesh,
                       c.sigma.as<double>(), c.tperm2.as<int32_t>(), s.T.as<double>(), s.H.as<double>(),
                       s.h.as<double>(), s.lo.as<double>(), s.hi.as<double>(), s.sig.as<double>(),
                       s.mesh.as<int32_t>(), s.orig.as<int32_t>(), s.status.as<int8_t>(), s.iters.as<int8_t>(),
                       s.seen.as<int8_t>(),
                       s.flag.as<int32_t>());
    LSS_CHECK_LAUNCH("k_chart_init");
    // initial active list: all non-degenerate nodes, in sorted order
    hipLaunchKernelGGL(k_iota, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, s.active2.as<int32_t>());
    LSS_CHECK_LAUNCH("k_iota");
    int32_t nN[3] = {(int32_t)N, (int32_t)N, 0};
    LSS_HIP(hipMemcpyAsync(s.nact.as<int32_t>() + 1, nN, 3 * sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
    LSS_HIP(hipMemsetAsync(s.hist.p, 0, sizeof(int32_t) * kHistCap, c.stream));
    // compact active2[0..N) by flag into active, count into nact[0]
    int32_t nb = (int32_t)ceil_div(N, kCompBlk);
    hipLaunchKernelGGL(k_block_count, dim3(nb), dim3(kCompBlk), 0, c.stream, s.nact.as<int32_t>() + 1,
                       s.flag.as<int32_t>(), s.blocksum.as<int32_t>());
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kCompBlk), 0, c.stream, nb, s.blocksum.as<int32_t>(),
                       s.nact.as<int32_t>());
    hipLaunchKernelGGL(k_block_scatter, dim3(nb), dim3(kCompBlk), 0, c.stream, s.nact.as<int32_t>() + 1,
                       s.flag.as<int32_t>(), s.blocksum.as<int32_t>(), s.active2.as<int32_t>(),
                       s.active.as<int32_t>());
    LSS_CHECK_LAUNCH("compact(init)");
    LSS_HIP(hipStreamSynchronize(c.stream));   // the host copy of nN above must not outlive the call
}

void launch_newton_targets(Ctx &c, int64_t N) {
    NewtonState &s = c.ns;
    hipLaunchKernelGGL(k_newton_targets, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, s.nact.as<int32_t>(),
                       s.active.as<int32_t>(), s.T.as<double>(), s.H.as<double>(), s.h.as<double>(),
                       s.mesh.as<int32_t>(), c.tx.as<double>(), c.ty.as<double>(), c.tz.as<double>(),
                       c.tmesh.as<int32_t>());
    LSS_CHECK_LAUNCH("k_newton_targets");
}

void launch_newton_update(Ctx &c, int64_t N, double tau, const double *phi, const double *grad) {
    NewtonState &s = c.ns;
    int32_t maxit = c.opt.newton_max_iter > 0 ? c.opt.newton_max_iter : kMaxIterDefault;
    hipLaunchKernelGGL(k_newton_update, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, s.nact.as<int32_t>(),
                       s.active.as<int32_t>(), phi, grad, s.H.as<double>(), s.h.as<double>(), s.lo.as<double>(),
                       s.hi.as<double>(), s.sig.as<double>(), s.status.as<int8_t>(), s.iters.as<int8_t>(),
                       s.seen.as<int8_t>(),
                       s.flag.as<int32_t>(), tau, maxit);
    LSS_CHECK_LAUNCH("k_newton_update");
}

// Newton iteration bookkeeping, all on the device (capturable): nact[0] is
// the active count, nact[1] the count at the start of the iteration, nact[2]
// the total N, nact[3] the number of non-empty iterations; hist[k] records
// the active count of iteration k.
void launch_iter_mark(Ctx &c) {
    NewtonState &s = c.ns;
    hipLaunchKernelGGL(k_iter_mark, dim3(1), dim3(64), 0, c.stream, s.nact.as<int32_t>(), s.hist.as<int32_t>(),
                       (int32_t)kHistCap);
    LSS_CHECK_LAUNCH("k_iter_mark");
}

// active <- compact(active, flag) over the nact[1] entries of this iteration
void launch_compact_active(Ctx &c, int64_t N) {
    NewtonState &s = c.ns;
    hipLaunchKernelGGL(k_copy_active, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, s.nact.as<int32_t>() + 1,
                       s.active.as<int32_t>(), s.active2.as<int32_t>());
    int32_t nb = (int32_t)ceil_div(N, kCompBlk);
    hipLaunchKernelGGL(k_block_count, dim3(nb), dim3(kCompBlk), 0, c.stream, s.nact.as<int32_t>() + 1,
                       s.flag.as<int32_t>(), s.blocksum.as<int32_t>());
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kCompBlk), 0, c.stream, nb, s.blocksum.as<int32_t>(),
                       s.nact.as<int32_t>());
    hipLaunchKernelGGL(k_block_scatter, dim3(nb), dim3(kCompBlk), 0, c.stream, s.nact.as<int32_t>() + 1,
                       s.flag.as<int32_t>(), s.blocksum.as<int32_t>(), s.active2.as<int32_t>(),
                       s.active.as<int32_t>());
    LSS_CHECK_LAUNCH("compact");
}

int32_t compact_blocks(int64_t n_max) { return (int32_t)ceil_div(n_max > 0 ? n_max : 1, kCompBlk); }

// out <- in[i] for flag[i] != 0, i < n (n = *n_dev if given, else n_max); count -> *count_dev
void compact_flags(Ctx &c, int64_t n_max, const int32_t *n_dev, const int32_t *flag, const int32_t *in,
                   int32_t *out, int32_t *count_dev, int32_t *blocksum) {
    const int32_t nb = compact_blocks(n_max);
    int32_t *bsp = blocksum;
    if (!bsp) {
        c.ns.blocksum.ensure(sizeof(int32_t) * (nb + 2));
        bsp = c.ns.blocksum.as<int32_t>();
    } else if (!n_dev) {
        throw Error{LSS_EHIP, "compact_flags: a caller workspace needs the count on the device"};
    }
    const int32_t *nd = n_dev;
    if (!nd) {
        int32_t *tmp = bsp + nb;
        int32_t v = (int32_t)n_max;
        LSS_HIP(hipMemcpyAsync(tmp, &v, sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        nd = tmp;
    }
    hipLaunchKernelGGL(k_block_count, dim3(nb), dim3(kCompBlk), 0, c.stream, nd, flag, bsp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kCompBlk), 0, c.stream, nb, bsp, count_dev);
    hipLaunchKernelGGL(k_block_scatter, dim3(nb), dim3(kCompBlk), 0, c.stream, nd, flag, bsp, in, out);
    LSS_CHECK_LAUNCH("compact_flags");
}

void launch_newton_output(Ctx &c, int64_t N, double *h, double *xout, int8_t *status, int8_t *iters) {
    NewtonState &s = c.ns;
    hipLaunchKernelGGL(k_newton_output, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, s.orig.as<int32_t>(),
                       s.T.as<double>(), s.H.as<double>(), s.h.as<double>(), s.status.as<int8_t>(),
                       s.iters.as<int8_t>(), h, xout, status, iters);
    LSS_CHECK_LAUNCH("k_newton_output");
}

}  // namespace lss

// ------------------------------------------------------- chart geometry
namespace lss {
namespace {

// chart point x = T + h H of node q (eq. chart) and its mesh (batches)
__global__ void k_chart_points(int64_t N, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                               const int32_t *__restrict__ tris6, const double *__restrict__ vH, const double *__restrict__ uv, int32_t np,
                               const int64_t *__restrict__ tri_off, int32_t nmesh, const double *__restrict__ h,
                               double *x, int32_t *xmesh) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    double T[3], H[3];
    int64_t j;
    chart_TH(verts, tris, tris6, vH, uv, np, q, T, H, j);
    const double hq = h[q];
    for (int c = 0; c < 3; ++c) x[3 * q + c] = T[c] + hq * H[c];
    if (xmesh) xmesh[q] = mesh_of_tri(tri_off, nmesh, j);
}

// Tangents, area element and unit normal of the chart x = T + h H at node q
// (section 3.1, eq. u_vector, U_vector_2, v_vector, v_vector_2, eq. da):
// H is linear in (u, v) on the triangle (eq. mkpseudovec), H_u = H2 - H1
// (likewise in v); T_u, T_v are those of the chart base (the corner triangle,
// or the curved patch); dh/du follows from x_u being tangent to the level
// set, i.e. orthogonal to grad Phi; the outward unit normal is
// -grad Phi / |grad Phi| (Phi grows inward).  Any output may be null.
__global__ void k_chart_geometry(int64_t N, const double *__restrict__ verts, const int32_t *__restrict__ tris,
                                 const int32_t *__restrict__ tris6, const double *__restrict__ vH,
                                 const double *__restrict__ uv, int32_t np, const double *__restrict__ h,
                                 const double *__restrict__ grad, double *xu, double *xv, double *da, double *nrm) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    ChartFrame f;
    int64_t j;
    chart_frame(verts, tris, tris6, vH, uv, np, q, f, j);
    const double *H = f.H, *Tu = f.Tu, *Tv = f.Tv, *Hu = f.Hu, *Hv = f.Hv;
    double g[3];
    for (int c = 0; c < 3; ++c) g[c] = grad[3 * q + c];
    const double hq = h[q];
    double au[3], av[3];                      // T_u + h H_u, T_v + h H_v
    for (int c = 0; c < 3; ++c) {
        au[c] = Tu[c] + hq * Hu[c];
        av[c] = Tv[c] + hq * Hv[c];
    }
    const double den = H[0] * g[0] + H[1] * g[1] + H[2] * g[2];
    const double hu = -(au[0] * g[0] + au[1] * g[1] + au[2] * g[2]) / den;
    const double hv = -(av[0] * g[0] + av[1] * g[1] + av[2] * g[2]) / den;
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = au[c] + hu * H[c];
        b[c] = av[c] + hv * H[c];
    }
    if (xu)
        for (int c = 0; c < 3; ++c) xu[3 * q + c] = a[c];
    if (xv)
        for (int c = 0; c < 3; ++c) xv[3 * q + c] = b[c];
    if (da) {
        const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
        da[q] = sqrt(cx * cx + cy * cy + cz * cz);
    }
    if (nrm) {
        const double ig = -1.0 / sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        for (int c = 0; c < 3; ++c) nrm[3 * q + c] = g[c] * ig;
    }
}

}  // namespace

void launch_chart_points(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, double *x,
                         int32_t *xmesh) {
    hipLaunchKernelGGL(k_chart_points, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, c.verts.as<double>(),
                       c.tris.as<int32_t>(), chart_tris6(c), c.vH.as<double>(), uv, np, c.tri_off.as<int64_t>(), c.nmesh, h, x,
                       xmesh);
    LSS_CHECK_LAUNCH("k_chart_points");
}

void launch_chart_geometry(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, const double *grad,
                           double *xu, double *xv, double *da, double *nrm) {
    hipLaunchKernelGGL(k_chart_geometry, dim3(grid_for(N)), dim3(kBlk), 0, c.stream, N, c.verts.as<double>(),
                       c.tris.as<int32_t>(), chart_tris6(c), c.vH.as<double>(), uv, np, h, grad, xu, xv, da, nrm);
    LSS_CHECK_LAUNCH("k_chart_geometry");
}

}  // namespace lss
