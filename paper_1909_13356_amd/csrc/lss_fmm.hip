// Laplace-dipole fast multipole far field (section 4.4, eq. kerdecomp: beyond
// the cut the kernel is the double-layer kernel, summed here by an FMM):
// translation operators as dense real matrices, dipole P2M at the leaves, and
// every translation (M2M, M2L, L2L) as a gathered matrix product
//     Y[dst_j] += scale_j * Op * X[src_j]
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  M2L runs one launch per
// displacement class (one dense operator per class, all levels share it in
// box-scaled form); inside a launch every destination box appears once, so
// the accumulation is race free and deterministic.
#include <cstring>
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cmath>

#include "fmm_math.h"
#include "lss_internal.h"

namespace lss {

namespace {

using fmm::cd;
constexpr int kBlk = 256;
constexpr int kR = 7;
constexpr int kNClass = (2 * kR + 1) * (2 * kR + 1) * (2 * kR + 1);
constexpr double kPi = 3.14159265358979323846;

inline unsigned grid_for(int64_t n, int blk = kBlk) { return (unsigned)ceil_div(n > 0 ? n : 1, blk); }

// ------------------------------------------------------------- operators
// one table per operator: irregular (M2L, order 2p) or regular (M2M/L2L, order p)
__global__ void k_op_tables(int nops, const double *__restrict__ vecs, int order, int irregular, int stride, cd *tabs) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nops) return;
    const double *v = vecs + 3 * o;
    if (irregular) fmm::irregular_table(v[0], v[1], v[2], order, tabs + (int64_t)o * stride);
    else fmm::regular_table(v[0], v[1], v[2], order, tabs + (int64_t)o * stride);
}

// entry (row, k) of operator o stored k-major: opT[o][k * ncp + row]
__global__ void k_fill_op(int kind, int p, int ncp, int nops, const cd *__restrict__ tabs, int stride, double *ops) {
    const int64_t per = (int64_t)ncp * ncp;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int o = blockIdx.y;
    if (e >= per || o >= nops) return;
    const int k = (int)(e / ncp), row = (int)(e - (int64_t)k * ncp);
    const int nc = fmm::ncoef(p);
    double v = 0.0;
    if (row < nc && k < nc) {
        int kk, l, n, m;
        bool oi, ii;
        fmm::decode(row, kk, l, oi);
        fmm::decode(k, n, m, ii);
        const cd *tab = tabs + (int64_t)o * stride;
        if (kind == 0) v = fmm::folded_entry(fmm::M2LMap{tab}, kk, l, oi, n, m, ii);
        else if (kind == 1) v = fmm::folded_entry(fmm::M2MMap{tab}, kk, l, oi, n, m, ii);
        else v = fmm::folded_entry(fmm::L2LMap{tab}, kk, l, oi, n, m, ii);
    }
    ops[(int64_t)o * per + e] = v;
}

// ------------------------------------------------------------------ P2M
// Neighbour lanes through DPP wave shifts (one VALU move per 32-bit half, no
// LDS round trip): the value of lane + 1 and of lane - 1; the lanes without a
// neighbour (63 and 0) receive 0.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_is_next) {
    const long long b = __double_as_longlong(v);
    int lo = (int)b, hi = (int)(b >> 32);
    if (ctrl_is_next) {
        lo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);     // wave_shl:1
        hi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);     // wave_shr:1
        hi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_next_lane(double v) { return dpp_f64(v, 1); }
__device__ __forceinline__ double from_prev_lane(double v) { return dpp_f64(v, 0); }

struct Geo {
    const double *root;         // per-mesh root cubes (corner xyz, side)
    const int32_t *bmesh;
};

// P2M by columns: one wavefront per non-empty leaf; lane (g, m) owns column
// m = 0..p of the regular solid harmonics of node g of a group of G = 64/(p+1)
// nodes.  At step s every lane holds U_s^m (zero for m > s; the diagonal is
// built up meanwhile), takes U_s^{m-1} and U_s^{m+1} from its neighbours and
// adds the dipole term of M_{s+1}^m into an LDS accumulator of its node slot.
// No division and no barrier inside the node loop.
__global__ __launch_bounds__(64) void k_p2m_cols(const int32_t *__restrict__ nleaf_dev,
                                                 const int32_t *__restrict__ leaves, int p, int ncp, Geo g,
                                                 const int32_t *__restrict__ lev, const int32_t *__restrict__ ijk,
                                                 const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                                                 const Src *__restrict__ src, double *M) {
    extern __shared__ double smem[];
    const int C = p + 1, G = 64 / C;
    const int ntri = (p + 1) * (p + 2) / 2;
    cd *acc = reinterpret_cast<cd *>(smem);               // G x ntri, at tri(n, m)
    double *rinv = smem + 2 * G * ntri;                   // 1/((n+m)(n-m)) at tri(n, m), n > m
    double *dfac = rinv + ntri;                           // -1/(2t), t = 1..p
    if ((int)blockIdx.x >= *nleaf_dev) return;
    const int lane = threadIdx.x;
    for (int i = lane; i < ntri; i += 64) {
        int n = 0;
        while ((n + 1) * (n + 2) / 2 <= i) ++n;
        const int m = i - n * (n + 1) / 2;
        rinv[i] = n > m ? 1.0 / ((double)(n + m) * (double)(n - m)) : 0.0;
    }
    for (int t = lane; t <= p; t += 64) dfac[t] = t > 0 ? -0.5 / (double)t : 0.0;
    for (int i = lane; i < G * ntri; i += 64) acc[i] = cd{0.0, 0.0};
    __syncthreads();
    const int32_t b = leaves[blockIdx.x];
    const double s = box_side(g.root, g.bmesh, b, lev[b]);
    const double *o = g.root + 4 * g.bmesh[b];
    const double c0 = o[0] + (ijk[3 * b] + 0.5) * s, c1 = o[1] + (ijk[3 * b + 1] + 0.5) * s,
                 c2 = o[2] + (ijk[3 * b + 2] + 0.5) * s;
    const double inv4pis = 1.0 / (4.0 * kPi * s);
    const double invs = 1.0 / s;
    const int gi = lane / C, m = lane % C;
    const bool slot = gi < G;                             // lane holds a (node, column) slot
    cd *accg = acc + (slot ? gi : 0) * ntri;
    const int64_t b0 = nb[b], b1 = ne[b];
    for (int64_t k0 = b0; k0 < b1; k0 += G) {
        const int64_t k = k0 + gi;
        const bool live = slot && k < b1;
        double x = 0, y = 0, z = 0, ax = 0, ay = 0, az = 0;
        if (live) {
            const Src sr = src[k];
            // unfold the dipole: a = a' / c(sigma), 1/c = 4 sqrt2 pi^1.5 sigma^3, sigma^2 = 1/(2 s2)
            const double sg2 = 0.5 / sr.s2;
            const double f = 4.0 * 1.4142135623730951 * 5.568327996831708 * sg2 * sqrt(sg2);
            x = (sr.yx - c0) * invs;
            y = (sr.yy - c1) * invs;
            z = (sr.yz - c2) * invs;
            ax = sr.ax * f;
            ay = sr.ay * f;
            az = sr.az * f;
        }
        const double r2 = x * x + y * y + z * z;
        cd d = {1.0, 0.0}, u1 = {0.0, 0.0}, u2 = {0.0, 0.0};
        for (int st = 0; st < p; ++st) {
            cd u = {0.0, 0.0};
            if (st == m) {
                u = d;
            } else if (st > m) {
                const double w = rinv[fmm::tri(st, m)];
                const double a2 = (double)(2 * st - 1) * z;
                u = cd{(a2 * u1.re - r2 * u2.re) * w, (a2 * u1.im - r2 * u2.im) * w};
            } else {
                d = fmm::cscale(fmm::cmul(d, cd{x, y}), dfac[st + 1]);
            }
            if (st >= m) { u2 = u1; u1 = u; }
            // neighbours' columns at order st (same node slot; U^{-1} = -conj(U^1))
            const double upre = from_next_lane(u.re), upim = from_next_lane(u.im);
            const double dnre = from_prev_lane(u.re), dnim = from_prev_lane(u.im);
            cd up = m + 1 < C ? cd{upre, upim} : cd{0.0, 0.0};
            cd dn = m >= 1 ? cd{dnre, dnim} : cd{-upre, upim};
            if (live && m <= st + 1) {
                const cd t = fmm::cadd(fmm::cadd(fmm::cmul(cd{0.5 * ax, -0.5 * ay}, up),
                                                 fmm::cmul(cd{-0.5 * ax, -0.5 * ay}, dn)),
                                       fmm::cscale(u, az));
                cd &A = accg[fmm::tri(st + 1, m)];
                A.re -= inv4pis * t.re;         // conj, times -1/(4 pi s)
                A.im += inv4pis * t.im;
            }
        }
    }
    __syncthreads();
    double *Mb = M + (int64_t)b * ncp;
    for (int i = lane; i < ntri; i += 64) {
        int n = 0;
        while ((n + 1) * (n + 2) / 2 <= i) ++n;
        const int mm = i - n * (n + 1) / 2;
        if (n == 0) continue;
        double re = 0.0, im = 0.0;
        for (int q = 0; q < G; ++q) { re += acc[q * ntri + i].re; im += acc[q * ntri + i].im; }
        Mb[fmm::ire(n, mm)] = re;
        if (mm > 0) Mb[fmm::iim(n, mm)] = im;
    }
}


// The same P2M for the default orders (P known at compile time): lane (g, m)
// keeps its column's contributions to M_n^m, n = 1..P, in registers across
// all the leaf's nodes (the step loop is unrolled), instead of a read-modify-
// write in LDS per step; the G node slots are summed by shuffles at the end,
// in the order the LDS version sums them.
template <int P>
__global__ __launch_bounds__(64) void k_p2m_reg(const int32_t *__restrict__ nleaf_dev,
                                                const int32_t *__restrict__ leaves, int ncp, Geo g,
                                                const int32_t *__restrict__ lev, const int32_t *__restrict__ ijk,
                                                const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                                                const Src *__restrict__ src, double *M) {
    constexpr int C = P + 1, G = 64 / C, ntri = (P + 1) * (P + 2) / 2;
    __shared__ double rinv[ntri];                         // 1/((n+m)(n-m)) at tri(n, m), n > m
    __shared__ double dfac[P + 1];                        // -1/(2t), t = 1..P
    if ((int)blockIdx.x >= *nleaf_dev) return;
    const int lane = threadIdx.x;
    for (int i = lane; i < ntri; i += 64) {
        int n = 0;
        while ((n + 1) * (n + 2) / 2 <= i) ++n;
        const int m = i - n * (n + 1) / 2;
        rinv[i] = n > m ? 1.0 / ((double)(n + m) * (double)(n - m)) : 0.0;
    }
    for (int t = lane; t <= P; t += 64) dfac[t] = t > 0 ? -0.5 / (double)t : 0.0;
    __syncthreads();
    const int32_t b = leaves[blockIdx.x];
    const double s = box_side(g.root, g.bmesh, b, lev[b]);
    const double *o = g.root + 4 * g.bmesh[b];
    const double c0 = o[0] + (ijk[3 * b] + 0.5) * s, c1 = o[1] + (ijk[3 * b + 1] + 0.5) * s,
                 c2 = o[2] + (ijk[3 * b + 2] + 0.5) * s;
    const double inv4pis = 1.0 / (4.0 * kPi * s);
    const double invs = 1.0 / s;
    const int gi = lane / C, m = lane % C;
    const bool slot = gi < G;
    double are[P], aim[P];                                // contributions to M_{st+1}^m
#pragma unroll
    for (int st = 0; st < P; ++st) are[st] = aim[st] = 0.0;
    double w[P];                                          // recurrence weights of column m
#pragma unroll
    for (int st = 0; st < P; ++st) w[st] = rinv[fmm::tri(st, m)];     // in range for every m <= P
    const int64_t b0 = nb[b], b1 = ne[b];
    for (int64_t k0 = b0; k0 < b1; k0 += G) {
        const int64_t k = k0 + gi;
        const bool live = slot && k < b1;
        double x = 0, y = 0, z = 0, ax = 0, ay = 0, az = 0;
        if (live) {
            const Src sr = src[k];
            // unfold the dipole: a = a' / c(sigma), 1/c = 4 sqrt2 pi^1.5 sigma^3, sigma^2 = 1/(2 s2)
            const double sg2 = 0.5 / sr.s2;
            const double f = 4.0 * 1.4142135623730951 * 5.568327996831708 * sg2 * sqrt(sg2);
            x = (sr.yx - c0) * invs;
            y = (sr.yy - c1) * invs;
            z = (sr.yz - c2) * invs;
            ax = sr.ax * f;
            ay = sr.ay * f;
            az = sr.az * f;
        }
        const double r2 = x * x + y * y + z * z;
        // The dipole term of M_{st+1}^m is t = hp U^{m+1} + hm U^{m-1} + az U^m
        // (hp = (ax - i ay) / 2, hm = (-ax - i ay) / 2, U at order st), taken
        // conjugated and times -1/(4 pi s).  Written out as real coefficients
        // of (Re, Im) of U^{m+1}, U^{m-1} and U^m, with the two edge columns
        // folded in: U^{-1} = -conj(U^1) for m = 0, and no U^{P+1} for m = P;
        // a dead slot has all coefficients 0.
        const double hpr = 0.5 * ax, hpi = -0.5 * ay, hmr = -0.5 * ax, hmi = -0.5 * ay;
        double qr[4] = {hpr, -hpi, hmr, -hmi}, qi[4] = {hpi, hpr, hmi, hmr};
        if (m == 0) {
            qr[0] = hpr - hmr; qr[1] = -hpi - hmi; qr[2] = 0.0; qr[3] = 0.0;
            qi[0] = hpi - hmi; qi[1] = hpr + hmr; qi[2] = 0.0; qi[3] = 0.0;
        } else if (m == P) {
            qr[0] = qr[1] = 0.0;
            qi[0] = qi[1] = 0.0;
        }
        const double sr_ = -inv4pis, si_ = inv4pis;
        const double cr0 = sr_ * qr[0], cr1 = sr_ * qr[1], cr2 = sr_ * qr[2], cr3 = sr_ * qr[3], cr4 = sr_ * az;
        const double ci0 = si_ * qi[0], ci1 = si_ * qi[1], ci2 = si_ * qi[2], ci3 = si_ * qi[3], ci4 = si_ * az;
        // U^m at order st, for every lane and step without branches: the
        // diagonal d = U^m_m is carried up (multiplied by (x + i y) / (-2 t)
        // at every step, read at st = m), the column recurrence starts from
        // zeros (so it is 0 for st <= m)
        double dr = 1.0, di = 0.0, u1r = 0.0, u1i = 0.0, u2r = 0.0, u2i = 0.0;
#pragma unroll
        for (int st = 0; st < P; ++st) {
            const double a2 = (double)(2 * st - 1) * z;
            double ur = (a2 * u1r - r2 * u2r) * w[st], ui = (a2 * u1i - r2 * u2i) * w[st];
            const bool diag = st == m;
            ur = diag ? dr : ur;
            ui = diag ? di : ui;
            const double sc = -0.5 / (double)(st + 1);
            const double ndr = (dr * x - di * y) * sc, ndi = (dr * y + di * x) * sc;
            dr = ndr;
            di = ndi;
            u2r = u1r; u2i = u1i;
            u1r = ur; u1i = ui;
            const double upr = from_next_lane(ur), upi = from_next_lane(ui);
            const double dnr = from_prev_lane(ur), dni = from_prev_lane(ui);
            are[st] = fma(cr0, upr, fma(cr1, upi, fma(cr2, dnr, fma(cr3, dni, fma(cr4, ur, are[st])))));
            aim[st] = fma(ci0, upr, fma(ci1, upi, fma(ci2, dnr, fma(ci3, dni, fma(ci4, ui, aim[st])))));
        }
    }
    // sum the node slots into lanes (0, m) and write M~_n^m, n = 1..P
    double *Mb = M + (int64_t)b * ncp;
#pragma unroll
    for (int st = 0; st < P; ++st) {
        double re = 0.0 + are[st], im = 0.0 + aim[st];
#pragma unroll
        for (int q = 1; q < G; ++q) {
            re += __shfl(are[st], lane + q * C);
            im += __shfl(aim[st], lane + q * C);
        }
        const int n = st + 1;
        if (gi == 0 && m <= n) {
            Mb[fmm::ire(n, m)] = re;
            if (m > 0) Mb[fmm::iim(n, m)] = im;
        }
    }
}

__global__ void k_leaf_flags(int64_t n, const int32_t *__restrict__ child, const int64_t *__restrict__ nb,
                             const int64_t *__restrict__ ne, int32_t *flag, int32_t *ids) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    flag[b] = (child[b] < 0 && ne[b] > nb[b]) ? 1 : 0;
    ids[b] = (int32_t)b;
}

// --------------------------------------------------------- gathered GEMM
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kKB = 16;

enum { G_LIST = 0, G_M2M = 1, G_L2L = 2 };

// One launch of translations Y[dst] += scale * Op X[src] over a list of pairs.
//   G_LIST: M2L pairs of one displacement class (dst = low 32 bits of mkey, src = mval).
//   G_M2M:  pair j = the j-th parent of a level; its 8 children (consecutive boxes
//           base + 8j ..) are one input column of 8 ncp coefficients and the 8 octant
//           operators, stored one after the other in k-major order, are one
//           ncp x 8 ncp operator, so each parent is written once per launch.
//   G_L2L:  grid.z = octant o; pair j writes child base + 8j + o from its parent with
//           operator o.  Children are distinct, so the 8 octants share the launch.
struct GemmArgs {
    int mode, ncp, nk;          // nk: length of the contraction (ncp, or 8 ncp for G_M2M)
    int64_t npairs;
    const double *opT;          // ncp rows, k-major (G_L2L: 8 such matrices)
    const double *X;
    double *Y;
    const uint64_t *mkey;       // G_LIST
    const int32_t *mval;        // G_LIST
    int64_t base;               // G_M2M / G_L2L: first child box of the level
    const int32_t *parent, *lev;
    const double *root;
    const int32_t *bmesh;
    int rows = 0;               // output rows (leading coefficients written); 0 = ncp
};

// destination box, first element of the input column and output scale of pair j
__device__ inline void pair_of(const GemmArgs &a, int64_t j, int oct, int64_t &dst, int64_t &col, double &scale) {
    scale = 1.0;
    if (a.mode == G_LIST) {
        dst = (int64_t)(uint32_t)(a.mkey[j] & 0xffffffffu);
        col = (int64_t)a.mval[j] * a.ncp;
        scale = 1.0 / box_side(a.root, a.bmesh, (int32_t)dst, a.lev[dst]);   // 1 / side of the target box
    } else if (a.mode == G_M2M) {
        const int64_t ch = a.base + 8 * j;
        dst = a.parent[ch];
        col = ch * a.ncp;
    } else {
        dst = a.base + 8 * j + oct;
        col = (int64_t)a.parent[dst] * a.ncp;
    }
}

// 64 output rows x 128 pairs per workgroup; wave w owns pairs 32w..32w+31 of
// the tile and eight 16x16 accumulator tiles (4 row groups x 2 pair groups).
// The operator (k-major) and the gathered input columns go through LDS in
// blocks of kKB coefficients; the next block is fetched into registers while
// the MFMAs of the current one run.  Asking for four waves per SIMD makes the
// compiler keep the accumulators in ordinary VGPRs (126 in all, no AGPRs):
// four workgroups share a CU instead of two, which hides the barrier and load
// latency of one workgroup behind the MFMAs of the others.
// TP = 128 pairs per workgroup for long pair lists, 64 for short ones (twice
// the workgroups for the same work where one launch would not fill the chip).
constexpr int kTR = 64;
template <int TP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm(GemmArgs a) {
    constexpr int kTP = TP, NT = TP / 64, TPC = 256 / TP;   // 16-pair groups per wave, threads per column
    __shared__ double As[kKB][kTR + 1];
    __shared__ double Bs[kKB][kTP + 1];
    __shared__ int64_t scol[kTP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.x * kTR;
    const int64_t j0 = (int64_t)blockIdx.y * kTP;
    const int oct = blockIdx.z;
    const double *__restrict__ op = a.opT + (int64_t)oct * a.ncp * a.ncp;
    if (threadIdx.x < kTP) {
        int64_t j = j0 + threadIdx.x, d, col;
        double sc;
        if (j < a.npairs) { pair_of(a, j, oct, d, col, sc); scol[threadIdx.x] = col; }
        else scol[threadIdx.x] = -1;
    }
    __syncthreads();
    // per thread: A elements (k, r) = (e / kTR, e % kTR) for e = tid + 256 i, i < 4;
    // B elements (k, c) with c = tid / TPC, k = kNB (tid % TPC) + i, i < kNB (TPC threads per column)
    constexpr int kNA = kKB * kTR / 256, kNB = kKB * kTP / 256;
    const int bc = threadIdx.x / TPC, bk = (threadIdx.x % TPC) * kNB;
    const int64_t bcol = scol[bc];
    double ra[kNA], rb[kNB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kNA; ++i) {
            const int e = threadIdx.x + 256 * i, kk = e / kTR, rr = e % kTR;
            ra[i] = (r0 + rr < a.rows) ? op[(int64_t)(k0 + kk) * a.ncp + r0 + rr] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kNB; ++i) rb[i] = bcol >= 0 ? a.X[bcol + k0 + bk + i] : 0.0;
    };
    d4 acc[4][NT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        for (int t = 0; t < NT; ++t) acc[i][t] = d4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < a.nk; k0 += kKB) {
        __syncthreads();                                   // previous block's MFMAs are done with LDS
#pragma unroll
        for (int i = 0; i < kNA; ++i) {
            const int e = threadIdx.x + 256 * i;
            As[e / kTR][e % kTR] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < kNB; ++i) Bs[bk + i][bc] = rb[i];
        __syncthreads();
        if (k0 + kKB < a.nk) fetch(k0 + kKB);
#pragma unroll
        for (int kk = 0; kk < kKB; kk += 4) {
            double bv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[t] = Bs[kk + (lane >> 4)][16 * NT * w + 16 * t + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double av = As[kk + (lane >> 4)][16 * i + (lane & 15)];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[t], acc[i][t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int64_t j = j0 + 16 * NT * w + 16 * t + (lane & 15);
        if (j >= a.npairs) continue;
        int64_t d, col;
        double sc;
        pair_of(a, j, oct, d, col, sc);
        double *y = a.Y + d * a.ncp;
        // v_mfma_f64_16x16x4f64 accumulator: register q of lane l holds row (l/16) + 4q, column l%16
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r0 + 16 * i + (lane >> 4) + 4 * q;
                if (row < a.rows) y[row] += sc * acc[i][t][q];
            }
    }
}

void gemm(Ctx &c, GemmArgs a) {
    if (a.rows <= 0) a.rows = a.ncp;
    // short lists (fewer than four 128-pair workgroups per CU) take 64-pair workgroups
    const bool small = a.npairs * (a.mode == G_L2L ? 8 : 1) * ceil_div(a.rows, kTR) < 4 * 256 * 128;
    const int tp = small ? 64 : 128;
    // split long pair lists so that grid.y stays within the launch limit
    const int64_t chunk = (int64_t)32768 * tp;
    for (int64_t j0 = 0; j0 < a.npairs; j0 += chunk) {
        GemmArgs b = a;
        b.npairs = a.npairs - j0 < chunk ? a.npairs - j0 : chunk;
        if (a.mode == G_LIST) { b.mkey = a.mkey + j0; b.mval = a.mval + j0; }
        else b.base = a.base + 8 * j0;
        dim3 grid((unsigned)ceil_div(b.rows, kTR), (unsigned)ceil_div(b.npairs, tp), a.mode == G_L2L ? 8u : 1u);
        if (small) hipLaunchKernelGGL(k_gemm<64>, grid, dim3(256), 0, c.stream, b);
        else hipLaunchKernelGGL(k_gemm<128>, grid, dim3(256), 0, c.stream, b);
        LSS_CHECK_LAUNCH("k_gemm");
    }
}

__global__ void k_fill_zero(int64_t n, double *y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 0.0;
}

__global__ void k_add(int64_t n, double *y, const double *x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

void launch_fill_zero(Ctx &c, double *y, int64_t n) {
    if (n <= 0) return;
    const int64_t g = ceil_div(n, kBlk);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlk), 0, c.stream, n, y);
    LSS_CHECK_LAUNCH("k_fill_zero");
}

void launch_add(Ctx &c, double *y, const double *x, int64_t n) {
    if (n <= 0) return;
    const int64_t g = ceil_div(n, kBlk);
    hipLaunchKernelGGL(k_add, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlk), 0, c.stream, n, y, x);
    LSS_CHECK_LAUNCH("k_add");
}

// M2L of the small displacement classes, target-major.  The pairs of all
// small classes are sorted by (target box, class) (key = T << 12 | class);
// the workgroup that meets the first pair of a target box applies every pair
// of that box in key order, each a matrix-vector product with the class
// operator (k-major, leading nkv coefficients in and out), and adds the sum,
// times 1 / side of the box, once.  A box is written by one workgroup only.
constexpr int kSmallClassPairs = 512;        // classes with at most this many pairs
constexpr int kSmallMaxCoeffs = 512;         // target-major only for ncp up to this
constexpr int kSmallRows = 2;                // rows per thread (256 threads)
static_assert(256 * kSmallRows >= kSmallMaxCoeffs, "k_m2l_small: every coefficient needs a thread");
static_assert(kNClass <= 4096, "k_m2l_small: the class index takes the low 12 bits of the key");
__global__ __launch_bounds__(256) void k_m2l_small(int64_t npairs, const uint64_t *__restrict__ key,
                                                   const int32_t *__restrict__ src, const int32_t *__restrict__ cls_slot,
                                                   const int32_t *__restrict__ cls_nkv, const double *__restrict__ ops,
                                                   const double *__restrict__ M, double *L, int ncp, Geo g,
                                                   const int32_t *__restrict__ lev) {
    extern __shared__ double xs[];           // the source box's leading coefficients
    const int tid = threadIdx.x;
    for (int64_t i = blockIdx.x; i < npairs; i += gridDim.x) {
        const uint32_t T = (uint32_t)(key[i] >> 12);
        if (i > 0 && (uint32_t)(key[i - 1] >> 12) == T) continue;      // uniform: not the box's first pair
        double acc[kSmallRows];
#pragma unroll
        for (int q = 0; q < kSmallRows; ++q) acc[q] = 0.0;
        for (int64_t j = i; j < npairs && (uint32_t)(key[j] >> 12) == T; ++j) {
            const int cls = (int)(key[j] & 0xfffu);
            const int nkv = cls_nkv[cls];
            const double *__restrict__ op = ops + (int64_t)cls_slot[cls] * ncp * ncp;
            const double *__restrict__ x = M + (int64_t)src[j] * ncp;
            __syncthreads();                 // the previous pair is done with xs
            for (int k = tid; k < nkv; k += 256) xs[k] = x[k];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kSmallRows; ++q) {
                const int r = tid + 256 * q;
                if (r < nkv) {
                    double sum = 0.0;
                    for (int k = 0; k < nkv; ++k) sum = fma(op[(int64_t)k * ncp + r], xs[k], sum);
                    acc[q] += sum;
                }
            }
        }
        const double sc = 1.0 / box_side(g.root, g.bmesh, (int32_t)T, lev[T]);
        double *y = L + (int64_t)T * ncp;
#pragma unroll
        for (int q = 0; q < kSmallRows; ++q) {
            const int r = tid + 256 * q;
            if (r < ncp) y[r] += sc * acc[q];
        }
    }
}

// keys (T << 12 | class) and sources of the pairs of the small classes:
// block b copies class b's segment [beg[b], beg[b] + n[b]) of the class-sorted
// M2L list to out + off[b]
__global__ void k_small_pairs(const int64_t *__restrict__ beg, const int64_t *__restrict__ off,
                              const int32_t *__restrict__ cls, const uint64_t *__restrict__ mkey,
                              const int32_t *__restrict__ mval, uint64_t *okey, int32_t *oval) {
    const int b = blockIdx.x;
    const int64_t b0 = beg[b], o0 = off[b], n = off[b + 1] - off[b];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const uint32_t T = (uint32_t)(mkey[b0 + j] & 0xffffffffu);
        okey[o0 + j] = ((uint64_t)T << 12) | (uint64_t)cls[b];
        oval[o0 + j] = mval[b0 + j];
    }
}

// class index -> offset vector
void class_vec(int cls, double v[3]) {
    const int W = 2 * kR + 1;
    v[0] = cls / (W * W) - kR;
    v[1] = (cls / W) % W - kR;
    v[2] = cls % W - kR;
}

// Order of the M2L of displacement class v (in box sides, |v|^2 >= K): the
// truncation error of the translation of a box's multipole to a same-size box
// at centre distance |v| falls like r^(p+1), r = a / |v|, a = sqrt(3)/2 the
// half-diagonal (on the octree workloads the error at the closest class
// follows this rate: p = 18 mixed loses 1.5e-7 at |v| = 2).  A class farther
// than the closest admissible one (|v| = sqrt(K)) reaches the same error at a
// lower order; kM2lMargin orders are kept on top.
constexpr int kM2lMargin = 2;

int m2l_order(int p, int K, const double v[3]) {
    const double a = 0.8660254037844386;
    const double d = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double r0 = a / std::sqrt((double)K), r = a / d;
    if (!(r < r0)) return p;
    const int pv = (int)std::ceil((p + 1) * std::log(r0) / std::log(r)) - 1 + kM2lMargin;
    return std::min(p, std::max(pv, 4));
}

void build_ops(Ctx &c, int kind, int nops, const std::vector<double> &vecs, int p, int ncp, double *dst) {
    const int order = kind == 0 ? 2 * p : p;
    const int stride = fmm::tri(order, order) + 1;
    DBuf dv, tabs;
    dv.ensure(sizeof(double) * 3 * nops);
    tabs.ensure(sizeof(cd) * (size_t)stride * nops);
    LSS_HIP(hipMemcpyAsync(dv.p, vecs.data(), sizeof(double) * 3 * nops, hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_op_tables, dim3(grid_for(nops, 64)), dim3(64), 0, c.stream, nops, dv.as<double>(), order,
                       kind == 0 ? 1 : 0, stride, tabs.as<cd>());
    LSS_CHECK_LAUNCH("k_op_tables");
    const int64_t per = (int64_t)ncp * ncp;
    hipLaunchKernelGGL(k_fill_op, dim3(grid_for(per), nops), dim3(kBlk), 0, c.stream, kind, p, ncp, nops,
                       tabs.as<cd>(), stride, dst);
    LSS_CHECK_LAUNCH("k_fill_op");
    LSS_HIP(hipStreamSynchronize(c.stream));
}

}  // namespace

// Expansions at the leaves (P2M) and up the tree (M2M) on c.stream; the
// workspace buffers belong to the caller and must outlive the kernels.
void upward_pass(Ctx &c, int p, int ncp, DBuf &flag, DBuf &ids, DBuf &leaves, DBuf &nleaf) {
    Tree &t = c.tree;
    // expansions
    LSS_HIP(hipMemsetAsync(t.M.p, 0, sizeof(double) * t.nboxes * ncp, c.stream));
    LSS_HIP(hipMemsetAsync(t.L.p, 0, sizeof(double) * t.nboxes * ncp, c.stream));
    Geo g{t.root.as<double>(), t.bmesh.as<int32_t>()};
    // P2M on the non-empty leaves
    flag.ensure(4 * t.nboxes); ids.ensure(4 * t.nboxes); leaves.ensure(4 * t.nboxes); nleaf.ensure(16);
    hipLaunchKernelGGL(k_leaf_flags, dim3(grid_for(t.nboxes)), dim3(kBlk), 0, c.stream, t.nboxes, t.child.as<int32_t>(),
                       t.nb.as<int64_t>(), t.ne.as<int64_t>(), flag.as<int32_t>(), ids.as<int32_t>());
    LSS_CHECK_LAUNCH("k_leaf_flags");
    compact_flags(c, t.nboxes, nullptr, flag.as<int32_t>(), ids.as<int32_t>(), leaves.as<int32_t>(), nleaf.as<int32_t>());
    int32_t nl = 0;
    LSS_HIP(hipMemcpyAsync(&nl, nleaf.p, 4, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    c.stats.n_leaves = nl;
    if (nl > 0) {
        if (p == 20 || p == 26) {
            auto k = p == 20 ? k_p2m_reg<20> : k_p2m_reg<26>;
            hipLaunchKernelGGL(k, dim3(nl), dim3(64), 0, c.stream, nleaf.as<int32_t>(), leaves.as<int32_t>(), ncp, g,
                               t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.nb.as<int64_t>(), t.ne.as<int64_t>(),
                               t.src.as<Src>(), t.M.as<double>());
            LSS_CHECK_LAUNCH("k_p2m_reg");
        } else {
            const int ntri = (p + 1) * (p + 2) / 2, G = 64 / (p + 1);
            size_t shm = sizeof(double) * (2 * G * ntri + ntri + p + 1);
            hipLaunchKernelGGL(k_p2m_cols, dim3(nl), dim3(64), shm, c.stream, nleaf.as<int32_t>(), leaves.as<int32_t>(),
                               p, ncp, g, t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.nb.as<int64_t>(),
                               t.ne.as<int64_t>(), t.src.as<Src>(), t.M.as<double>());
            LSS_CHECK_LAUNCH("k_p2m_cols");
        }
    }
    // upward pass: M2M from level depth to 1 into their parents
    for (int lvl = t.depth; lvl >= 1; --lvl) {
        const int64_t base = t.level_begin[lvl], npar = (t.level_begin[lvl + 1] - base) / 8;
        GemmArgs a{G_M2M, ncp, 8 * ncp, npar, t.opM2M.as<double>(), t.M.as<double>(), t.M.as<double>(), nullptr,
                   nullptr, base, t.parent.as<int32_t>(), t.level.as<int32_t>(), t.root.as<double>(),
                   t.bmesh.as<int32_t>()};
        gemm(c, a);
    }
}

void build_fmm(Ctx &c) {
    build_tree_boxes(c);
    Tree &t = c.tree;
    const int p = fmm_order_for(c);
    const int ncp = (int)ceil_div(fmm::ncoef(p), kKB) * kKB;
    const int64_t per = (int64_t)ncp * ncp;
    // operators: M2M / L2L for the 8 octants, M2L for the classes in use
    if (t.ops_p != p) {
        std::vector<double> w(24);
        for (int o = 0; o < 8; ++o) {
            w[3 * o] = (o & 1) ? 0.5 : -0.5;
            w[3 * o + 1] = ((o >> 1) & 1) ? 0.5 : -0.5;
            w[3 * o + 2] = ((o >> 2) & 1) ? 0.5 : -0.5;
        }
        t.opM2M.ensure(sizeof(double) * 8 * per);
        t.opL2L.ensure(sizeof(double) * 8 * per);
        build_ops(c, 1, 8, w, p, ncp, t.opM2M.as<double>());
        build_ops(c, 2, 8, w, p, ncp, t.opL2L.as<double>());
        t.op_class_slot.assign(kNClass, -1);
        t.opM2L.release();
        t.ops_p = p;
    }
    t.p = p;
    t.ncp = ncp;
    t.M.ensure(sizeof(double) * t.nboxes * ncp);
    t.L.ensure(sizeof(double) * t.nboxes * ncp);
    // The upward pass (P2M, M2M) needs only the boxes: it runs on the
    // auxiliary stream while the interaction lists are built on the context
    // stream; the M2L waits for both.  The direct and M2P lists are sorted
    // on the auxiliary stream after the upward pass, beside the
    // translations; the context stream waits for them before returning.
    // Same kernels, same order per buffer, so the results do not depend on
    // the overlap.
    if (!c.aux_stream) {
        LSS_HIP(hipStreamCreateWithFlags(&c.aux_stream, hipStreamNonBlocking));
        for (hipEvent_t &e : c.aux_ev) LSS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    struct StreamSwap {
        Ctx &c;
        hipStream_t saved;
        ~StreamSwap() { c.stream = saved; }
    };
    LSS_HIP(hipEventRecord(c.aux_ev[0], c.stream));
    LSS_HIP(hipStreamWaitEvent(c.aux_stream, c.aux_ev[0], 0));
    DBuf flag, ids, leaves, nleaf;
    {
        StreamSwap swap{c, c.stream};
        c.stream = c.aux_stream;
        upward_pass(c, p, ncp, flag, ids, leaves, nleaf);
        LSS_HIP(hipEventRecord(c.aux_ev[1], c.aux_stream));
    }
    build_tree_lists(c);
    LSS_HIP(hipEventRecord(c.aux_ev[2], c.stream));        // lists emitted, M2L list sorted
    {
        StreamSwap swap{c, c.stream};
        c.stream = c.aux_stream;
        LSS_HIP(hipStreamWaitEvent(c.aux_stream, c.aux_ev[2], 0));
        sort_near_lists(c);
        LSS_HIP(hipEventRecord(c.aux_ev[3], c.aux_stream));
    }
    LSS_HIP(hipStreamWaitEvent(c.stream, c.aux_ev[1], 0));
    {   // M2L operators of the classes in use not built yet
        std::vector<int> need;
        for (int cls : t.class_used)
            if (t.op_class_slot[cls] < 0) need.push_back(cls);
        if (!need.empty()) {
            int have = 0;
            for (int s : t.op_class_slot) have += s >= 0;
            t.opM2L.grow_copy(sizeof(double) * (size_t)(have + need.size()) * per, sizeof(double) * (size_t)have * per,
                              c.stream);
            std::vector<double> v(3 * need.size());
            for (size_t i = 0; i < need.size(); ++i) class_vec(need[i], &v[3 * i]);
            build_ops(c, 0, (int)need.size(), v, p, ncp, t.opM2L.as<double>() + (int64_t)have * per);
            for (size_t i = 0; i < need.size(); ++i) t.op_class_slot[need[i]] = have + (int)i;
        }
    }
    // M2L, one launch per displacement class, each at its own order: the
    // leading (p_v + 1)^2 coefficients in and out (the real layout orders them
    // by degree), p_v = m2l_order(p, K, v).  Within a class every target box
    // occurs once, so a launch has no write conflicts; the classes run in two
    // sets, one on each stream, into two accumulators (L, and L2 on the
    // auxiliary stream), so that each stream's launches fill the other's gaps;
    // L += L2 once both are done.  The sets depend only on the class sizes, so
    // every box sums its classes in a fixed order.
    struct M2LJob { int cls; int nkv; int64_t b0, n; };
    std::vector<M2LJob> jobs;
    for (int cls : t.class_used) {
        double v[3];
        class_vec(cls, v);
        const int pv = m2l_order(p, t.K, v);
        const int nkv = std::min(ncp, (int)ceil_div((int64_t)(pv + 1) * (pv + 1), kKB) * kKB);
        jobs.push_back({cls, nkv, t.class_beg[cls], t.class_end[cls] - t.class_beg[cls]});
    }
    // classes with few pairs would be one short launch each (graded meshes use
    // thousands of classes): they go to one target-major launch instead.  That
    // launch reads a class operator once per pair rather than once per tile of
    // pairs, so it pays only while the operators are small (measured: faster
    // at order 20, 441 coefficients; slower at order 26, 729)
    std::vector<M2LJob> small;
    {
        std::vector<M2LJob> big;
        const bool use_small = ncp <= kSmallMaxCoeffs;
        for (const M2LJob &j : jobs) (use_small && j.n <= kSmallClassPairs ? small : big).push_back(j);
        jobs.swap(big);
    }
    std::vector<char> on_aux(jobs.size(), 0);
    {   // largest work first to the less loaded set (ties: the class index)
        std::vector<size_t> ord(jobs.size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
        auto work = [&](size_t i) { return (double)jobs[i].n * jobs[i].nkv * jobs[i].nkv; };
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return work(a) > work(b); });
        double load[2] = {0.0, 0.0};
        for (size_t i : ord) {
            const int side = load[1] < load[0] ? 1 : 0;
            on_aux[i] = (char)side;
            load[side] += work(i);
        }
    }
    t.L2.ensure(sizeof(double) * t.nboxes * ncp);
    LSS_HIP(hipEventRecord(c.aux_ev[4], c.stream));         // operators built
    auto m2l = [&](const M2LJob &j, double *L) {
        GemmArgs a{G_LIST, ncp, j.nkv, j.n, t.opM2L.as<double>() + (int64_t)t.op_class_slot[j.cls] * per, t.M.as<double>(),
                   L, t.m2l_key2.as<uint64_t>() + j.b0, t.m2l_val2.as<int32_t>() + j.b0, 0,
                   t.parent.as<int32_t>(), t.level.as<int32_t>(), t.root.as<double>(), t.bmesh.as<int32_t>(), j.nkv};
        gemm(c, a);
    };
    {
        StreamSwap swap{c, c.stream};
        c.stream = c.aux_stream;
        LSS_HIP(hipStreamWaitEvent(c.aux_stream, c.aux_ev[4], 0));
        launch_fill_zero(c, t.L2.as<double>(), t.nboxes * (int64_t)ncp);
        for (size_t i = 0; i < jobs.size(); ++i)
            if (on_aux[i]) m2l(jobs[i], t.L2.as<double>());
        LSS_HIP(hipEventRecord(c.aux_ev[5], c.aux_stream));
    }
    if (!small.empty()) {
        // host arrays kept in the tree until the next build: the copies below
        // are asynchronous
        std::vector<int64_t> &hb = t.sm_hb, &ho = t.sm_ho;
        std::vector<int32_t> &hc = t.sm_hc, &hslot = t.sm_hslot, &hnkv = t.sm_hnkv;
        hb.assign(small.size(), 0);
        ho.assign(small.size() + 1, 0);
        hc.assign(small.size(), 0);
        hslot.assign(kNClass, 0);
        hnkv.assign(kNClass, 0);
        for (size_t i = 0; i < small.size(); ++i) {
            hb[i] = small[i].b0;
            hc[i] = small[i].cls;
            ho[i + 1] = ho[i] + small[i].n;
            hslot[small[i].cls] = t.op_class_slot[small[i].cls];
            hnkv[small[i].cls] = small[i].nkv;
        }
        const int64_t nsp = ho.back();
        const size_t ns = small.size();
        t.sm_meta.ensure(sizeof(int64_t) * (2 * ns + 1) + sizeof(int32_t) * (ns + 2 * kNClass));
        char *mp = t.sm_meta.as<char>();
        int64_t *db = reinterpret_cast<int64_t *>(mp), *dofs = db + ns;
        int32_t *dc = reinterpret_cast<int32_t *>(dofs + ns + 1), *dslot = dc + ns, *dnkv = dslot + kNClass;
        LSS_HIP(hipMemcpyAsync(db, hb.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(dofs, ho.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(dc, hc.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(dslot, hslot.data(), sizeof(int32_t) * kNClass, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(dnkv, hnkv.data(), sizeof(int32_t) * kNClass, hipMemcpyHostToDevice, c.stream));
        t.sm_key.ensure(8 * nsp); t.sm_key2.ensure(8 * nsp); t.sm_val.ensure(4 * nsp); t.sm_val2.ensure(4 * nsp);
        hipLaunchKernelGGL(k_small_pairs, dim3((unsigned)ns), dim3(kBlk), 0, c.stream, db, dofs, dc,
                           t.m2l_key2.as<uint64_t>(), t.m2l_val2.as<int32_t>(), t.sm_key.as<uint64_t>(),
                           t.sm_val.as<int32_t>());
        LSS_CHECK_LAUNCH("k_small_pairs");
        int tb = 1;
        while ((int64_t(1) << tb) < t.nboxes) ++tb;
        // own sort workspace: the near lists may be sorted on the other stream meanwhile
        const size_t stb = sort_pairs_u64_tmp_bytes(nsp);
        t.sm_tmp.ensure(stb);
        sort_pairs_u64(t.sm_tmp.p, stb, t.sm_key.as<uint64_t>(), t.sm_key2.as<uint64_t>(), t.sm_val.as<int32_t>(),
                       t.sm_val2.as<int32_t>(), nsp, 0, 12 + tb, c.stream);
        const int64_t gs = std::min<int64_t>(nsp, 65535);
        hipLaunchKernelGGL(k_m2l_small, dim3((unsigned)gs), dim3(256), sizeof(double) * (size_t)ncp, c.stream, nsp,
                           t.sm_key2.as<uint64_t>(), t.sm_val2.as<int32_t>(), dslot, dnkv, t.opM2L.as<double>(),
                           t.M.as<double>(), t.L.as<double>(), ncp, Geo{t.root.as<double>(), t.bmesh.as<int32_t>()},
                           t.level.as<int32_t>());
        LSS_CHECK_LAUNCH("k_m2l_small");
    }
    for (size_t i = 0; i < jobs.size(); ++i)
        if (!on_aux[i]) m2l(jobs[i], t.L.as<double>());
    LSS_HIP(hipStreamWaitEvent(c.stream, c.aux_ev[5], 0));
    launch_add(c, t.L.as<double>(), t.L2.as<double>(), t.nboxes * (int64_t)ncp);
    // downward pass: L2L from level 0 to depth-1 into their children
    for (int lvl = 1; lvl <= t.depth; ++lvl) {
        const int64_t base = t.level_begin[lvl], npar = (t.level_begin[lvl + 1] - base) / 8;
        GemmArgs a{G_L2L, ncp, ncp, npar, t.opL2L.as<double>(), t.L.as<double>(), t.L.as<double>(), nullptr, nullptr,
                   base, t.parent.as<int32_t>(), t.level.as<int32_t>(), t.root.as<double>(), t.bmesh.as<int32_t>()};
        gemm(c, a);
    }
    LSS_HIP(hipStreamWaitEvent(c.stream, c.aux_ev[3], 0));   // the direct and M2P lists
    c.stats.fmm_order = p;
}

}  // namespace lss
