// Octree over the quadrature nodes, near/far interaction lists and target
// binning for the fast multipole far field (section 4.4, eq. kerdecomp:
// interactions beyond the cut radius R = cut * sigma use the Laplace double
// layer, those inside it the full kernel).
//
// Tree: a forest with one root cube per mesh, holding that mesh's nodes
// (padded by 2 R_max); a box is split in eight when more than
// `leaf_capacity` of its nodes have near radii R_k at most shrink times the
// children's side (on a smoothly graded mesh: when the children would still
// be at least 1/shrink as wide as the box's largest R_k; where fine and coarse
// triangles meet, the fine nodes still reach leaves of their own scale and
// the box's largest R_k only governs the admissibility).  All eight children are
// kept (empty ones too), so the leaves partition each root cube and any target
// position has a leaf.  Node and target keys carry the mesh id above the
// Morton bits, so a sort groups them by mesh first; meshes never interact.
//
// Lists: one dual-tree traversal over (target box T, source box S) pairs:
//   same level and admissible (|d|_inf >= 2, |d|^2 >= K, d = integer offset
//   of the boxes, and Euclidean box gap >= R_max(S))  -> M2L(S -> T)
//   otherwise: T leaf -> direct pairs with all nodes of S, unless S is not a
//   leaf and holds more than kDirectMax nodes: then S is split against the
//   leaf T; a deeper S whose centre is at least sqrt(K) of its sides away from
//   T's box and whose gap to it is at least R_max(S) is evaluated at T's
//   targets from its multipole expansion (M2P);  else split the non-leaf
//   box(es) and continue.
// Every (target leaf, node) pair is covered exactly once, by a direct pair, by
// one M2L at some level, or by one M2P.  Without the M2P descent a coarse leaf
// (an empty box next to the surface, say) would sum millions of nodes directly.
#include <cstring>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lss_internal.h"

namespace lss {

namespace {

constexpr int kBlk = 256;
constexpr int kR = 7;             // class offsets in [-kR, kR]^3
constexpr int kNClass = (2 * kR + 1) * (2 * kR + 1) * (2 * kR + 1);

// bits that hold every value below n (radix sorts skip the bits above)
inline int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

inline unsigned grid_for(int64_t n, int blk = kBlk) { return (unsigned)ceil_div(n > 0 ? n : 1, blk); }

__device__ inline uint64_t spread21(uint64_t x) { return tree_spread21(x); }

__device__ inline uint64_t point_key(double x, double y, double z, int32_t m, const double *__restrict__ root,
                                     int bits, bool &inside) {
    return tree_point_key(x, y, z, m, root, bits, inside);
}

__device__ inline int32_t mesh_of_node(int64_t k, const int64_t *__restrict__ node_off, int32_t nmesh) {
    int32_t lo = 0, hi = nmesh;                 // last m with node_off[m] <= k
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (node_off[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_node_keys(int64_t n, const Src *__restrict__ src, const int64_t *__restrict__ node_off,
                            int32_t nmesh, const double *__restrict__ root, int bits, uint64_t *keys, int32_t *idx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    bool inside;
    keys[k] = point_key(src[k].yx, src[k].yy, src[k].yz, mesh_of_node(k, node_off, nmesh), root, bits, inside);
    idx[k] = (int32_t)k;
}

// per-mesh bounding boxes of the nodes: block (m, g) reduces chunk g of mesh
// m; min / max fold through an order-preserving map of the doubles to u64
constexpr int64_t kBoxChunk = 16384;

// Leaves stop splitting at a side in [R, 2R) of their largest near radius
// R, so the direct pairs per target grow with (side / R)^2.  Enlarging a
// root cube by 2^phi (phi in [0, 1)) shifts every side; the histogram of
// frac(log2(L0 / R_k)) per mesh lets the host pick the phi that brings the
// sides closest to R.
constexpr int kPhiBins = 64;

__global__ void k_radius_hist(int64_t n, const Src *__restrict__ src, const int64_t *__restrict__ node_off,
                              int32_t nmesh, const double *__restrict__ L0, double cut, unsigned int *hist) {
    // per-block histogram in LDS (the block's nodes are contiguous, so they
    // belong to few meshes: a block folds one mesh at a time)
    __shared__ unsigned int h[kPhiBins];
    __shared__ int32_t mesh_lo, mesh_hi;
    const int64_t k0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t k = k0 + threadIdx.x;
    if (threadIdx.x == 0) {
        mesh_lo = mesh_of_node(k0, node_off, nmesh);
        mesh_hi = mesh_of_node(min(k0 + (int64_t)blockDim.x, n) - 1, node_off, nmesh);
    }
    __syncthreads();
    const int32_t m = k < n ? mesh_of_node(k, node_off, nmesh) : -1;
    int b = -1;
    if (k < n) {
        const double R = cut * sqrt(0.5 / src[k].s2);
        const double t = log2(L0[m] / R);
        b = (int)floor((t - floor(t)) * kPhiBins);
        b = b < 0 ? 0 : (b >= kPhiBins ? kPhiBins - 1 : b);
    }
    for (int32_t mm = mesh_lo; mm <= mesh_hi; ++mm) {
        for (int i = threadIdx.x; i < kPhiBins; i += blockDim.x) h[i] = 0u;
        __syncthreads();
        if (m == mm) atomicAdd(&h[b], 1u);
        __syncthreads();
        for (int i = threadIdx.x; i < kPhiBins; i += blockDim.x)
            if (h[i]) atomicAdd(&hist[(int64_t)mm * kPhiBins + i], h[i]);
        __syncthreads();
    }
}

__device__ inline unsigned long long ordered_bits(double d) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ void k_mesh_bbox(const int64_t *__restrict__ node_off, const Src *__restrict__ src,
                            unsigned long long *lo, unsigned long long *hi) {
    __shared__ unsigned long long sl[3][kBlk], sh[3][kBlk];
    const int m = blockIdx.x;
    const int64_t k0 = node_off[m] + (int64_t)blockIdx.y * kBoxChunk;
    const int64_t k1 = min(node_off[m + 1], k0 + kBoxChunk);
    if (k0 >= k1) return;
    unsigned long long a[3] = {~0ull, ~0ull, ~0ull}, b[3] = {0, 0, 0};
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kBlk) {
        const double y[3] = {src[k].yx, src[k].yy, src[k].yz};
        for (int c = 0; c < 3; ++c) {
            const unsigned long long u = ordered_bits(y[c]);
            a[c] = u < a[c] ? u : a[c];
            b[c] = u > b[c] ? u : b[c];
        }
    }
    for (int c = 0; c < 3; ++c) { sl[c][threadIdx.x] = a[c]; sh[c][threadIdx.x] = b[c]; }
    __syncthreads();
    for (int st = kBlk / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int c = 0; c < 3; ++c) {
                const unsigned long long u = sl[c][threadIdx.x + st], v = sh[c][threadIdx.x + st];
                sl[c][threadIdx.x] = u < sl[c][threadIdx.x] ? u : sl[c][threadIdx.x];
                sh[c][threadIdx.x] = v > sh[c][threadIdx.x] ? v : sh[c][threadIdx.x];
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        atomicMin(&lo[3 * m + threadIdx.x], sl[threadIdx.x][0]);
        atomicMax(&hi[3 * m + threadIdx.x], sh[threadIdx.x][0]);
    }
}

__global__ void k_permute_src(int64_t n, const Src *__restrict__ in, const int32_t *__restrict__ perm, Src *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = in[perm[k]];
}

// largest near radius cut * sigma_k over the nodes of each box of a level,
// and how many of its nodes have a radius that the box's children could
// carry (R_k <= child side * shrink): block (i, g) reduces chunk g
// (kRmaxChunk nodes) of box lb + i and folds it with an atomic max on the bits
// of the (positive) double and an atomic add of the count
constexpr int64_t kRmaxChunk = 8192;

__global__ void k_box_rmax(int64_t lb, const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                           const Src *__restrict__ src, double cut, const double *__restrict__ root,
                           const int32_t *__restrict__ bmesh, int level, double shrink,
                           unsigned long long *rmax_bits, unsigned long long *fit) {
    __shared__ double sh[kBlk];
    __shared__ unsigned long long shc[kBlk];
    const int64_t b = lb + blockIdx.x;
    const int64_t k0 = nb[b] + (int64_t)blockIdx.y * kRmaxChunk;
    const int64_t k1 = min(ne[b], k0 + kRmaxChunk);
    if (k0 >= k1) return;
    const double cs = box_side(root, bmesh, (int32_t)b, level + 1) * shrink;   // child side * shrink
    const double lim = cs * cs / (0.5 * cut * cut);     // R_k <= cs  <=>  1 / s2 <= lim
    double m = 0.0;
    unsigned long long nf = 0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kBlk) {
        const double s2 = src[k].s2;                   // sigma = sqrt(1 / (2 s2))
        m = fmax(m, cut * sqrt(0.5 / s2));
        nf += (1.0 <= lim * s2) ? 1ull : 0ull;
    }
    sh[threadIdx.x] = m;
    shc[threadIdx.x] = nf;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
            shc[threadIdx.x] += shc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&rmax_bits[b], (unsigned long long)__double_as_longlong(sh[0]));
        atomicAdd(&fit[blockIdx.x], shc[0]);
    }
}

// A box splits when more than `cap` of its nodes have near radii its
// children can carry (and the depth allows): in a box where fine and coarse
// triangles meet (steeply graded meshes), the fine nodes still get leaves of
// their own scale, and only the few coarse nodes sit in leaves narrower than
// their cut radius.
__global__ void k_split_flags(int64_t lb, int64_t nlev, int level, int max_level, int64_t cap,
                              const unsigned long long *__restrict__ fit, int32_t *flag, int32_t *ids) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlev) return;
    flag[i] = ((int64_t)fit[i] > cap && level < max_level) ? 1 : 0;
    ids[i] = (int32_t)(lb + i);
}

__device__ inline int64_t lower_bound_key(const uint64_t *keys, int64_t lo, int64_t hi, uint64_t v, int shift) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> shift) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_make_children(const int32_t *__restrict__ nsplit_dev, const int32_t *__restrict__ split,
                                int64_t child_base, int level, int bits, const uint64_t *__restrict__ keys,
                                int32_t *lev, int32_t *ijk, int64_t *nb, int64_t *ne, int32_t *child, int32_t *parent,
                                int32_t *bmesh, unsigned long long *maxcnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= *nsplit_dev) return;
    int32_t b = split[r];
    int64_t first = child_base + 8 * r;
    child[b] = (int32_t)first;
    // the box holds nodes (it is split), so its first key carries its prefix
    // (mesh id and the cell bits of the levels above)
    const int shift = 3 * (bits - (level + 1));
    const uint64_t pre = keys[nb[b]] >> (3 * (bits - level));
    int64_t lo = nb[b], hi = ne[b];
    int64_t bound[9];
    bound[0] = lo;
    bound[8] = hi;
    for (int c = 1; c < 8; ++c) bound[c] = lower_bound_key(keys, lo, hi, (pre << 3) | (uint64_t)c, shift);
    for (int c = 0; c < 8; ++c) {
        int64_t q = first + c;
        lev[q] = level + 1;
        ijk[3 * q] = 2 * ijk[3 * b] + (c & 1);
        ijk[3 * q + 1] = 2 * ijk[3 * b + 1] + ((c >> 1) & 1);
        ijk[3 * q + 2] = 2 * ijk[3 * b + 2] + ((c >> 2) & 1);
        nb[q] = bound[c];
        ne[q] = bound[c + 1];
        child[q] = -1;
        parent[q] = b;
        bmesh[q] = bmesh[b];
        atomicMax(maxcnt, (unsigned long long)(bound[c + 1] - bound[c]));
    }
}

// ---------------------------------------------------------- dual traversal
struct DttArgs {
    const int32_t *lev, *ijk, *child;
    const int64_t *nb, *ne;
    const double *rmax;
    const double *root;
    const int32_t *bmesh;
    int K;
    const double *tcut;     // target-side cut radius per box, or null (source radii rmax)
};

// cut radius an interaction (T, S) must clear: the largest cut radius of the
// targets in T when the targets carry their own widths, else of S's nodes
__device__ inline double dtt_cut(const DttArgs &a, int32_t T, int32_t S) {
    return a.tcut ? a.tcut[T] : a.rmax[S];
}

__device__ inline bool is_empty(const DttArgs &a, int32_t S) { return a.ne[S] == a.nb[S]; }

// action codes
enum { A_DROP = 0, A_M2L = 1, A_P2P = 2, A_SPLIT_BOTH = 3, A_SPLIT_T = 4, A_SPLIT_S = 5, A_M2P = 6 };

// a non-leaf source box with more nodes than this is split against a leaf target
constexpr int64_t kDirectMax = 2048;

__device__ inline void box_bounds(const DttArgs &a, int32_t b, double lo[3], double &side) {
    side = box_side(a.root, a.bmesh, b, a.lev[b]);
    const double *o = a.root + 4 * a.bmesh[b];
    for (int d = 0; d < 3; ++d) lo[d] = o[d] + a.ijk[3 * b + d] * side;
}

// M2P of the (smaller) box S at the targets of box T: S's centre at least
// sqrt(K) sides of S from T's box, and a gap of at least the cut radius of
// S's nodes between the boxes
__device__ inline bool m2p_ok(const DttArgs &a, int32_t T, int32_t S) {
    double lt[3], ls[3], ht, hs;
    box_bounds(a, T, lt, ht);
    box_bounds(a, S, ls, hs);
    double dc = 0.0, gap = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double c = ls[d] + 0.5 * hs;
        const double e = fmax(fmax(lt[d] - c, c - (lt[d] + ht)), 0.0);     // centre of S to T's box
        const double g = fmax(fmax(lt[d] - (ls[d] + hs), ls[d] - (lt[d] + ht)), 0.0);   // box to box
        dc += e * e;
        gap += g * g;
    }
    const double r = dtt_cut(a, T, S);
    return dc >= (double)a.K * hs * hs && gap >= r * r;
}

__device__ inline int64_t box_nodes(const DttArgs &a, int32_t b) { return a.ne[b] - a.nb[b]; }

__device__ inline int dtt_action(const DttArgs &a, int32_t T, int32_t S, int &cls) {
    if (is_empty(a, S)) return A_DROP;
    const bool leafT = a.child[T] < 0, leafS = a.child[S] < 0;
    if (T == S) return leafT ? A_P2P : A_SPLIT_BOTH;
    const int lT = a.lev[T], lS = a.lev[S];
    if (lT == lS) {
        int dx = a.ijk[3 * T] - a.ijk[3 * S], dy = a.ijk[3 * T + 1] - a.ijk[3 * S + 1], dz = a.ijk[3 * T + 2] - a.ijk[3 * S + 2];
        int m = max(abs(dx), max(abs(dy), abs(dz)));
        // admissible: K-criterion and a gap of at least the cut radius; the
        // gap between two equal boxes offset by d sides is side * |max(|d| - 1, 0)|
        const int gx = max(abs(dx) - 1, 0), gy = max(abs(dy) - 1, 0), gz = max(abs(dz) - 1, 0);
        const double side = box_side(a.root, a.bmesh, S, lT), cutr = dtt_cut(a, T, S);
        if (m >= 2 && dx * dx + dy * dy + dz * dz >= a.K && m <= kR &&
            (double)(gx * gx + gy * gy + gz * gz) * side * side >= cutr * cutr) {
            cls = ((dx + kR) * (2 * kR + 1) + (dy + kR)) * (2 * kR + 1) + (dz + kR);
            return A_M2L;
        }
        if (leafT) return (leafS || box_nodes(a, S) <= kDirectMax) ? A_P2P : A_SPLIT_S;
        if (leafS) return A_SPLIT_T;
        return A_SPLIT_BOTH;
    }
    if (lT > lS) return leafT ? A_P2P : A_SPLIT_T;     // T deeper than S (S is a leaf by construction)
    // S deeper than the leaf T (reached by A_SPLIT_S only)
    if (m2p_ok(a, T, S)) return A_M2P;
    return (leafS || box_nodes(a, S) <= kDirectMax) ? A_P2P : A_SPLIT_S;
}

__device__ inline int nonempty_children(const DttArgs &a, int32_t S, int32_t sl[8]) {
    const int32_t s0 = a.child[S];
    int ns = 0;
    for (int v = 0; v < 8; ++v)
        if (a.ne[s0 + v] > a.nb[s0 + v]) sl[ns++] = s0 + v;
    return ns;
}

__global__ void k_dtt_count(int64_t n, const uint64_t *__restrict__ fr, DttArgs a, unsigned long long *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t T = (int32_t)(fr[i] >> 32), S = (int32_t)(fr[i] & 0xffffffffu);
    int cls = 0;
    int act = dtt_action(a, T, S, cls);
    if (act == A_M2L) atomicAdd(&cnt[1], 1ull);
    else if (act == A_P2P) atomicAdd(&cnt[2], 1ull);
    else if (act == A_M2P) atomicAdd(&cnt[6], 1ull);
    else if (act == A_SPLIT_BOTH || act == A_SPLIT_S) {
        // only source children that hold nodes are paired
        int32_t sl[8];
        const unsigned long long ns = (unsigned long long)nonempty_children(a, S, sl);
        atomicAdd(&cnt[0], act == A_SPLIT_BOTH ? 8ull * ns : ns);
    } else if (act == A_SPLIT_T) atomicAdd(&cnt[0], 8ull);
}

__global__ void k_dtt_emit(int64_t n, const uint64_t *__restrict__ fr, DttArgs a, unsigned long long *cnt,
                           uint64_t *next, uint64_t *m2l_key, int32_t *m2l_val, int64_t m2l_base,
                           uint64_t *p2p_key, int32_t *p2p_val, int64_t p2p_base, uint64_t *m2p_key,
                           int32_t *m2p_val, int64_t m2p_base) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t T = (int32_t)(fr[i] >> 32), S = (int32_t)(fr[i] & 0xffffffffu);
    int cls = 0;
    int act = dtt_action(a, T, S, cls);
    if (act == A_M2L) {
        int64_t q = m2l_base + (int64_t)atomicAdd(&cnt[4], 1ull);
        m2l_key[q] = ((uint64_t)cls << 32) | (uint32_t)T;
        m2l_val[q] = S;
    } else if (act == A_P2P) {
        int64_t q = p2p_base + (int64_t)atomicAdd(&cnt[5], 1ull);
        p2p_key[q] = ((uint64_t)(uint32_t)T << 32) | (uint32_t)S;
        p2p_val[q] = S;
    } else if (act == A_M2P) {
        int64_t q = m2p_base + (int64_t)atomicAdd(&cnt[7], 1ull);
        m2p_key[q] = ((uint64_t)(uint32_t)T << 32) | (uint32_t)S;
        m2p_val[q] = S;
    } else if (act == A_SPLIT_BOTH) {
        const int32_t t0 = a.child[T];
        int32_t sl[8];
        const int ns = nonempty_children(a, S, sl);
        int64_t q = (int64_t)atomicAdd(&cnt[3], 8ull * (unsigned long long)ns);
        for (int u = 0; u < 8; ++u)
            for (int v = 0; v < ns; ++v) next[q + ns * u + v] = ((uint64_t)(uint32_t)(t0 + u) << 32) | (uint32_t)sl[v];
    } else if (act == A_SPLIT_S) {
        int32_t sl[8];
        const int ns = nonempty_children(a, S, sl);
        int64_t q = (int64_t)atomicAdd(&cnt[3], (unsigned long long)ns);
        for (int v = 0; v < ns; ++v) next[q + v] = ((uint64_t)(uint32_t)T << 32) | (uint32_t)sl[v];
    } else if (act == A_SPLIT_T) {
        int64_t q = (int64_t)atomicAdd(&cnt[3], 8ull);
        int32_t t0 = a.child[T];
        for (int u = 0; u < 8; ++u) next[q + u] = ((uint64_t)(uint32_t)(t0 + u) << 32) | (uint32_t)S;
    }
}

// per-box [beg, end) in the sorted direct-pair list
__global__ void k_p2p_ranges(int64_t n, const uint64_t *__restrict__ keys, int32_t *beg, int32_t *end) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t T = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != T) beg[T] = (int32_t)i;
    if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != T) end[T] = (int32_t)(i + 1);
}

// class segments of the sorted M2L list
__global__ void k_class_ranges(int64_t n, const uint64_t *__restrict__ keys, int64_t *beg, int64_t *end) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != c) beg[c] = i;
    if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != c) end[c] = i + 1;
}

// ----------------------------------------------------------- targets
// Key of each target: mesh id and Morton cell in that mesh's root cube, or
// bit 63 plus the mesh id outside the cube; sorting by it groups the targets
// of a leaf (a leaf is a key prefix range) and keeps every wave of a tile
// spatially compact.  A target's leaf is nboxes + m outside mesh m's cube.
constexpr uint64_t kOutside = 1ull << 63;

__device__ inline int32_t descend(uint64_t k, int32_t m, int bits, const int32_t *__restrict__ child) {
    int32_t b = m;
    int lvl = 0;
    while (child[b] >= 0) {
        b = child[b] + (int)((k >> (3 * (bits - (lvl + 1)))) & 7ull);
        ++lvl;
    }
    return b;
}

__global__ void k_locate(int64_t n_max, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
                         const double *__restrict__ ty, const double *__restrict__ tz,
                         const int32_t *__restrict__ tmesh, const double *__restrict__ root, int bits,
                         uint64_t *keys, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    if (i >= n) {                       // unused slots sort after every real target
        keys[i] = ~0ull;
        idx[i] = (int32_t)i;
        return;
    }
    const int32_t m = tmesh ? tmesh[i] : 0;
    bool inside;
    const uint64_t k = point_key(tx[i], ty[i], tz[i], m, root, bits, inside);
    keys[i] = inside ? k : (kOutside | ((uint64_t)m << (3 * bits)));
    idx[i] = (int32_t)i;
}

// leaf of each sorted target (nboxes + mesh outside the root, -1 for unused slots)
__global__ void k_sorted_leaf(int64_t n_max, const int32_t *__restrict__ n_dev, const uint64_t *__restrict__ keys,
                              int bits, const int32_t *__restrict__ child, int32_t nboxes, int32_t *leaf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    if (i >= n) { leaf[i] = -1; return; }
    const uint64_t k = keys[i];
    const int32_t m = (int32_t)((k & ~kOutside) >> (3 * bits));
    leaf[i] = (k & kOutside) ? nboxes + m : descend(k, m, bits, child);
}

// tile heads: first target of a leaf segment and every TILE-th after it.  The
// segment of leaf b starts at the first key >= its key prefix.
__global__ void k_tile_flags(int64_t n_max, const int32_t *__restrict__ n_dev, const uint64_t *__restrict__ keys,
                             const int32_t *__restrict__ leaf, const int32_t *__restrict__ lev,
                             const int32_t *__restrict__ ijk, const int32_t *__restrict__ bmesh, int bits,
                             int32_t nboxes, int tile, int32_t *flag, int32_t *pos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    pos[i] = (int32_t)i;
    if (i >= n) { flag[i] = 0; return; }
    const int32_t b = leaf[i];
    uint64_t lo_key;
    if (b >= nboxes) lo_key = kOutside | ((uint64_t)(b - nboxes) << (3 * bits));
    else {
        const int l = lev[b];
        const uint64_t pre = spread21((uint64_t)ijk[3 * b]) | (spread21((uint64_t)ijk[3 * b + 1]) << 1) |
                             (spread21((uint64_t)ijk[3 * b + 2]) << 2);
        lo_key = ((uint64_t)bmesh[b] << (3 * bits)) | (pre << (3 * (bits - l)));
    }
    int64_t lo = 0, hi = i;           // first index with key >= lo_key
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < lo_key) lo = mid + 1; else hi = mid;
    }
    flag[i] = ((i - lo) % tile) == 0 ? 1 : 0;
}

// leaf of each target in its current order (nboxes + mesh outside the root, -1 unused)
__global__ void k_leaf_direct(int64_t n_max, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
                              const double *__restrict__ ty, const double *__restrict__ tz,
                              const int32_t *__restrict__ tmesh, const double *__restrict__ root, int bits,
                              const int32_t *__restrict__ child, int32_t nboxes, int32_t *leaf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_dev;
    if (i >= n_max) return;
    if (i >= n) { leaf[i] = -1; return; }
    const int32_t m = tmesh ? tmesh[i] : 0;
    bool inside;
    const uint64_t k = point_key(tx[i], ty[i], tz[i], m, root, bits, inside);
    leaf[i] = inside ? descend(k, m, bits, child) : nboxes + m;
}

// Target-side cut radii (targets with their own widths): cut * sigma(x) of
// each target folded into its leaf by an atomic max on the bits of the
// (positive) double, then into every ancestor, level by level.
__global__ void k_tcut_scatter(int64_t n, const double *__restrict__ x, const int32_t *__restrict__ xm,
                               const double *__restrict__ sig, double cut, const double *__restrict__ root, int bits,
                               const int32_t *__restrict__ child, unsigned long long *tbits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t m = xm ? xm[i] : 0;
    bool inside;
    const uint64_t k = point_key(x[3 * i], x[3 * i + 1], x[3 * i + 2], m, root, bits, inside);
    const double r = cut * sig[i];
    if (!inside || !(r > 0.0)) return;      // outside the root cube: summed directly
    atomicMax(&tbits[descend(k, m, bits, child)], (unsigned long long)__double_as_longlong(r));
}

__global__ void k_tcut_up(int64_t lb, int64_t nl, const int32_t *__restrict__ child, double *tcut) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl) return;
    const int64_t b = lb + i;
    const int32_t c0 = child[b];
    if (c0 < 0) return;
    double r = tcut[b];
    for (int k = 0; k < 8; ++k) r = fmax(r, tcut[c0 + k]);
    tcut[b] = r;
}

__global__ void k_tile_flags_runs(int64_t n_max, const int32_t *__restrict__ n_dev, const int32_t *__restrict__ leaf,
                                  int tile, int32_t *flag, int32_t *pos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_dev;
    if (i >= n_max) return;
    pos[i] = (int32_t)i;
    flag[i] = (i < n && (i == 0 || leaf[i] != leaf[i - 1] || (i % tile) == 0)) ? 1 : 0;
}

// cost of a target of every box, in node pairs: the nodes on its direct list
// plus m2p_weight per M2P box; and of every mesh's outside range
__global__ void k_near_count(int64_t nboxes, int32_t nmesh, const int32_t *__restrict__ beg,
                             const int32_t *__restrict__ end, const int32_t *__restrict__ src,
                             const int32_t *__restrict__ mbeg, const int32_t *__restrict__ mend, int64_t m2p_weight,
                             const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t *cnt) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nboxes) {
        int64_t s = 0;
        for (int32_t e = beg[b]; e < end[b]; ++e) s += ne[src[e]] - nb[src[e]];
        cnt[b] = s + m2p_weight * (int64_t)(mend[b] - mbeg[b]);
    } else if (b < nboxes + nmesh) {
        const int64_t m = b - nboxes;
        cnt[b] = ne[m] - nb[m];
    }
}

__device__ inline int cost_bucket(int64_t c) {           // 0 = most expensive
    const int lg = c > 0 ? 63 - __clzll((unsigned long long)c) : 0;
    return kCostBuckets - 1 - lg;
}

// grid-stride over the tiles (their count is on the device); per-block LDS
// histograms keep the global atomics at one per bucket per block
__global__ void k_tile_bucket_count(int64_t max_tiles, const int32_t *__restrict__ ntiles_dev,
                                    const int32_t *__restrict__ tile_start, const int32_t *__restrict__ leaf,
                                    const int64_t *__restrict__ cnt, int32_t *bucket) {
    __shared__ int32_t h[kCostBuckets];
    for (int i = threadIdx.x; i < kCostBuckets; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t nt = min((int64_t)*ntiles_dev, max_tiles);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[cost_bucket(cnt[leaf[tile_start[t]]])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kCostBuckets; i += blockDim.x)
        if (h[i]) atomicAdd(&bucket[i], h[i]);
}

// single block: offsets from the counts, counts cleared for the next use
__global__ void k_tile_bucket_scan(int32_t *bucket) {
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int i = 0; i < kCostBuckets; ++i) {
            bucket[kCostBuckets + i] = s;
            s += bucket[i];
            bucket[i] = 0;
        }
    }
}

__global__ void k_tile_bucket_scatter(int64_t max_tiles, const int32_t *__restrict__ ntiles_dev,
                                      const int32_t *__restrict__ tile_start, const int32_t *__restrict__ leaf,
                                      const int64_t *__restrict__ cnt, int32_t *bucket, int32_t *order) {
    __shared__ int32_t h[kCostBuckets], base[kCostBuckets];
    const int64_t nt = min((int64_t)*ntiles_dev, max_tiles);
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < nt; t0 += (int64_t)gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < kCostBuckets; i += blockDim.x) h[i] = 0;
        __syncthreads();
        const int64_t t = t0 + threadIdx.x;
        int bk = -1, r = 0;
        if (t < nt) {
            bk = cost_bucket(cnt[leaf[tile_start[t]]]);
            r = atomicAdd(&h[bk], 1);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kCostBuckets; i += blockDim.x)
            base[i] = h[i] ? atomicAdd(&bucket[kCostBuckets + i], h[i]) : 0;
        __syncthreads();
        if (bk >= 0) order[base[bk] + r] = (int32_t)t;
        __syncthreads();
    }
}

__global__ void k_leaf_keys(int64_t n, const int32_t *__restrict__ leaf, uint64_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = (uint64_t)(uint32_t)leaf[i];
}

__global__ void k_soa(int64_t n, const double *__restrict__ x, double *tx, double *ty, double *tz) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tx[i] = x[3 * i];
    ty[i] = x[3 * i + 1];
    tz[i] = x[3 * i + 2];
}

__global__ void k_level0(int32_t nmesh, const int64_t *__restrict__ node_off, int32_t *lev, int32_t *ijk,
                         int64_t *nb, int64_t *ne, int32_t *child, int32_t *parent, int32_t *bmesh, uint64_t *fr) {
    int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmesh) return;
    lev[m] = 0;
    ijk[3 * m] = ijk[3 * m + 1] = ijk[3 * m + 2] = 0;
    nb[m] = node_off[m];
    ne[m] = node_off[m + 1];
    child[m] = -1;
    parent[m] = -1;
    bmesh[m] = m;
    fr[m] = ((uint64_t)(uint32_t)m << 32) | (uint32_t)m;     // traversal starts at (root, root)
}

}  // namespace

// ======================================================== tree + lists
void build_tree_boxes(Ctx &c) {
    Tree &t = c.tree;
    const int64_t n = c.nnodes;
    const int32_t nm = c.nmesh;
    const double cut = c.opt.cut_factor > 0 ? c.opt.cut_factor : (c.opt.precision == LSS_MIXED ? kCutMixed : kCutFP64);
    const int64_t cap = c.opt.leaf_capacity > 0 ? c.opt.leaf_capacity : 64;
    const double shrink = c.opt.leaf_shrink > 0 ? c.opt.leaf_shrink : (c.opt.precision == LSS_MIXED ? 1.5 : 2.0);
    t.K = c.opt.admissibility > 0 ? c.opt.admissibility : (c.opt.precision == LSS_MIXED ? 4 : 7);
    // key layout: mesh id above `bits` Morton bits per dimension, bit 63 free
    int mb = 0;
    while ((int64_t(1) << mb) < nm) ++mb;
    t.bits = std::min(21, (63 - mb) / 3);
    t.nroot = nm;
    // root cube per mesh: its nodes' bounding box padded by 2 R_max on every side
    const double rmax = cut * c.sigma_max;
    std::vector<double> lo(3 * nm), hi(3 * nm);
    if (nm == 1) {
        for (int k = 0; k < 3; ++k) { lo[k] = c.bbox_lo[k]; hi[k] = c.bbox_hi[k]; }
    } else {
        DBuf bb;
        bb.ensure(sizeof(unsigned long long) * 6 * nm);
        std::vector<unsigned long long> init(6 * nm);
        for (int i = 0; i < 3 * nm; ++i) { init[i] = ~0ull; init[3 * nm + i] = 0ull; }
        LSS_HIP(hipMemcpyAsync(bb.p, init.data(), 8 * init.size(), hipMemcpyHostToDevice, c.stream));
        int64_t most = 0;
        for (int m = 0; m < nm; ++m) most = std::max(most, (c.h_tri_off[m + 1] - c.h_tri_off[m]) * c.nq);
        const unsigned gy = (unsigned)ceil_div(most > 0 ? most : 1, kBoxChunk);
        unsigned long long *ulo = bb.as<unsigned long long>(), *uhi = ulo + 3 * nm;
        hipLaunchKernelGGL(k_mesh_bbox, dim3((unsigned)nm, gy), dim3(kBlk), 0, c.stream, c.node_off.as<int64_t>(),
                           c.src.as<Src>(), ulo, uhi);
        LSS_CHECK_LAUNCH("k_mesh_bbox");
        LSS_HIP(hipMemcpyAsync(init.data(), bb.p, 8 * init.size(), hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        auto unmap = [](unsigned long long u) {
            u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
            double d;
            std::memcpy(&d, &u, 8);
            return d;
        };
        for (int i = 0; i < 3 * nm; ++i) {
            if (init[i] == ~0ull) { lo[i] = 0.0; hi[i] = 0.0; continue; }     // mesh without nodes
            lo[i] = unmap(init[i]);
            hi[i] = unmap(init[3 * nm + i]);
        }
    }
    std::vector<double> L0(nm);
    for (int m = 0; m < nm; ++m) {
        double ext = 0.0;
        for (int k = 0; k < 3; ++k) ext = fmax(ext, hi[3 * m + k] - lo[3 * m + k]);
        L0[m] = (ext + 4.0 * rmax) * (1.0 + 1e-9);
        if (!(L0[m] > 0.0)) L0[m] = 1.0;
    }
    {   // enlarge each root by the 2^phi that brings the leaf sides closest to R
        DBuf dL, dh;
        dL.ensure(sizeof(double) * nm);
        dh.ensure(sizeof(unsigned int) * kPhiBins * nm);
        LSS_HIP(hipMemcpyAsync(dL.p, L0.data(), sizeof(double) * nm, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemsetAsync(dh.p, 0, sizeof(unsigned int) * kPhiBins * nm, c.stream));
        hipLaunchKernelGGL(k_radius_hist, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, c.src.as<Src>(),
                           c.node_off.as<int64_t>(), nm, dL.as<double>(), cut, dh.as<unsigned int>());
        LSS_CHECK_LAUNCH("k_radius_hist");
        std::vector<unsigned int> hist((size_t)kPhiBins * nm);
        LSS_HIP(hipMemcpyAsync(hist.data(), dh.p, sizeof(unsigned int) * hist.size(), hipMemcpyDeviceToHost,
                               c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        for (int m = 0; m < nm; ++m) {
            double best = -1.0;
            int bj = 0;
            for (int j = 0; j < kPhiBins; ++j) {          // phi = j / bins
                double cost = 0.0;
                for (int b = 0; b < kPhiBins; ++b) {
                    const unsigned int h = hist[(size_t)m * kPhiBins + b];
                    if (!h) continue;
                    double f = (b + 0.5 + j) / kPhiBins;
                    f -= std::floor(f);
                    cost += h * std::exp2(2.0 * f);          // (side / R)^2
                }
                if (best < 0.0 || cost < best) { best = cost; bj = j; }
            }
            L0[m] *= std::exp2((double)bj / kPhiBins);
        }
    }
    t.h_root.assign(4 * nm, 0.0);
    for (int m = 0; m < nm; ++m) {
        for (int k = 0; k < 3; ++k) t.h_root[4 * m + k] = 0.5 * (lo[3 * m + k] + hi[3 * m + k]) - 0.5 * L0[m];
        t.h_root[4 * m + 3] = L0[m];
    }
    t.root.ensure(sizeof(double) * 4 * nm);
    LSS_HIP(hipMemcpyAsync(t.root.p, t.h_root.data(), sizeof(double) * 4 * nm, hipMemcpyHostToDevice, c.stream));
    // nodes in key order (mesh, then Morton)
    t.key.ensure(8 * n); t.key2.ensure(8 * n); t.perm.ensure(4 * n); t.perm2.ensure(4 * n);
    hipLaunchKernelGGL(k_node_keys, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, c.src.as<Src>(),
                       c.node_off.as<int64_t>(), nm, t.root.as<double>(), t.bits, t.key.as<uint64_t>(),
                       t.perm.as<int32_t>());
    LSS_CHECK_LAUNCH("k_node_keys");
    sort_pairs(c, t.key.as<uint64_t>(), t.key2.as<uint64_t>(), t.perm.as<int32_t>(), t.perm2.as<int32_t>(), n, 63);
    t.src.ensure(sizeof(Src) * n);
    hipLaunchKernelGGL(k_permute_src, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, c.src.as<Src>(),
                       t.perm2.as<int32_t>(), t.src.as<Src>());
    LSS_CHECK_LAUNCH("k_permute_src");
    const uint64_t *keys = t.key2.as<uint64_t>();
    // level 0: one root box per mesh
    int64_t cap_boxes = std::max<int64_t>(1024, 2 * (int64_t)nm);
    auto grow = [&](int64_t need, int64_t have) {
        if (need <= cap_boxes && t.level.p) return;
        int64_t nc = need > cap_boxes ? need + need / 2 : cap_boxes;
        t.level.grow_copy(4 * nc, 4 * have, c.stream);
        t.ijk.grow_copy(12 * nc, 12 * have, c.stream);
        t.nb.grow_copy(8 * nc, 8 * have, c.stream);
        t.ne.grow_copy(8 * nc, 8 * have, c.stream);
        t.child.grow_copy(4 * nc, 4 * have, c.stream);
        t.parent.grow_copy(4 * nc, 4 * have, c.stream);
        t.bmesh.grow_copy(4 * nc, 4 * have, c.stream);
        t.rmax.grow_copy(8 * nc, 8 * have, c.stream);
        cap_boxes = nc;
    };
    // the box arrays keep the capacity of the previous build (they grow
    // together, so the level array's capacity holds for all eight): a rebuild
    // after a change of sigma copies and reallocates nothing
    if (t.level.p) cap_boxes = std::max<int64_t>(cap_boxes, (int64_t)(t.level.bytes / sizeof(int32_t)));
    grow(cap_boxes, 0);
    t.fr.ensure(8 * std::max<int64_t>(64, nm));
    hipLaunchKernelGGL(k_level0, dim3(grid_for(nm)), dim3(kBlk), 0, c.stream, nm, c.node_off.as<int64_t>(),
                       t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.nb.as<int64_t>(), t.ne.as<int64_t>(),
                       t.child.as<int32_t>(), t.parent.as<int32_t>(), t.bmesh.as<int32_t>(), t.fr.as<uint64_t>());
    LSS_CHECK_LAUNCH("k_level0");
    t.level_begin.assign({0, (int64_t)nm});
    DBuf flag, ids, split, nsplit, fitc;
    int64_t maxcnt = 0;                     // largest node count of a box of the current level
    for (int m = 0; m < nm; ++m) maxcnt = std::max(maxcnt, (c.h_tri_off[m + 1] - c.h_tri_off[m]) * c.nq);
    for (int lvl = 0;; ++lvl) {
        int64_t lb = t.level_begin[lvl], le = t.level_begin[lvl + 1], nl = le - lb;
        LSS_HIP(hipMemsetAsync(t.rmax.as<double>() + lb, 0, sizeof(double) * nl, c.stream));
        fitc.ensure(8 * nl);
        LSS_HIP(hipMemsetAsync(fitc.p, 0, 8 * nl, c.stream));
        const unsigned gy = (unsigned)ceil_div(maxcnt > 0 ? maxcnt : 1, kRmaxChunk);
        hipLaunchKernelGGL(k_box_rmax, dim3((unsigned)nl, gy), dim3(kBlk), 0, c.stream, lb, t.nb.as<int64_t>(),
                           t.ne.as<int64_t>(), t.src.as<Src>(), cut, t.root.as<double>(), t.bmesh.as<int32_t>(), lvl,
                           shrink, reinterpret_cast<unsigned long long *>(t.rmax.p),
                           fitc.as<unsigned long long>());
        LSS_CHECK_LAUNCH("k_box_rmax");
        flag.ensure(4 * nl); ids.ensure(4 * nl); split.ensure(4 * nl); nsplit.ensure(16);
        hipLaunchKernelGGL(k_split_flags, dim3(grid_for(nl)), dim3(kBlk), 0, c.stream, lb, nl, lvl, t.bits - 1, cap,
                           fitc.as<unsigned long long>(), flag.as<int32_t>(), ids.as<int32_t>());
        LSS_CHECK_LAUNCH("k_split_flags");
        compact_flags(c, nl, nullptr, flag.as<int32_t>(), ids.as<int32_t>(), split.as<int32_t>(), nsplit.as<int32_t>());
        int32_t ns = 0;
        LSS_HIP(hipMemcpyAsync(&ns, nsplit.p, 4, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (ns == 0) { t.depth = lvl; break; }
        int64_t child_base = le;
        grow(le + 8 * (int64_t)ns, le);
        unsigned long long *mc = reinterpret_cast<unsigned long long *>(nsplit.as<int32_t>() + 2);
        LSS_HIP(hipMemsetAsync(mc, 0, 8, c.stream));
        hipLaunchKernelGGL(k_make_children, dim3(grid_for(ns)), dim3(kBlk), 0, c.stream, nsplit.as<int32_t>(),
                           split.as<int32_t>(), child_base, lvl, t.bits, keys, t.level.as<int32_t>(),
                           t.ijk.as<int32_t>(), t.nb.as<int64_t>(), t.ne.as<int64_t>(), t.child.as<int32_t>(),
                           t.parent.as<int32_t>(), t.bmesh.as<int32_t>(), mc);
        LSS_CHECK_LAUNCH("k_make_children");
        unsigned long long hm = 0;
        LSS_HIP(hipMemcpyAsync(&hm, mc, 8, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        maxcnt = (int64_t)hm;
        t.level_begin.push_back(le + 8 * (int64_t)ns);
    }
    t.nboxes = t.level_begin.back();
    // targets with their own widths: the cut radius of each box's targets
    const double *tcut = nullptr;
    if (c.target_widths && c.target_widths->n > 0) {
        const TargetWidths &tw = *c.target_widths;
        t.tcut.ensure(sizeof(double) * t.nboxes);
        LSS_HIP(hipMemsetAsync(t.tcut.p, 0, sizeof(double) * t.nboxes, c.stream));
        hipLaunchKernelGGL(k_tcut_scatter, dim3(grid_for(tw.n)), dim3(kBlk), 0, c.stream, tw.n, tw.x,
                           nm > 1 ? tw.xm : nullptr, tw.sig, cut, t.root.as<double>(), t.bits,
                           t.child.as<int32_t>(), reinterpret_cast<unsigned long long *>(t.tcut.p));
        LSS_CHECK_LAUNCH("k_tcut_scatter");
        for (int l = t.depth - 1; l >= 0; --l) {
            const int64_t lb = t.level_begin[l], nl = t.level_begin[l + 1] - lb;
            hipLaunchKernelGGL(k_tcut_up, dim3(grid_for(nl)), dim3(kBlk), 0, c.stream, lb, nl, t.child.as<int32_t>(),
                               t.tcut.as<double>());
        }
        LSS_CHECK_LAUNCH("k_tcut_up");
        tcut = t.tcut.as<double>();
    }
    t.has_tcut = tcut != nullptr;
}

// ---------------------------------------------------- dual traversal
void build_tree_lists(Ctx &c) {
    Tree &t = c.tree;
    const int32_t nm = c.nmesh;
    const double *tcut = t.has_tcut ? t.tcut.as<double>() : nullptr;
    DttArgs a{t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.child.as<int32_t>(), t.nb.as<int64_t>(),
              t.ne.as<int64_t>(), t.rmax.as<double>(), t.root.as<double>(), t.bmesh.as<int32_t>(), t.K, tcut};
    t.cnt.ensure(8 * 8);
    int64_t nfr = nm;                       // (root m, root m) pairs written by k_level0
    t.n_m2l = 0;
    t.n_p2p = 0;
    t.n_m2p = 0;
    int64_t cap_m2l = 0, cap_p2p = 0, cap_m2p = 0;
    while (nfr > 0) {
        LSS_HIP(hipMemsetAsync(t.cnt.p, 0, 8 * 8, c.stream));
        hipLaunchKernelGGL(k_dtt_count, dim3(grid_for(nfr)), dim3(kBlk), 0, c.stream, nfr, t.fr.as<uint64_t>(), a,
                           t.cnt.as<unsigned long long>());
        LSS_CHECK_LAUNCH("k_dtt_count");
        unsigned long long h[8];
        LSS_HIP(hipMemcpyAsync(h, t.cnt.p, 64, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        const int64_t npush = (int64_t)h[0], nm = (int64_t)h[1], np2 = (int64_t)h[2], nmp = (int64_t)h[6];
        if (t.n_m2p + nmp > cap_m2p) {
            int64_t nc = (t.n_m2p + nmp) * 2 + 1024;
            t.m2p_key.grow_copy(8 * nc, 8 * t.n_m2p, c.stream);
            t.m2p_val.grow_copy(4 * nc, 4 * t.n_m2p, c.stream);
            cap_m2p = nc;
        }
        if (t.n_m2l + nm > cap_m2l) {
            int64_t nc = (t.n_m2l + nm) * 2 + 1024;
            t.m2l_key.grow_copy(8 * nc, 8 * t.n_m2l, c.stream);
            t.m2l_val.grow_copy(4 * nc, 4 * t.n_m2l, c.stream);
            cap_m2l = nc;
        }
        if (t.n_p2p + np2 > cap_p2p) {
            int64_t nc = (t.n_p2p + np2) * 2 + 1024;
            t.p2p_key.grow_copy(8 * nc, 8 * t.n_p2p, c.stream);
            t.p2p_val.grow_copy(4 * nc, 4 * t.n_p2p, c.stream);
            cap_p2p = nc;
        }
        t.fr2.ensure(8 * (npush > 0 ? npush : 1));
        hipLaunchKernelGGL(k_dtt_emit, dim3(grid_for(nfr)), dim3(kBlk), 0, c.stream, nfr, t.fr.as<uint64_t>(), a,
                           t.cnt.as<unsigned long long>(), t.fr2.as<uint64_t>(), t.m2l_key.as<uint64_t>(),
                           t.m2l_val.as<int32_t>(), t.n_m2l, t.p2p_key.as<uint64_t>(), t.p2p_val.as<int32_t>(), t.n_p2p,
                           t.m2p_key.as<uint64_t>(), t.m2p_val.as<int32_t>(), t.n_m2p);
        LSS_CHECK_LAUNCH("k_dtt_emit");
        t.n_m2l += nm;
        t.n_p2p += np2;
        t.n_m2p += nmp;
        std::swap(t.fr.p, t.fr2.p);
        std::swap(t.fr.bytes, t.fr2.bytes);
        nfr = npush;
    }
    // the M2L list sorted by class; the direct and M2P lists are sorted by
    // sort_near_lists (the translations do not need them)
    t.m2l_key2.ensure(8 * (t.n_m2l + 1)); t.m2l_val2.ensure(4 * (t.n_m2l + 1));
    sort_pairs(c, t.m2l_key.as<uint64_t>(), t.m2l_key2.as<uint64_t>(), t.m2l_val.as<int32_t>(),
               t.m2l_val2.as<int32_t>(), t.n_m2l, 32 + bits_for(kNClass));
    DBuf cb, ce;
    cb.ensure(8 * kNClass); ce.ensure(8 * kNClass);
    LSS_HIP(hipMemsetAsync(cb.p, 0, 8 * kNClass, c.stream));
    LSS_HIP(hipMemsetAsync(ce.p, 0, 8 * kNClass, c.stream));
    if (t.n_m2l > 0)
        hipLaunchKernelGGL(k_class_ranges, dim3(grid_for(t.n_m2l)), dim3(kBlk), 0, c.stream, t.n_m2l,
                           t.m2l_key2.as<uint64_t>(), cb.as<int64_t>(), ce.as<int64_t>());
    LSS_CHECK_LAUNCH("list ranges");
    t.class_beg.assign(kNClass, 0);
    t.class_end.assign(kNClass, 0);
    LSS_HIP(hipMemcpyAsync(t.class_beg.data(), cb.p, 8 * kNClass, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipMemcpyAsync(t.class_end.data(), ce.p, 8 * kNClass, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    t.class_used.clear();
    for (int k = 0; k < kNClass; ++k)
        if (t.class_end[k] > t.class_beg[k]) t.class_used.push_back(k);
    c.stats.n_boxes = t.nboxes;
    c.stats.tree_depth = t.depth;
    c.stats.n_m2l = t.n_m2l;
    c.stats.n_m2p = t.n_m2p;
}

// Direct and M2P lists sorted by target box (then source box), their
// per-box ranges and each box's tile cost.  Keys are (T << 32) | S with
// T, S < nboxes + nmesh, so only the low 32 + bits(nboxes + nmesh) bits
// are sorted.
void sort_near_lists(Ctx &c) {
    Tree &t = c.tree;
    const int32_t nm = c.nmesh;
    const int kbits = 32 + bits_for(t.nboxes + nm);
    t.p2p_key2.ensure(8 * (t.n_p2p + 1)); t.p2p_val2.ensure(4 * (t.n_p2p + 1));
    sort_pairs(c, t.p2p_key.as<uint64_t>(), t.p2p_key2.as<uint64_t>(), t.p2p_val.as<int32_t>(),
               t.p2p_val2.as<int32_t>(), t.n_p2p, kbits);
    t.p2p_beg.ensure(4 * (t.nboxes + 1)); t.p2p_end.ensure(4 * (t.nboxes + 1));
    LSS_HIP(hipMemsetAsync(t.p2p_beg.p, 0, 4 * (t.nboxes + 1), c.stream));
    LSS_HIP(hipMemsetAsync(t.p2p_end.p, 0, 4 * (t.nboxes + 1), c.stream));
    if (t.n_p2p > 0)
        hipLaunchKernelGGL(k_p2p_ranges, dim3(grid_for(t.n_p2p)), dim3(kBlk), 0, c.stream, t.n_p2p,
                           t.p2p_key2.as<uint64_t>(), t.p2p_beg.as<int32_t>(), t.p2p_end.as<int32_t>());
    t.m2p_key2.ensure(8 * (t.n_m2p + 1)); t.m2p_val2.ensure(4 * (t.n_m2p + 1));
    sort_pairs(c, t.m2p_key.as<uint64_t>(), t.m2p_key2.as<uint64_t>(), t.m2p_val.as<int32_t>(),
               t.m2p_val2.as<int32_t>(), t.n_m2p, kbits);
    t.m2p_beg.ensure(4 * (t.nboxes + 1)); t.m2p_end.ensure(4 * (t.nboxes + 1));
    LSS_HIP(hipMemsetAsync(t.m2p_beg.p, 0, 4 * (t.nboxes + 1), c.stream));
    LSS_HIP(hipMemsetAsync(t.m2p_end.p, 0, 4 * (t.nboxes + 1), c.stream));
    if (t.n_m2p > 0)
        hipLaunchKernelGGL(k_p2p_ranges, dim3(grid_for(t.n_m2p)), dim3(kBlk), 0, c.stream, t.n_m2p,
                           t.m2p_key2.as<uint64_t>(), t.m2p_beg.as<int32_t>(), t.m2p_end.as<int32_t>());
    // an M2P costs about as much as (p + 2)^2 / 4 direct pairs
    const int p_est = fmm_order_for(c);
    t.near_cnt.ensure(8 * (t.nboxes + nm));
    hipLaunchKernelGGL(k_near_count, dim3(grid_for(t.nboxes + nm)), dim3(kBlk), 0, c.stream, t.nboxes, nm,
                       t.p2p_beg.as<int32_t>(), t.p2p_end.as<int32_t>(), t.p2p_val2.as<int32_t>(),
                       t.m2p_beg.as<int32_t>(), t.m2p_end.as<int32_t>(), (int64_t)(p_est + 2) * (p_est + 2) / 4,
                       t.nb.as<int64_t>(), t.ne.as<int64_t>(), t.near_cnt.as<int64_t>());
    LSS_CHECK_LAUNCH("k_near_count");
}

void build_tree(Ctx &c) {
    build_tree_boxes(c);
    build_tree_lists(c);
    sort_near_lists(c);
}

void launch_soa(Ctx &c, const double *x, int64_t n, double *tx, double *ty, double *tz) {
    hipLaunchKernelGGL(k_soa, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, x, tx, ty, tz);
    LSS_CHECK_LAUNCH("k_soa");
}

void launch_locate_targets(Ctx &c, int64_t n_max, const int32_t *n_dev, const double *tx, const double *ty,
                           const double *tz, const int32_t *tmesh, uint64_t *keys, int32_t *idx) {
    Tree &t = c.tree;
    hipLaunchKernelGGL(k_locate, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, tx, ty, tz,
                       t.nroot > 1 ? tmesh : nullptr, t.root.as<double>(), t.bits, keys, idx);
    LSS_CHECK_LAUNCH("k_locate");
}

// leaf of every sorted target, tile starts over the sorted list and their
// count on the device
int64_t build_tiles(Ctx &c, int64_t n_max, const int32_t *n_dev, const uint64_t *sorted_keys, int tile,
                    int32_t *sorted_leaf, int32_t *tile_start, int32_t *ntiles_dev, int32_t *flag, int32_t *pos,
                    int32_t *blocksum) {
    Tree &t = c.tree;
    hipLaunchKernelGGL(k_sorted_leaf, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, sorted_keys,
                       t.bits, t.child.as<int32_t>(), (int32_t)t.nboxes, sorted_leaf);
    LSS_CHECK_LAUNCH("k_sorted_leaf");
    hipLaunchKernelGGL(k_tile_flags, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, sorted_keys,
                       sorted_leaf, t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.bmesh.as<int32_t>(), t.bits,
                       (int32_t)t.nboxes, tile, flag, pos);
    LSS_CHECK_LAUNCH("k_tile_flags");
    compact_flags(c, n_max, n_dev, flag, pos, tile_start, ntiles_dev, blocksum);
    return n_max;
}

// Newton targets keep the order of their chart points (sorted once by Morton
// key): each iteration finds the leaf of every active target in place and
// starts a tile wherever the leaf changes or TILE targets have been taken.
// No sort, no host synchronisation, no allocation: safe under stream capture
// once the buffers have been sized by ensure_tiles.
void order_tiles(Ctx &c, int64_t max_tiles, const int32_t *ntiles_dev, const int32_t *tile_start,
                 const int32_t *leaf, int32_t *order) {
    Tree &t = c.tree;
    const unsigned g = grid_for(max_tiles) < 2048u ? grid_for(max_tiles) : 2048u;
    hipLaunchKernelGGL(k_tile_bucket_count, dim3(g), dim3(kBlk), 0, c.stream, max_tiles, ntiles_dev, tile_start, leaf,
                       t.near_cnt.as<int64_t>(), c.tile_bucket.as<int32_t>());
    hipLaunchKernelGGL(k_tile_bucket_scan, dim3(1), dim3(64), 0, c.stream, c.tile_bucket.as<int32_t>());
    hipLaunchKernelGGL(k_tile_bucket_scatter, dim3(g), dim3(kBlk), 0, c.stream, max_tiles, ntiles_dev, tile_start,
                       leaf, t.near_cnt.as<int64_t>(), c.tile_bucket.as<int32_t>(), order);
    LSS_CHECK_LAUNCH("order_tiles");
}

void ensure_tiles(Ctx &c, int64_t n_max) {
    c.tile_order.ensure(4 * (n_max + 1));
    c.tflag.ensure(4 * (n_max + 1));
    c.tpos.ensure(4 * (n_max + 1));
    c.tstart.ensure(4 * (n_max + 1));
    c.tleaf.ensure(4 * (n_max + 1));
    c.ntiles.ensure(16);
    c.ns.blocksum.ensure(sizeof(int32_t) * (ceil_div(n_max > 0 ? n_max : 1, 1024) + 4));
}

// Newton targets drift off their chart points, so after a step the active
// list is re-ordered by the leaf of each target's current position (stable:
// chart order within a leaf); the captured iterations then tile full leaves.
void rebin_active(Ctx &c, int64_t N, int64_t nact) {
    if (nact <= 0) return;
    NewtonState &s = c.ns;
    Tree &t = c.tree;
    launch_newton_targets(c, N);
    hipLaunchKernelGGL(k_leaf_direct, dim3(grid_for(nact)), dim3(kBlk), 0, c.stream, nact, s.nact.as<int32_t>(),
                       c.tx.as<double>(), c.ty.as<double>(), c.tz.as<double>(),
                       t.nroot > 1 ? c.tmesh.as<int32_t>() : nullptr, t.root.as<double>(), t.bits,
                       t.child.as<int32_t>(), (int32_t)t.nboxes, c.tleaf.as<int32_t>());
    hipLaunchKernelGGL(k_leaf_keys, dim3(grid_for(nact)), dim3(kBlk), 0, c.stream, nact, c.tleaf.as<int32_t>(),
                       c.tkey.as<uint64_t>());
    LSS_CHECK_LAUNCH("rebin_active");
    int bits = 1;
    while ((int64_t(1) << bits) <= t.nboxes + t.nroot) ++bits;
    sort_pairs(c, c.tkey.as<uint64_t>(), c.tkey2.as<uint64_t>(), s.active.as<int32_t>(), s.active2.as<int32_t>(), nact,
               bits);
    LSS_HIP(hipMemcpyAsync(s.active.p, s.active2.p, sizeof(int32_t) * nact, hipMemcpyDeviceToDevice, c.stream));
}

void build_tiles_unsorted(Ctx &c, int64_t n_max, const int32_t *n_dev, int tile) {
    Tree &t = c.tree;
    int32_t *leaf = c.tleaf.as<int32_t>();
    hipLaunchKernelGGL(k_leaf_direct, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, c.tx.as<double>(),
                       c.ty.as<double>(), c.tz.as<double>(), t.nroot > 1 ? c.tmesh.as<int32_t>() : nullptr,
                       t.root.as<double>(), t.bits, t.child.as<int32_t>(), (int32_t)t.nboxes, leaf);
    LSS_CHECK_LAUNCH("k_leaf_direct");
    hipLaunchKernelGGL(k_tile_flags_runs, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, leaf, tile,
                       c.tflag.as<int32_t>(), c.tpos.as<int32_t>());
    LSS_CHECK_LAUNCH("k_tile_flags_runs");
    compact_flags(c, n_max, n_dev, c.tflag.as<int32_t>(), c.tpos.as<int32_t>(), c.tstart.as<int32_t>(),
                  c.ntiles.as<int32_t>());
}

}  // namespace lss
