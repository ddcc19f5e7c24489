// Octree over the quadrature nodes, near/far interaction lists and target
// binning for the fast multipole far field (section 4.4, eq. kerdecomp:
// interactions beyond the cut radius R = cut * sigma use the Laplace double
// layer, those inside it the full kernel).
//
// Tree: the root cube holds every node (padded by 2 R_max); a box is split in
// eight when it holds more than `leaf_capacity` nodes and its children would
// still be at least 1/shrink as wide as the largest near radius R_k of its
// nodes.  All eight children are kept (empty ones too), so the leaves
// partition the root cube and any target position has a leaf.
//
// Lists: one dual-tree traversal over (target box T, source box S) pairs:
//   same level and admissible (|d|_inf >= 2, |d|^2 >= K, d = integer offset
//   of the boxes, and box gap >= R_max(S))  -> M2L(S -> T)
//   otherwise: T leaf -> direct pairs with all nodes of S;  else split the
//   non-leaf box(es) and continue.
// Every (target leaf, node) pair is covered exactly once, by a direct pair or
// by one M2L at some level.
#include <cstring>
#include <hip/hip_runtime.h>

#include <cmath>

#include "lss_internal.h"

namespace lss {

namespace {

constexpr int kBlk = 256;
constexpr int kMaxLevel = 20;     // 21-bit Morton coordinates
constexpr int kR = 7;             // class offsets in [-kR, kR]^3
constexpr int kNClass = (2 * kR + 1) * (2 * kR + 1) * (2 * kR + 1);

inline unsigned grid_for(int64_t n, int blk = kBlk) { return (unsigned)ceil_div(n > 0 ? n : 1, blk); }

__device__ inline uint64_t spread21(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

struct Root {
    double o[3];
    double inv;      // 2^21 / L0
};

__device__ inline uint64_t key21(double x, double y, double z, const Root &r) {
    double q[3] = {(x - r.o[0]) * r.inv, (y - r.o[1]) * r.inv, (z - r.o[2]) * r.inv};
    uint64_t b[3];
    for (int c = 0; c < 3; ++c) {
        double t = q[c];
        t = t != t ? 0.0 : fmin(fmax(t, 0.0), 2097151.0);
        b[c] = (uint64_t)t;
    }
    return spread21(b[0]) | (spread21(b[1]) << 1) | (spread21(b[2]) << 2);
}

__global__ void k_node_keys(int64_t n, const Src *__restrict__ src, Root r, uint64_t *keys, int32_t *idx) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    keys[k] = key21(src[k].yx, src[k].yy, src[k].yz, r);
    idx[k] = (int32_t)k;
}

__global__ void k_permute_src(int64_t n, const Src *__restrict__ in, const int32_t *__restrict__ perm, Src *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = in[perm[k]];
}

// largest near radius cut * sigma_k over the nodes of each box of a level:
// block (i, g) reduces chunk g (kRmaxChunk nodes) of box lb + i and folds it
// with an atomic max on the bits of the (positive) double
constexpr int64_t kRmaxChunk = 8192;

__global__ void k_box_rmax(int64_t lb, const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                           const Src *__restrict__ src, double cut, unsigned long long *rmax_bits) {
    __shared__ double sh[kBlk];
    const int64_t b = lb + blockIdx.x;
    const int64_t k0 = nb[b] + (int64_t)blockIdx.y * kRmaxChunk;
    const int64_t k1 = min(ne[b], k0 + kRmaxChunk);
    if (k0 >= k1) return;
    double m = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kBlk) {
        const double s2 = src[k].s2;                   // sigma = sqrt(1 / (2 s2))
        m = fmax(m, cut * sqrt(0.5 / s2));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&rmax_bits[b], (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ void k_split_flags(int64_t lb, int64_t nlev, int level, double L0, int64_t cap, double shrink,
                              const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                              const double *__restrict__ rmax, int32_t *flag, int32_t *ids) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlev) return;
    int64_t b = lb + i;
    double half = ldexp(L0, -(level + 1));      // side of the children
    int64_t cnt = ne[b] - nb[b];
    flag[i] = (cnt > cap && half * shrink >= rmax[b] && level < kMaxLevel) ? 1 : 0;
    ids[i] = (int32_t)b;
}

__device__ inline int64_t lower_bound_key(const uint64_t *keys, int64_t lo, int64_t hi, uint64_t v, int shift) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> shift) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_make_children(const int32_t *__restrict__ nsplit_dev, const int32_t *__restrict__ split,
                                int64_t child_base, int level, const uint64_t *__restrict__ keys, int32_t *lev,
                                int32_t *ijk, int64_t *nb, int64_t *ne, int32_t *child, int32_t *parent,
                                unsigned long long *maxcnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= *nsplit_dev) return;
    int32_t b = split[r];
    int64_t first = child_base + 8 * r;
    child[b] = (int32_t)first;
    const int shift = 3 * (21 - (level + 1));
    const uint64_t pre = (level == 0) ? 0 : (keys[nb[b]] >> (3 * (21 - level)));
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
        atomicMax(maxcnt, (unsigned long long)(bound[c + 1] - bound[c]));
    }
}

// ---------------------------------------------------------- dual traversal
struct DttArgs {
    const int32_t *lev, *ijk, *child;
    const int64_t *nb, *ne;
    const double *rmax;
    double L0;
    int K;
};

__device__ inline bool is_empty(const DttArgs &a, int32_t S) { return a.ne[S] == a.nb[S]; }

// action codes
enum { A_DROP = 0, A_M2L = 1, A_P2P = 2, A_SPLIT_BOTH = 3, A_SPLIT_T = 4 };

__device__ inline int dtt_action(const DttArgs &a, int32_t T, int32_t S, int &cls) {
    if (is_empty(a, S)) return A_DROP;
    const bool leafT = a.child[T] < 0, leafS = a.child[S] < 0;
    if (T == S) return leafT ? A_P2P : A_SPLIT_BOTH;
    const int lT = a.lev[T], lS = a.lev[S];
    if (lT == lS) {
        int dx = a.ijk[3 * T] - a.ijk[3 * S], dy = a.ijk[3 * T + 1] - a.ijk[3 * S + 1], dz = a.ijk[3 * T + 2] - a.ijk[3 * S + 2];
        int m = max(abs(dx), max(abs(dy), abs(dz)));
        // admissible: K-criterion and a gap of at least the cut radius of S's nodes
        if (m >= 2 && dx * dx + dy * dy + dz * dz >= a.K && m <= kR &&
            (double)(m - 1) * ldexp(a.L0, -lT) >= a.rmax[S]) {
            cls = ((dx + kR) * (2 * kR + 1) + (dy + kR)) * (2 * kR + 1) + (dz + kR);
            return A_M2L;
        }
        if (leafT) return A_P2P;
        if (leafS) return A_SPLIT_T;
        return A_SPLIT_BOTH;
    }
    // T deeper than S (S is a leaf by construction), or the reverse
    if (leafT) return A_P2P;
    return A_SPLIT_T;
}

__global__ void k_dtt_count(int64_t n, const uint64_t *__restrict__ fr, DttArgs a, unsigned long long *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t T = (int32_t)(fr[i] >> 32), S = (int32_t)(fr[i] & 0xffffffffu);
    int cls = 0;
    int act = dtt_action(a, T, S, cls);
    if (act == A_M2L) atomicAdd(&cnt[1], 1ull);
    else if (act == A_P2P) atomicAdd(&cnt[2], 1ull);
    else if (act == A_SPLIT_BOTH) {
        // only source children that hold nodes are paired
        const int32_t s0 = a.child[S];
        unsigned long long ns = 0;
        for (int v = 0; v < 8; ++v) ns += a.ne[s0 + v] > a.nb[s0 + v] ? 1ull : 0ull;
        atomicAdd(&cnt[0], 8ull * ns);
    } else if (act == A_SPLIT_T) atomicAdd(&cnt[0], 8ull);
}

__global__ void k_dtt_emit(int64_t n, const uint64_t *__restrict__ fr, DttArgs a, unsigned long long *cnt,
                           uint64_t *next, uint64_t *m2l_key, int32_t *m2l_val, int64_t m2l_base,
                           uint64_t *p2p_key, int32_t *p2p_val, int64_t p2p_base) {
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
    } else if (act == A_SPLIT_BOTH) {
        const int32_t t0 = a.child[T], s0 = a.child[S];
        int32_t sl[8];
        int ns = 0;
        for (int v = 0; v < 8; ++v)
            if (a.ne[s0 + v] > a.nb[s0 + v]) sl[ns++] = s0 + v;
        int64_t q = (int64_t)atomicAdd(&cnt[3], 8ull * (unsigned long long)ns);
        for (int u = 0; u < 8; ++u)
            for (int v = 0; v < ns; ++v) next[q + ns * u + v] = ((uint64_t)(uint32_t)(t0 + u) << 32) | (uint32_t)sl[v];
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
// Morton key of each target (bit 63 set outside the root cube); sorting by it
// groups the targets of a leaf (a leaf is a Morton prefix range) and keeps
// every wave of a tile spatially compact.
constexpr uint64_t kOutside = 1ull << 63;

__global__ void k_locate(int64_t n_max, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
                         const double *__restrict__ ty, const double *__restrict__ tz, Root r, double L0,
                         uint64_t *keys, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    if (i >= n) {                       // unused slots sort after every real target
        keys[i] = ~0ull;
        idx[i] = (int32_t)i;
        return;
    }
    double q[3] = {(tx[i] - r.o[0]) / L0, (ty[i] - r.o[1]) / L0, (tz[i] - r.o[2]) / L0};
    bool inside = q[0] >= 0.0 && q[0] < 1.0 && q[1] >= 0.0 && q[1] < 1.0 && q[2] >= 0.0 && q[2] < 1.0;
    keys[i] = inside ? key21(tx[i], ty[i], tz[i], r) : kOutside;
    idx[i] = (int32_t)i;
}

// leaf of each sorted target (nboxes outside the root, -1 for unused slots)
__global__ void k_sorted_leaf(int64_t n_max, const int32_t *__restrict__ n_dev, const uint64_t *__restrict__ keys,
                              const int32_t *__restrict__ child, int32_t nboxes, int32_t *leaf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    if (i >= n) { leaf[i] = -1; return; }
    const uint64_t k = keys[i];
    if (k & kOutside) { leaf[i] = nboxes; return; }
    int32_t b = 0;
    int lvl = 0;
    while (child[b] >= 0) {
        int oct = (int)((k >> (3 * (21 - (lvl + 1)))) & 7ull);
        b = child[b] + oct;
        ++lvl;
    }
    leaf[i] = b;
}

// tile heads: first target of a leaf segment and every TILE-th after it.  The
// segment of leaf b starts at the first key >= its Morton prefix.
__global__ void k_tile_flags(int64_t n_max, const int32_t *__restrict__ n_dev, const uint64_t *__restrict__ keys,
                             const int32_t *__restrict__ leaf, const int32_t *__restrict__ lev,
                             const int32_t *__restrict__ ijk, int32_t nboxes, int tile, int32_t *flag, int32_t *pos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = n_dev ? (int64_t)*n_dev : n_max;
    if (i >= n_max) return;
    pos[i] = (int32_t)i;
    if (i >= n) { flag[i] = 0; return; }
    const int32_t b = leaf[i];
    uint64_t lo_key;
    if (b >= nboxes) lo_key = kOutside;
    else {
        const int l = lev[b];
        const uint64_t pre = spread21((uint64_t)ijk[3 * b]) | (spread21((uint64_t)ijk[3 * b + 1]) << 1) |
                             (spread21((uint64_t)ijk[3 * b + 2]) << 2);
        lo_key = pre << (3 * (21 - l));
    }
    int64_t lo = 0, hi = i;           // first index with key >= lo_key
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < lo_key) lo = mid + 1; else hi = mid;
    }
    flag[i] = ((i - lo) % tile) == 0 ? 1 : 0;
}

// leaf of each target in its current order (nboxes outside the root, -1 unused)
__global__ void k_leaf_direct(int64_t n_max, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
                              const double *__restrict__ ty, const double *__restrict__ tz, Root r, double L0,
                              const int32_t *__restrict__ child, int32_t nboxes, int32_t *leaf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_dev;
    if (i >= n_max) return;
    if (i >= n) { leaf[i] = -1; return; }
    double q[3] = {(tx[i] - r.o[0]) / L0, (ty[i] - r.o[1]) / L0, (tz[i] - r.o[2]) / L0};
    bool inside = q[0] >= 0.0 && q[0] < 1.0 && q[1] >= 0.0 && q[1] < 1.0 && q[2] >= 0.0 && q[2] < 1.0;
    if (!inside) { leaf[i] = nboxes; return; }
    const uint64_t k = key21(tx[i], ty[i], tz[i], r);
    int32_t b = 0;
    int lvl = 0;
    while (child[b] >= 0) {
        b = child[b] + (int)((k >> (3 * (21 - (lvl + 1)))) & 7ull);
        ++lvl;
    }
    leaf[i] = b;
}

__global__ void k_tile_flags_runs(int64_t n_max, const int32_t *__restrict__ n_dev, const int32_t *__restrict__ leaf,
                                  int tile, int32_t *flag, int32_t *pos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_dev;
    if (i >= n_max) return;
    pos[i] = (int32_t)i;
    flag[i] = (i < n && (i == 0 || leaf[i] != leaf[i - 1] || (i % tile) == 0)) ? 1 : 0;
}

__global__ void k_soa(int64_t n, const double *__restrict__ x, double *tx, double *ty, double *tz) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tx[i] = x[3 * i];
    ty[i] = x[3 * i + 1];
    tz[i] = x[3 * i + 2];
}

Root make_root(const Tree &t) {
    Root r;
    for (int k = 0; k < 3; ++k) r.o[k] = t.origin[k];
    r.inv = 2097152.0 / t.L0;
    return r;
}

}  // namespace

// ======================================================== tree + lists
void build_tree(Ctx &c) {
    Tree &t = c.tree;
    const int64_t n = c.nnodes;
    if (c.nmesh > 1) throw Error{LSS_EINVAL, "far_field = LSS_FAR_FMM supports one mesh per context"};
    const double cut = c.opt.cut_factor > 0 ? c.opt.cut_factor : (c.opt.precision == LSS_MIXED ? kCutMixed : kCutFP64);
    const int64_t cap = c.opt.leaf_capacity > 0 ? c.opt.leaf_capacity : (c.opt.precision == LSS_MIXED ? 256 : 128);
    const double shrink = c.opt.leaf_shrink > 0 ? c.opt.leaf_shrink : (c.opt.precision == LSS_MIXED ? 1.0 : 2.0);
    t.K = c.opt.precision == LSS_MIXED ? 4 : 8;
    // root cube: node bounding box padded by 2 R_max on every side
    double rmax = cut * c.sigma_max, ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = fmax(ext, c.bbox_hi[k] - c.bbox_lo[k]);
    t.L0 = ext + 4.0 * rmax;
    t.L0 *= 1.0 + 1e-9;
    for (int k = 0; k < 3; ++k) t.origin[k] = 0.5 * (c.bbox_lo[k] + c.bbox_hi[k]) - 0.5 * t.L0;
    Root root = make_root(t);
    // nodes in Morton order
    t.key.ensure(8 * n); t.key2.ensure(8 * n); t.perm.ensure(4 * n); t.perm2.ensure(4 * n);
    hipLaunchKernelGGL(k_node_keys, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, c.src.as<Src>(), root,
                       t.key.as<uint64_t>(), t.perm.as<int32_t>());
    LSS_CHECK_LAUNCH("k_node_keys");
    sort_pairs(c, t.key.as<uint64_t>(), t.key2.as<uint64_t>(), t.perm.as<int32_t>(), t.perm2.as<int32_t>(), n, 63);
    t.src.ensure(sizeof(Src) * n);
    hipLaunchKernelGGL(k_permute_src, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, c.src.as<Src>(),
                       t.perm2.as<int32_t>(), t.src.as<Src>());
    LSS_CHECK_LAUNCH("k_permute_src");
    const uint64_t *keys = t.key2.as<uint64_t>();
    // level 0
    int64_t cap_boxes = 1024;
    auto grow = [&](int64_t need, int64_t have) {
        if (need <= cap_boxes && t.level.p) return;
        int64_t nc = need > cap_boxes ? need + need / 2 : cap_boxes;
        t.level.grow_copy(4 * nc, 4 * have, c.stream);
        t.ijk.grow_copy(12 * nc, 12 * have, c.stream);
        t.nb.grow_copy(8 * nc, 8 * have, c.stream);
        t.ne.grow_copy(8 * nc, 8 * have, c.stream);
        t.child.grow_copy(4 * nc, 4 * have, c.stream);
        t.parent.grow_copy(4 * nc, 4 * have, c.stream);
        t.rmax.grow_copy(8 * nc, 8 * have, c.stream);
        cap_boxes = nc;
    };
    t.level.release(); t.ijk.release(); t.nb.release(); t.ne.release(); t.child.release(); t.parent.release();
    t.rmax.release();
    grow(1024, 0);
    {
        int32_t lv = 0, ij[3] = {0, 0, 0}, ch = -1, pa = -1;
        int64_t b0 = 0, e0 = n;
        LSS_HIP(hipMemcpyAsync(t.level.p, &lv, 4, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(t.ijk.p, ij, 12, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(t.nb.p, &b0, 8, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(t.ne.p, &e0, 8, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(t.child.p, &ch, 4, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipMemcpyAsync(t.parent.p, &pa, 4, hipMemcpyHostToDevice, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
    }
    t.level_begin.assign({0, 1});
    DBuf flag, ids, split, nsplit;
    int64_t maxcnt = n;                     // largest node count of a box of the current level
    for (int lvl = 0;; ++lvl) {
        int64_t lb = t.level_begin[lvl], le = t.level_begin[lvl + 1], nl = le - lb;
        LSS_HIP(hipMemsetAsync(t.rmax.as<double>() + lb, 0, sizeof(double) * nl, c.stream));
        const unsigned gy = (unsigned)ceil_div(maxcnt > 0 ? maxcnt : 1, kRmaxChunk);
        hipLaunchKernelGGL(k_box_rmax, dim3((unsigned)nl, gy), dim3(kBlk), 0, c.stream, lb, t.nb.as<int64_t>(),
                           t.ne.as<int64_t>(), t.src.as<Src>(), cut, reinterpret_cast<unsigned long long *>(t.rmax.p));
        LSS_CHECK_LAUNCH("k_box_rmax");
        flag.ensure(4 * nl); ids.ensure(4 * nl); split.ensure(4 * nl); nsplit.ensure(16);
        hipLaunchKernelGGL(k_split_flags, dim3(grid_for(nl)), dim3(kBlk), 0, c.stream, lb, nl, lvl, t.L0, cap, shrink,
                           t.nb.as<int64_t>(), t.ne.as<int64_t>(), t.rmax.as<double>(), flag.as<int32_t>(),
                           ids.as<int32_t>());
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
                           split.as<int32_t>(), child_base, lvl, keys, t.level.as<int32_t>(), t.ijk.as<int32_t>(),
                           t.nb.as<int64_t>(), t.ne.as<int64_t>(), t.child.as<int32_t>(), t.parent.as<int32_t>(), mc);
        LSS_CHECK_LAUNCH("k_make_children");
        unsigned long long hm = 0;
        LSS_HIP(hipMemcpyAsync(&hm, mc, 8, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        maxcnt = (int64_t)hm;
        t.level_begin.push_back(le + 8 * (int64_t)ns);
    }
    t.nboxes = t.level_begin.back();
    // ---------------------------------------------------- dual traversal
    DttArgs a{t.level.as<int32_t>(), t.ijk.as<int32_t>(), t.child.as<int32_t>(), t.nb.as<int64_t>(),
              t.ne.as<int64_t>(), t.rmax.as<double>(), t.L0, t.K};
    t.cnt.ensure(8 * 8);
    int64_t nfr = 1;
    t.fr.ensure(8 * 64);
    {
        uint64_t rr = 0;
        LSS_HIP(hipMemcpyAsync(t.fr.p, &rr, 8, hipMemcpyHostToDevice, c.stream));
    }
    t.n_m2l = 0;
    t.n_p2p = 0;
    int64_t cap_m2l = 0, cap_p2p = 0;
    while (nfr > 0) {
        LSS_HIP(hipMemsetAsync(t.cnt.p, 0, 8 * 8, c.stream));
        hipLaunchKernelGGL(k_dtt_count, dim3(grid_for(nfr)), dim3(kBlk), 0, c.stream, nfr, t.fr.as<uint64_t>(), a,
                           t.cnt.as<unsigned long long>());
        LSS_CHECK_LAUNCH("k_dtt_count");
        unsigned long long h[3];
        LSS_HIP(hipMemcpyAsync(h, t.cnt.p, 24, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        const int64_t npush = (int64_t)h[0], nm = (int64_t)h[1], np2 = (int64_t)h[2];
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
                           t.m2l_val.as<int32_t>(), t.n_m2l, t.p2p_key.as<uint64_t>(), t.p2p_val.as<int32_t>(), t.n_p2p);
        LSS_CHECK_LAUNCH("k_dtt_emit");
        t.n_m2l += nm;
        t.n_p2p += np2;
        std::swap(t.fr.p, t.fr2.p);
        std::swap(t.fr.bytes, t.fr2.bytes);
        nfr = npush;
    }
    // sort the lists; per-box direct ranges and per-class M2L segments
    t.p2p_key2.ensure(8 * (t.n_p2p + 1)); t.p2p_val2.ensure(4 * (t.n_p2p + 1));
    sort_pairs(c, t.p2p_key.as<uint64_t>(), t.p2p_key2.as<uint64_t>(), t.p2p_val.as<int32_t>(),
               t.p2p_val2.as<int32_t>(), t.n_p2p);
    t.p2p_beg.ensure(4 * (t.nboxes + 1)); t.p2p_end.ensure(4 * (t.nboxes + 1));
    LSS_HIP(hipMemsetAsync(t.p2p_beg.p, 0, 4 * (t.nboxes + 1), c.stream));
    LSS_HIP(hipMemsetAsync(t.p2p_end.p, 0, 4 * (t.nboxes + 1), c.stream));
    if (t.n_p2p > 0)
        hipLaunchKernelGGL(k_p2p_ranges, dim3(grid_for(t.n_p2p)), dim3(kBlk), 0, c.stream, t.n_p2p,
                           t.p2p_key2.as<uint64_t>(), t.p2p_beg.as<int32_t>(), t.p2p_end.as<int32_t>());
    t.m2l_key2.ensure(8 * (t.n_m2l + 1)); t.m2l_val2.ensure(4 * (t.n_m2l + 1));
    sort_pairs(c, t.m2l_key.as<uint64_t>(), t.m2l_key2.as<uint64_t>(), t.m2l_val.as<int32_t>(),
               t.m2l_val2.as<int32_t>(), t.n_m2l);
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
    c.stats.n_leaves = 0;
    c.stats.tree_depth = t.depth;
    c.stats.n_m2l = t.n_m2l;
}

void launch_soa(Ctx &c, const double *x, int64_t n, double *tx, double *ty, double *tz) {
    hipLaunchKernelGGL(k_soa, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, n, x, tx, ty, tz);
    LSS_CHECK_LAUNCH("k_soa");
}

void launch_locate_targets(Ctx &c, int64_t n_max, const int32_t *n_dev, const double *tx, const double *ty,
                           const double *tz, uint64_t *keys, int32_t *idx) {
    Tree &t = c.tree;
    hipLaunchKernelGGL(k_locate, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, tx, ty, tz,
                       make_root(t), t.L0, keys, idx);
    LSS_CHECK_LAUNCH("k_locate");
}

// leaf of every sorted target, tile starts over the sorted list and their
// count on the device
int64_t build_tiles(Ctx &c, int64_t n_max, const int32_t *n_dev, const uint64_t *sorted_keys, int tile,
                    int32_t *sorted_leaf, int32_t *tile_start, int32_t *ntiles_dev) {
    Tree &t = c.tree;
    DBuf &fl = c.tflag, &pos = c.tpos;
    fl.ensure(4 * (n_max + 1));
    pos.ensure(4 * (n_max + 1));
    hipLaunchKernelGGL(k_sorted_leaf, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, sorted_keys,
                       t.child.as<int32_t>(), (int32_t)t.nboxes, sorted_leaf);
    LSS_CHECK_LAUNCH("k_sorted_leaf");
    hipLaunchKernelGGL(k_tile_flags, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, sorted_keys,
                       sorted_leaf, t.level.as<int32_t>(), t.ijk.as<int32_t>(), (int32_t)t.nboxes, tile,
                       fl.as<int32_t>(), pos.as<int32_t>());
    LSS_CHECK_LAUNCH("k_tile_flags");
    compact_flags(c, n_max, nullptr, fl.as<int32_t>(), pos.as<int32_t>(), tile_start, ntiles_dev);
    return n_max;
}

// Newton targets keep the order of their chart points (sorted once by Morton
// key): each iteration finds the leaf of every active target in place and
// starts a tile wherever the leaf changes or TILE targets have been taken.
// No sort, no host synchronisation, no allocation: safe under stream capture
// once the buffers have been sized by ensure_tiles.
void ensure_tiles(Ctx &c, int64_t n_max) {
    c.tflag.ensure(4 * (n_max + 1));
    c.tpos.ensure(4 * (n_max + 1));
    c.tstart.ensure(4 * (n_max + 1));
    c.tleaf.ensure(4 * (n_max + 1));
    c.ntiles.ensure(16);
    c.ns.blocksum.ensure(sizeof(int32_t) * (ceil_div(n_max > 0 ? n_max : 1, 1024) + 4));
}

void build_tiles_unsorted(Ctx &c, int64_t n_max, const int32_t *n_dev, int tile) {
    Tree &t = c.tree;
    int32_t *leaf = c.tleaf.as<int32_t>();
    hipLaunchKernelGGL(k_leaf_direct, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, c.tx.as<double>(),
                       c.ty.as<double>(), c.tz.as<double>(), make_root(t), t.L0, t.child.as<int32_t>(),
                       (int32_t)t.nboxes, leaf);
    LSS_CHECK_LAUNCH("k_leaf_direct");
    hipLaunchKernelGGL(k_tile_flags_runs, dim3(grid_for(n_max)), dim3(kBlk), 0, c.stream, n_max, n_dev, leaf, tile,
                       c.tflag.as<int32_t>(), c.tpos.as<int32_t>());
    LSS_CHECK_LAUNCH("k_tile_flags_runs");
    compact_flags(c, n_max, n_dev, c.tflag.as<int32_t>(), c.tpos.as<int32_t>(), c.tstart.as<int32_t>(),
                  c.ntiles.as<int32_t>());
}

}  // namespace lss
