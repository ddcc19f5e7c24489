// Internal declarations of liblss: the context, device buffers and the
// host-side launch wrappers of the kernels.  Everything here is C++ behind
// the C ABI of include/lss.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "lss.h"

namespace lss {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};

#define LSS_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            throw ::lss::Error{e_ == hipErrorOutOfMemory ? LSS_ENOMEM : LSS_EHIP,  \
                               std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define LSS_CHECK_LAUNCH(name)                                                      \
    do {                                                                            \
        hipError_t e_ = hipGetLastError();                                          \
        if (e_ != hipSuccess)                                                       \
            throw ::lss::Error{LSS_EHIP, std::string("launch ") + (name) + ": " +   \
                                             hipGetErrorString(e_)};                \
    } while (0)

// ------------------------------------------------------------ device buffer
// Grow-only device allocation owned by the context.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void ensure(size_t nb) {
        if (nb <= bytes) return;
        release();
        size_t want = nb < 256 ? 256 : nb;
        LSS_HIP(hipMalloc(&p, want));
        bytes = want;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow keeping the first `keep` bytes (stream-ordered copy)
    void grow_copy(size_t nb, size_t keep, hipStream_t s) {
        if (nb <= bytes) return;
        void *q = nullptr;
        size_t want = nb + nb / 2;
        LSS_HIP(hipMalloc(&q, want));
        if (p && keep) LSS_HIP(hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, s));
        if (p) {
            LSS_HIP(hipStreamSynchronize(s));
            (void)hipFree(p);
        }
        p = q;
        bytes = want;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Packed quadrature-node record (one 64-byte line per node): position, the
// folded dipole vector a' = c(sigma) w J, s2 = 1/(2 sigma^2) and 2 s2.
struct alignas(64) Src {
    double yx, yy, yz, s2;
    double ax, ay, az, s2x2;
};

// Node without a width (target-attached sigma): position and a = w J.
struct RawNode {
    double yx, yy, yz, ax, ay, az;
};

// Triangle centroid and sigma_j = D_j / lambda (multiscale width, section 2).
struct Cen {
    double cx, cy, cz, sj;
};

// Target-attached width through the tree: sigma(x) and grad sigma per target
// (original order).
struct MsArgs {
    const double *sig, *gsig;
    double tcut;    // t = rho^2 / (2 sigma(x)^2) at the cut: pairs beyond it take the dipole form
};

// Targets whose own widths set the near/far split of the lists (target-
// attached sigma): AoS positions x (n,3), mesh ids (null: one mesh) and
// sigma(x).  While a context holds one, build_tree makes a box admissible for
// M2L / M2P when its gap to the source box is at least cut * sigma(x) for
// every target in it, instead of the source nodes' cut radii.
struct TargetWidths {
    const double *x;
    const int32_t *xm;
    const double *sig;
    int64_t n;
};

// FP32 staging record of the mixed path: position relative to a tile origin
// as an unevaluated float-float sum hi + lo (lo = the FP64 remainder).  The
// far-form constants are folded in: ax, ay, az hold sqrt(pi)/2 a' and s2x2
// holds 1.5 * 2 s2, so that the pair kernels work with S / (sqrt(pi)/2) and
// T / (1.5 sqrt(pi)/2), which beyond the cut are x^-3/2 and x^-5/2.
struct alignas(16) SrcF {
    float yx, yy, yz, s2;
    float ax, ay, az, s2x2;
    float lx, ly, lz, pad;
};

// Per-chart-node Newton state, structure of arrays in sorted order.
constexpr int kHistCap = 128;   // >= the largest newton_max_iter (120)

struct NewtonState {
    DBuf T, H;           // 3 doubles each, AoS
    DBuf h, lo, hi;      // doubles
    DBuf sig;            // sigma_j (double)
    DBuf mesh;           // int32
    DBuf orig;           // int32 original output index
    DBuf status, iters;  // int8
    DBuf seen;           // int8: bit 1 Phi > 1/2 seen, bit 2 Phi < 1/2 seen
    DBuf active, active2, flag;   // int32 lists / flags
    DBuf blocksum;       // int32 per block counts
    DBuf nact;           // int32[4]: active count, count at iteration start, N
    DBuf hist;           // int32[kHistCap]: active count per iteration
    DBuf phi, grad;      // Phi and grad Phi of the evaluated targets
    // the captured iterations and what they were captured for (kernel
    // arguments: buffer addresses, sizes, options); reused while it matches
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> exec_key;
};

// Octree over the quadrature nodes and the FMM state (far_field = LSS_FAR_FMM).
// Octree forest: one root cube per mesh.  root[4m .. 4m+2] is the lower
// corner and root[4m+3] the side of mesh m's cube; level-0 box m is that cube
// and every box b belongs to the mesh bmesh[b].
__host__ __device__ inline double box_side(const double *root, const int32_t *bmesh, int32_t b, int lev) {
    return ldexp(root[4 * bmesh[b] + 3], -lev);
}

// 1/sqrt(x) in FP64: the hardware estimate (about 24 correct bits) and one
// third-order correction r (1 + e/2 + 3e^2/8), e = 1 - x r^2, whose error is
// 2.5 d^3 for a starting relative error d, far below FP64 rounding (two
// Newton steps reach the same accuracy with two more operations)
__device__ __forceinline__ double rsq64(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * r, r, 1.0);
    return fma(r * e, fma(0.375, e, 0.5), r);
}

__device__ inline uint64_t tree_spread21(uint64_t x) {     // 21 bits -> every third bit
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// tree key of a point of mesh m: mesh id above the interleaved `bits`-bit
// cell coordinates of the point in that mesh's root cube; `inside` tells
// whether the point lies in the cube (NaN: outside)
__device__ inline uint64_t tree_point_key(double x, double y, double z, int32_t m, const double *__restrict__ root,
                                          int bits, bool &inside) {
    const double *r = root + 4 * m;
    const double lim = ldexp(1.0, bits), scale = lim / r[3];
    double q[3] = {(x - r[0]) * scale, (y - r[1]) * scale, (z - r[2]) * scale};
    inside = q[0] >= 0.0 && q[0] < lim && q[1] >= 0.0 && q[1] < lim && q[2] >= 0.0 && q[2] < lim;
    uint64_t b[3];
    for (int c = 0; c < 3; ++c) {
        double t = q[c];
        t = t != t ? 0.0 : fmin(fmax(t, 0.0), lim - 1.0);
        b[c] = (uint64_t)t;
    }
    return ((uint64_t)m << (3 * bits)) | tree_spread21(b[0]) | (tree_spread21(b[1]) << 1) |
           (tree_spread21(b[2]) << 2);
}

struct Tree {
    int nroot = 1;                  // meshes = level-0 boxes
    int bits = 21;                  // Morton bits per dimension (mesh id above them)
    std::vector<double> h_root;     // host copy of root (4 per mesh)
    DBuf root, bmesh;               // double[4 * nroot], int32 per box
    int depth = 0;                  // deepest level
    bool has_tcut = false;          // tcut holds target-side cut radii (else the source radii rule)
    int64_t nboxes = 0;
    std::vector<int64_t> level_begin;   // box ids of level l: [level_begin[l], level_begin[l+1])
    // boxes (BFS order; the 8 children of a box are consecutive)
    DBuf level, ijk, nb, ne, child, parent;   // int32, int32x3, int64, int64, int32, int32
    DBuf rmax;                                // double: largest near radius of the box's nodes
    // nodes in Morton order
    DBuf key, key2, perm, perm2, src;         // u64, u64, int32, int32, Src
    // interaction lists
    DBuf p2p_key, p2p_key2, p2p_val, p2p_val2;    // u64 (T<<32|S), int32
    int64_t n_p2p = 0;
    DBuf p2p_beg, p2p_end;                    // per box, int32 offsets into the sorted p2p list
    DBuf m2p_key, m2p_key2, m2p_val, m2p_val2;    // u64 (T<<32|S), int32 S: multipole of S at T's targets
    int64_t n_m2p = 0;
    DBuf m2p_beg, m2p_end;                    // per box, int32 offsets into the sorted m2p list
    DBuf near_cnt;                            // per box + per mesh (outside targets): cost of a target in node pairs
    DBuf m2l_key, m2l_key2, m2l_val, m2l_val2;    // u64 (class<<32|T), int32 S
    int64_t n_m2l = 0;
    std::vector<int64_t> class_beg, class_end;    // host: segments of the sorted m2l list per class
    std::vector<int32_t> class_used;
    // expansions and operators
    int p = 0, ncp = 0, K = 4;
    DBuf M, L, L2;                            // nboxes * ncp doubles (L2: the M2L classes of the second stream)
    DBuf sm_meta, sm_key, sm_key2, sm_val, sm_val2, sm_tmp;   // M2L pairs of the small classes (target-major launch)
    std::vector<int64_t> sm_hb, sm_ho;                       // and their host-side tables
    std::vector<int32_t> sm_hc, sm_hslot, sm_hnkv;
    DBuf opM2M, opL2L, opM2L;                 // 8, 8 and nclass_used operators (ncp*ncp, k-major)
    std::vector<int32_t> op_class_slot;       // class -> slot in opM2L (-1 if not built)
    int ops_p = -1, ops_R = -1;
    // frontier scratch
    DBuf fr, fr2, cnt;
    // target-side cut radius per box (built with Ctx::target_widths)
    DBuf tcut;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;   // created on first use (default priority) for graph capture
    // second stream of the FMM build (created on first use, default priority,
    // non-blocking): the upward pass runs on it while the interaction lists
    // are built on `stream`; aux_ev orders the two
    hipStream_t aux_stream = nullptr;
    hipEvent_t aux_ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    std::string err;
    lss_options opt{};
    lss_stats stats{};

    // --- source set
    int64_t nverts = 0, ntris = 0;
    int32_t nmesh = 0, nq = 0;
    std::vector<int64_t> h_tri_off;   // nmesh + 1
    DBuf verts, tris, tri_off, node_off, rule;
    DBuf tris6;               // quadratic skeleton: 6 indices per triangle (tris then holds the corners)
    bool quadratic = false;
    bool have_sources = false;
    uint64_t sources_gen = 0;           // bumped by every lss_set_sources
    uint64_t vH_gen = ~0ull;            // sources_gen the vertex pseudonormals were built for
    int vH_curved = -1;                 // and their curved_charts setting

    // --- sigma
    bool have_sigma = false;
    DBuf sigma;               // ntris doubles (constant sigma broadcast)
    double sigma_max = 0.0, sigma_min = 0.0;

    // --- built state
    bool built = false;
    int64_t nnodes = 0;
    DBuf src;                 // nnodes Src records
    DBuf vH;                  // vertex pseudonormals (nverts * 3)
    double bbox_lo[3] = {0, 0, 0}, bbox_hi[3] = {0, 0, 0};

    Tree tree;
    const TargetWidths *target_widths = nullptr;   // set by lss_eval_multiscale around its build

    // --- per-eval scratch
    DBuf tkey, tkey2, tperm, tperm2, tx, ty, tz, tmesh, sort_tmp;
    DBuf tflag, tpos, tstart, ntiles, tleaf;   // FMM eval: leaf of each sorted target, tile heads
    DBuf pairs;               // double accumulator of executed pairs (stats)
    DBuf tile_queue;          // uint32[2] work queue of the FMM evaluation (zero between launches)
    DBuf tile_order;          // FMM tiles, most expensive first (int32 per tile)
    DBuf tile_bucket;         // int32[2 * kCostBuckets]: bucket counts (zero between uses), offsets
    bool pairs_pending = false;   // counter not yet read back into stats.last_pairs
    NewtonState ns;

    // --- HIP events around the pair-kernel launches (stats.pair_kernel_ms)
    std::vector<hipEvent_t> ev_start, ev_stop;
    int ev_used = 0;
    bool ev_pending = false;
    void ev_reset() { ev_used = 0; ev_pending = false; }
    void ev_begin() {
        if (ev_used == (int)ev_start.size()) {
            hipEvent_t a, b;
            LSS_HIP(hipEventCreate(&a));
            LSS_HIP(hipEventCreate(&b));
            ev_start.push_back(a);
            ev_stop.push_back(b);
        }
        LSS_HIP(hipEventRecord(ev_start[ev_used], stream));
    }
    void ev_end() {
        LSS_HIP(hipEventRecord(ev_stop[ev_used], stream));
        ++ev_used;
        ev_pending = true;
    }
};

// six-point triangles of a quadratic skeleton when the chart bases are the
// curved patches (lss_options.curved_charts), else null (corner triangles)
inline const int32_t *chart_tris6(const Ctx &c) {
    return (c.quadratic && c.opt.curved_charts) ? c.tris6.as<int32_t>() : nullptr;
}

// ------------------------------------------------------- launch wrappers
// prep (lss_kernels.hip)
void launch_prep_sources(Ctx &c);
void launch_prep_raw(Ctx &c, RawNode *out);
void launch_centroids(Ctx &c, double lambda, Cen *out, double *D);
void launch_cen_boxes(Ctx &c, const Cen *cen, double *box);
void launch_sigma_field(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen, const double *cbox,
                        const double *sigma0, double *sig, double *gsig);
// sigma(x) and grad sigma by Chebyshev interpolation of the weight sums in
// cells of side 1.5 sigma0 (lss_sigma.hip), the direct sum for the points no
// cell serves; s0_host / s0_dev: sigma0 per mesh.  Returns false, having
// written nothing, when the cells would hold more than a quarter as many
// nodes as there are points (unless force) or more than the storage cap.
bool sigma_field_interp(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen, const double *cbox,
                        const double *s0_dev, const double *s0_host, double *sig, double *gsig, bool force);
void launch_eval_multiscale(Ctx &c, int64_t n, const double *x, const int32_t *xm, const Cen *cen,
                            const double *cbox, const RawNode *nodes, const double *sigma0, double *phi,
                            double *grad, double *sig);
void launch_pseudonormals(Ctx &c);
void launch_bbox(Ctx &c);
double launch_check_orientation(Ctx &c, std::vector<double> &vol_per_mesh, int64_t &ndegenerate);

// targets: Morton keys, sort, gather into SoA (lss_kernels.hip)
void launch_target_keys(Ctx &c, const double *x, const int32_t *x_mesh, int64_t n,
                        uint64_t *keys, int32_t *idx);
void launch_gather_targets(Ctx &c, const double *x, const int32_t *x_mesh, const int32_t *perm,
                           int64_t n, double *tx, double *ty, double *tz, int32_t *tmesh);

// pair kernels (lss_p2p.hip); pairs: the statistics counters (null: none)
void launch_p2p_direct(Ctx &c, int64_t n, const int32_t *n_dev, const double *tx, const double *ty,
                       const double *tz, const int32_t *tmesh, const int32_t *out_idx,
                       double *phi, double *grad, int grad_stride, double *pairs);

// Newton (lss_kernels.hip)
void launch_chart_init(Ctx &c, const double *chart_uv, int32_t np, int64_t N);
void launch_chart_points(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, double *x,
                         int32_t *xmesh);
void launch_chart_geometry(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, const double *grad,
                           double *xu, double *xv, double *da, double *nrm);
void launch_hessian_direct(Ctx &c, int64_t n, const double *x, const int32_t *xm, double *phi, double *grad,
                           double *hess);
void launch_chart_curvature(Ctx &c, const double *uv, int32_t np, int64_t N, const double *h, const double *grad,
                            const double *hess, double *xuu, double *xuv, double *xvv, double *gauss,
                            double *mean);
void chart_interp(Ctx &c, const double *chart_uv, int32_t np, const double *f, int32_t ncomp, const double *eval_uv,
                  int32_t ne, double *out, unsigned flags);
void launch_newton_targets(Ctx &c, int64_t N);
void launch_newton_update(Ctx &c, int64_t N, double tau, const double *phi, const double *grad);
void launch_compact_active(Ctx &c, int64_t N);
void launch_iter_mark(Ctx &c);
void launch_newton_output(Ctx &c, int64_t N, double *h, double *xout, int8_t *status, int8_t *iters);

// octree, lists, FMM (lss_tree.hip, lss_fmm.hip)
// expansion order of the far field: the caller's, else 20 (mixed) or 26 (FP64)
inline int fmm_order_for(const Ctx &c) {
    return c.opt.fmm_order > 0 ? c.opt.fmm_order : (c.opt.precision == LSS_MIXED ? 20 : 26);
}
void build_tree(Ctx &c);
// the two halves of build_tree: the boxes (levels, radii, target cuts), then
// the interaction lists of the dual traversal (sorted, per class)
void build_tree_boxes(Ctx &c);
void build_tree_lists(Ctx &c);     // traversal and the sorted M2L list
void sort_near_lists(Ctx &c);      // the sorted direct and M2P lists, per-box tile costs
void build_fmm(Ctx &c);
void launch_locate_targets(Ctx &c, int64_t n_max, const int32_t *n_dev, const double *tx, const double *ty,
                           const double *tz, const int32_t *tmesh, uint64_t *keys, int32_t *idx);
// tile heads of sorted targets; flag, pos (n_max + 1 each) and blocksum
// (compact_blocks(n_max) + 2) are workspace; n_dev may be null (count n_max)
int64_t build_tiles(Ctx &c, int64_t n_max, const int32_t *n_dev, const uint64_t *sorted_keys, int tile,
                    int32_t *sorted_leaf, int32_t *tile_start, int32_t *ntiles_dev, int32_t *flag, int32_t *pos,
                    int32_t *blocksum);
int fmm_tile(const Ctx &c);
// order: the tile order of order_tiles; pairs: statistics counters (null: none)
void launch_eval_fmm(Ctx &c, int64_t max_tiles, const int32_t *ntiles_dev, const int32_t *tile_start,
                     const int32_t *n_dev, int64_t n_max, const int32_t *sorted_leaf, const int32_t *sorted_idx,
                     const double *tx, const double *ty, const double *tz, const int32_t *out_idx, double *phi,
                     double *grad, const int32_t *order, double *pairs, double *hess = nullptr,
                     const MsArgs *ms = nullptr);
void launch_soa(Ctx &c, const double *x, int64_t n, double *tx, double *ty, double *tz);
// Newton targets in FMM mode: leaf of each target in its current order and
// tile heads at leaf changes and every TILE-th position (no sort; capturable)
void ensure_tiles(Ctx &c, int64_t n_max);
// tile order for the work queue: tiles bucketed by log2 of their direct-list
// size, most expensive bucket first (kernels only: capturable)
constexpr int kCostBuckets = 64;
void order_tiles(Ctx &c, int64_t max_tiles, const int32_t *ntiles_dev, const int32_t *tile_start,
                 const int32_t *leaf, int32_t *order);
void build_tiles_unsorted(Ctx &c, int64_t n_max, const int32_t *n_dev, int tile);
void rebin_active(Ctx &c, int64_t N, int64_t nact);

// sorting and scans (lss_sort.hip)
size_t sort_pairs_u64_tmp_bytes(int64_t n);
void sort_pairs_u64(void *tmp, size_t tmp_bytes, const uint64_t *kin, uint64_t *kout,
                    const int32_t *vin, int32_t *vout, int64_t n, int begin_bit, int end_bit,
                    hipStream_t s);
// sort (key, value) pairs with a context-owned temporary; keys/values end in kout/vout
void sort_pairs(Ctx &c, const uint64_t *kin, uint64_t *kout, const int32_t *vin, int32_t *vout, int64_t n,
                int end_bit = 64);
// order-preserving compaction helpers (lss_kernels.hip).  blocksum: null =
// the context's own buffer (grown as needed), else compact_blocks(n_max) + 2
// int32 of workspace, and then n_dev must be given.
int32_t compact_blocks(int64_t n_max);
void compact_flags(Ctx &c, int64_t n_max, const int32_t *n_dev, const int32_t *flag, const int32_t *in,
                   int32_t *out, int32_t *count_dev, int32_t *blocksum = nullptr);

// Per-call device buffers of an evaluation (targets, keys, tiles, sort
// workspace).  eval_bufs_ctx() takes them from the context's grow-only
// buffers; the allocation-free entry point carves them out of its static
// scratch array (lss_noalloc.hip).
struct EvalBufs {
    double *tx, *ty, *tz;
    int32_t *tmesh;
    uint64_t *key, *key2;
    int32_t *perm, *perm2;
    int32_t *flag, *pos, *blocksum;       // tile-head workspace
    int32_t *tstart, *tleaf, *ntiles, *order;
    void *sort_tmp;
    size_t sort_bytes;
    double *pairs;                        // statistics counters, or null
    const int32_t *n_dev;                 // target count on the device, or null
};
EvalBufs eval_bufs_ctx(Ctx &c, int64_t n);
// FMM evaluation of the n targets in b.tx/ty/tz (b.tmesh for batches);
// outputs at the targets' indices
void eval_fmm_bufs(Ctx &c, const EvalBufs &b, int64_t n, double *phi, double *grad, double *hess = nullptr,
                   const MsArgs *ms = nullptr);
// direct evaluation of n targets x (device, AoS), mesh ids xm (null: one mesh)
void eval_direct_bufs(Ctx &c, const EvalBufs &b, const double *x, const int32_t *xm, int64_t n, double *phi,
                      double *grad);

// allocation-free evaluation (lss_noalloc.hip): the device address of the
// static scratch array on `device` (looked up once per device; null on
// failure, message in *err), and lss_eval_noalloc's body
void *noalloc_scratch(int device, std::string *err);
void eval_noalloc(Ctx &c, const double *x, const int32_t *xm, int64_t n, double *phi, double *grad, unsigned flags);

// ------------------------------------------------------------ constants
constexpr int kMaxIterDefault = 40;
constexpr double kCutFP64 = 8.0;                 // x = u^2 = 32 at the cut
constexpr double kCutMixed = 6.324555320336759;  // sqrt(40): x = 20 at the cut

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace lss
