// C ABI of liblss (include/lss.h): argument checking, context state and the
// orchestration of the kernels on the context's stream.
#include <cstring>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <new>
#include <sstream>

#include "lss_internal.h"

struct lss_ctx {
    lss::Ctx c;
};

namespace lss {
namespace {

__global__ void k_check_tris(int64_t n3, const int32_t *__restrict__ tris, int64_t nverts, unsigned long long *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) {
        int32_t v = tris[i];
        if (v < 0 || v >= nverts) atomicAdd(bad, 1ull);
    }
}

// corner triangles P1 P2 P3 of a quadratic skeleton
__global__ void k_corners(int64_t ntris, const int32_t *__restrict__ t6, int32_t *__restrict__ t3) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ntris)
        for (int k = 0; k < 3; ++k) t3[3 * j + k] = t6[6 * j + k];
}

__global__ void k_check_verts(int64_t n3, const double *__restrict__ v, unsigned long long *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3 && !isfinite(v[i])) atomicAdd(bad, 1ull);
}

// sigma: broadcast or copy, count invalid, min/max via the order of positive
// doubles' bit patterns
__global__ void k_sigma_set(int64_t ntris, const double *__restrict__ in, int64_t nin, double *out,
                            unsigned long long *stat) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntris) return;
    double s = in[nin == 1 ? 0 : j];
    out[j] = s;
    if (!(s > 0.0) || !isfinite(s)) {
        atomicAdd(&stat[0], 1ull);
        return;
    }
    unsigned long long b = (unsigned long long)__double_as_longlong(s);
    atomicMin(&stat[1], b);
    atomicMax(&stat[2], b);
}

// triangle centroids as points (n,3) with their mesh ids, for sigma(x) there
__global__ void k_cen_points(int64_t ntris, const Cen *__restrict__ cen, const int64_t *__restrict__ tri_off,
                             int32_t nmesh, double *x, int32_t *xm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntris) return;
    x[3 * j] = cen[j].cx;
    x[3 * j + 1] = cen[j].cy;
    x[3 * j + 2] = cen[j].cz;
    int32_t lo = 0, hi = nmesh;                  // mesh m with tri_off[m] <= j < tri_off[m + 1]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (tri_off[mid] <= j) lo = mid; else hi = mid;
    }
    xm[j] = lo;
}

__global__ void k_check_mesh_ids(int64_t n, const int32_t *__restrict__ xm, int32_t nmesh, unsigned long long *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (xm[i] < 0 || xm[i] >= nmesh)) atomicAdd(bad, 1ull);
}

inline unsigned grid_for(int64_t n, int blk = 256) { return (unsigned)ceil_div(n > 0 ? n : 1, blk); }

// The default source rule: Dunavant's 12-point symmetric rule of degree 6 on
// T0 (two three-point orbits (a, a, 1 - 2a) and one six-point orbit (b, c,
// 1 - b - c) in barycentric coordinates; weights normalised to 1 over the
// triangle, then halved for the area of T0).  The orbit parameters are the
// published ones carried to full double precision (exact on the 28 moment
// equations of degree <= 6 to rounding).  Rows are (u, v, w) = (l2, l3, w/2).
constexpr int kDefaultRuleNodes = 12;

void default_rule(double *r) {
    const double s21[2][2] = {{0.2492867451709104212916386, 0.1167862757263793660252896},
                              {0.0630890144915022283403316, 0.05084490637020681692093681}};
    const double s111[3] = {0.05314504984481694735324967, 0.3103524510337844054166077,
                            0.08285107561837357519355346};
    int k = 0;
    for (int o = 0; o < 2; ++o) {
        const double a = s21[o][0], w = s21[o][1], b = 1.0 - 2.0 * a;
        const double l23[3][2] = {{a, b}, {b, a}, {a, a}};     // (l2, l3) of (a,a,b), (a,b,a), (b,a,a)
        for (int q = 0; q < 3; ++q, ++k) {
            r[3 * k] = l23[q][0];
            r[3 * k + 1] = l23[q][1];
            r[3 * k + 2] = 0.5 * w;
        }
    }
    const double b = s111[0], c = s111[1], w = s111[2], d = 1.0 - b - c;
    // (l2, l3) of the six permutations (b,c,d), (b,d,c), (c,b,d), (c,d,b), (d,b,c), (d,c,b)
    const double l23[6][2] = {{c, d}, {d, c}, {b, d}, {d, b}, {b, c}, {c, b}};
    for (int q = 0; q < 6; ++q, ++k) {
        r[3 * k] = l23[q][0];
        r[3 * k + 1] = l23[q][1];
        r[3 * k + 2] = 0.5 * w;
    }
}

void fail(int code, const std::string &m) { throw Error{code, m}; }

// copy n bytes of caller data (host or device) into a context buffer
void upload(Ctx &c, DBuf &dst, const void *src, size_t nb, unsigned flags) {
    dst.ensure(nb);
    LSS_HIP(hipMemcpyAsync(dst.p, src, nb, (flags & LSS_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c.stream));
}

void validate_options(const lss_options &o) {
    if (o.precision != LSS_FP64 && o.precision != LSS_MIXED) fail(LSS_EINVAL, "precision must be LSS_FP64 or LSS_MIXED");
    if (o.far_field != LSS_FAR_DIRECT && o.far_field != LSS_FAR_FMM) fail(LSS_EINVAL, "unknown far_field");
    if (o.fmm_order < 0 || o.fmm_order > 40) fail(LSS_EINVAL, "fmm_order must be in [0, 40]");
    if (o.leaf_capacity < 0) fail(LSS_EINVAL, "leaf_capacity < 0");
    if (!(o.cut_factor >= 0.0) || !std::isfinite(o.cut_factor)) fail(LSS_EINVAL, "cut_factor must be >= 0 and finite");
    if (o.cut_factor != 0.0 && o.cut_factor < 4.0) fail(LSS_EINVAL, "cut_factor must be 0 (default) or >= 4");
    if (!(o.newton_tau >= 0.0) || !std::isfinite(o.newton_tau)) fail(LSS_EINVAL, "newton_tau must be >= 0");
    if (o.newton_max_iter < 0 || o.newton_max_iter > 120) fail(LSS_EINVAL, "newton_max_iter must be in [0, 120]");
    if (o.tile != 0 && o.tile != 64 && o.tile != 128 && o.tile != 256) fail(LSS_EINVAL, "tile must be 0, 64, 128 or 256");
    if (!(o.leaf_shrink == 0.0 || (o.leaf_shrink >= 1.0 && o.leaf_shrink <= 3.0)))
        fail(LSS_EINVAL, "leaf_shrink must be 0 (default) or in [1, 3]");
    if (o.count_useful != 0 && o.count_useful != 1) fail(LSS_EINVAL, "count_useful must be 0 or 1");
    if (o.admissibility != 0 && (o.admissibility < 4 || o.admissibility > 18))
        fail(LSS_EINVAL, "admissibility must be 0 (default) or in [4, 18]");
    if (o.curved_charts != 0 && o.curved_charts != 1) fail(LSS_EINVAL, "curved_charts must be 0 or 1");
    if (o.sigma_interp < 0 || o.sigma_interp > 2) fail(LSS_EINVAL, "sigma_interp must be 0, 1 or 2");
    for (int k = 0; k < 2; ++k)
        if (o.reserved[k] != 0) fail(LSS_EINVAL, "reserved option fields must be zero");
}

void build(Ctx &c) {
    if (!c.have_sources) fail(LSS_ESTATE, "lss_build: no sources (call lss_set_sources)");
    if (!c.have_sigma) fail(LSS_ESTATE, "lss_build: no sigma (call lss_set_sigma after lss_set_sources)");
    if (c.built) return;
    c.nnodes = c.ntris * (int64_t)c.nq;
    c.src.ensure(sizeof(Src) * (size_t)c.nnodes);
    launch_prep_sources(c);
    launch_bbox(c);
    if (c.vH_gen != c.sources_gen || c.vH_curved != c.opt.curved_charts) {
        // the vertex pseudonormals depend on the skeleton alone, not on sigma
        launch_pseudonormals(c);
        c.vH_gen = c.sources_gen;
        c.vH_curved = c.opt.curved_charts;
    }
    c.pairs.ensure(sizeof(double) * 4);
    c.tile_queue.ensure(sizeof(unsigned int) * 4);
    LSS_HIP(hipMemsetAsync(c.tile_queue.p, 0, sizeof(unsigned int) * 4, c.stream));
    c.tile_bucket.ensure(sizeof(int32_t) * 2 * kCostBuckets);
    LSS_HIP(hipMemsetAsync(c.tile_bucket.p, 0, sizeof(int32_t) * 2 * kCostBuckets, c.stream));
    c.stats.n_boxes = c.stats.n_leaves = c.stats.n_m2l = c.stats.n_m2p = 0;
    c.stats.tree_depth = c.stats.fmm_order = 0;
    if (c.opt.far_field == LSS_FAR_FMM) build_fmm(c);
    c.built = true;
    c.stats.n_tris = c.ntris;
    c.stats.n_nodes = c.nnodes;
    c.stats.n_mesh = c.nmesh;
}

void ensure_targets(Ctx &c, int64_t n) {
    c.tkey.ensure(sizeof(uint64_t) * n);
    c.tkey2.ensure(sizeof(uint64_t) * n);
    c.tperm.ensure(sizeof(int32_t) * n);
    c.tperm2.ensure(sizeof(int32_t) * n);
    c.tx.ensure(sizeof(double) * n);
    c.ty.ensure(sizeof(double) * n);
    c.tz.ensure(sizeof(double) * n);
    c.tmesh.ensure(sizeof(int32_t) * n);
}

}  // namespace

// The context's grow-only buffers as the per-call buffers of an evaluation of
// n targets (statistics counters and timing events on).
EvalBufs eval_bufs_ctx(Ctx &c, int64_t n) {
    ensure_targets(c, n);
    c.tflag.ensure(sizeof(int32_t) * (n + 1));
    c.tpos.ensure(sizeof(int32_t) * (n + 1));
    c.tstart.ensure(sizeof(int32_t) * (n + 1));
    c.tleaf.ensure(sizeof(int32_t) * (n + 1));
    c.tile_order.ensure(sizeof(int32_t) * (n + 1));
    c.ntiles.ensure(16);
    c.ns.blocksum.ensure(sizeof(int32_t) * (compact_blocks(n) + 2));
    const size_t tb = sort_pairs_u64_tmp_bytes(n);
    c.sort_tmp.ensure(tb);
    EvalBufs b;
    b.tx = c.tx.as<double>();
    b.ty = c.ty.as<double>();
    b.tz = c.tz.as<double>();
    b.tmesh = c.tmesh.as<int32_t>();
    b.key = c.tkey.as<uint64_t>();
    b.key2 = c.tkey2.as<uint64_t>();
    b.perm = c.tperm.as<int32_t>();
    b.perm2 = c.tperm2.as<int32_t>();
    b.flag = c.tflag.as<int32_t>();
    b.pos = c.tpos.as<int32_t>();
    b.blocksum = nullptr;                 // compact_flags uses (and grows) the context's own
    b.tstart = c.tstart.as<int32_t>();
    b.tleaf = c.tleaf.as<int32_t>();
    b.ntiles = c.ntiles.as<int32_t>();
    b.order = c.tile_order.as<int32_t>();
    b.sort_tmp = c.sort_tmp.p;
    b.sort_bytes = tb;
    b.pairs = c.pairs.as<double>();
    b.n_dev = nullptr;
    return b;
}

// FMM evaluation of the targets already in b.tx/ty/tz[0..n): leaf of each
// target, targets sorted by leaf, tiles, near field + L2P.  Outputs at the
// target's index in tx/ty/tz.  With b.pairs the counters are cleared first and
// HIP events bracket the evaluation launch (lss_stats).
void eval_fmm_bufs(Ctx &c, const EvalBufs &b, int64_t n, double *phi, double *grad, double *hess, const MsArgs *ms) {
    launch_locate_targets(c, n, b.n_dev, b.tx, b.ty, b.tz, b.tmesh, b.key, b.perm);
    sort_pairs_u64(b.sort_tmp, b.sort_bytes, b.key, b.key2, b.perm, b.perm2, n, 0, 64, c.stream);
    build_tiles(c, n, b.n_dev, b.key2, fmm_tile(c), b.tleaf, b.tstart, b.ntiles, b.flag, b.pos, b.blocksum);
    order_tiles(c, n, b.ntiles, b.tstart, b.tleaf, b.order);
    if (b.pairs) {
        LSS_HIP(hipMemsetAsync(b.pairs, 0, 4 * sizeof(double), c.stream));
        c.ev_begin();
    }
    launch_eval_fmm(c, n, b.ntiles, b.tstart, b.n_dev, n, b.tleaf, b.perm2, b.tx, b.ty, b.tz, nullptr, phi, grad,
                    b.order, b.pairs, hess, ms);
    if (b.pairs) c.ev_end();
}

// Direct evaluation: targets sorted by (mesh, Morton key), gathered into SoA,
// every pair of the target's mesh; outputs at the caller's target index.
void eval_direct_bufs(Ctx &c, const EvalBufs &b, const double *x, const int32_t *xm, int64_t n, double *phi,
                      double *grad) {
    launch_target_keys(c, x, xm, n, b.key, b.perm);
    sort_pairs_u64(b.sort_tmp, b.sort_bytes, b.key, b.key2, b.perm, b.perm2, n, 0, 64, c.stream);
    launch_gather_targets(c, x, xm, b.perm2, n, b.tx, b.ty, b.tz, b.tmesh);
    if (b.pairs) {
        LSS_HIP(hipMemsetAsync(b.pairs, 0, 4 * sizeof(double), c.stream));
        c.ev_begin();
    }
    launch_p2p_direct(c, n, b.n_dev, b.tx, b.ty, b.tz, b.tmesh, b.perm2, phi, grad, 3, b.pairs);
    if (b.pairs) c.ev_end();
}

namespace {

void eval(Ctx &c, const double *x, const int32_t *xm, int64_t n, double *phi, double *grad, unsigned flags) {
    if (n < 0) fail(LSS_EINVAL, "lss_eval: n < 0");
    if (n == 0) return;
    if (n > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_eval: n exceeds 2^31-1");
    if (!x || !phi) fail(LSS_EINVAL, "lss_eval: x and phi must be non-null");
    if (c.nmesh > 1 && !xm) fail(LSS_EINVAL, "lss_eval: x_mesh is required for a batch of meshes");
    build(c);
    const bool dev = flags & LSS_PTR_DEVICE;
    DBuf hx, hxm, hphi, hgrad;
    const double *dx = x;
    const int32_t *dxm = c.nmesh > 1 ? xm : nullptr;
    double *dphi = phi, *dgrad = grad;
    if (!dev) {
        upload(c, hx, x, sizeof(double) * 3 * n, 0);
        dx = hx.as<double>();
        if (dxm) {
            upload(c, hxm, xm, sizeof(int32_t) * n, 0);
            dxm = hxm.as<int32_t>();
        }
        hphi.ensure(sizeof(double) * n);
        dphi = hphi.as<double>();
        if (grad) {
            hgrad.ensure(sizeof(double) * 3 * n);
            dgrad = hgrad.as<double>();
        }
    }
    if (dxm) {      // mesh ids index per-mesh tables in every kernel: checked for device pointers too
        DBuf bad;
        bad.ensure(8);
        LSS_HIP(hipMemsetAsync(bad.p, 0, 8, c.stream));
        hipLaunchKernelGGL(k_check_mesh_ids, dim3(grid_for(n)), dim3(256), 0, c.stream, n, dxm, c.nmesh,
                           bad.as<unsigned long long>());
        unsigned long long nb = 0;
        LSS_HIP(hipMemcpyAsync(&nb, bad.p, 8, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (nb) fail(LSS_EINVAL, "lss_eval: x_mesh values outside [0, nmesh)");
    }
    const EvalBufs b = eval_bufs_ctx(c, n);
    c.ev_reset();
    if (c.opt.far_field == LSS_FAR_FMM) {
        launch_soa(c, dx, n, b.tx, b.ty, b.tz);
        if (dxm) LSS_HIP(hipMemcpyAsync(b.tmesh, dxm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        eval_fmm_bufs(c, b, n, dphi, dgrad);
    } else {
        eval_direct_bufs(c, b, dx, dxm, n, dphi, dgrad);
    }
    if (!dev) {
        LSS_HIP(hipMemcpyAsync(phi, dphi, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
        if (grad) LSS_HIP(hipMemcpyAsync(grad, dgrad, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        hx.release(); hxm.release(); hphi.release(); hgrad.release();
    }
    c.stats.last_targets = n;
    c.pairs_pending = true;
}

// One Newton iteration over the active list, entirely on the device: no host
// read, allocation, memset or sort, so a run of iterations can be captured.
void newton_iteration(Ctx &c, int64_t N, double tau, double *phi, double *grad) {
    NewtonState &s = c.ns;
    const int32_t *nact = s.nact.as<int32_t>();
    launch_iter_mark(c);
    launch_newton_targets(c, N);
    if (c.opt.far_field == LSS_FAR_FMM) {
        build_tiles_unsorted(c, N, nact, fmm_tile(c));
        order_tiles(c, N, c.ntiles.as<int32_t>(), c.tstart.as<int32_t>(), c.tleaf.as<int32_t>(),
                    c.tile_order.as<int32_t>());
        launch_eval_fmm(c, N, c.ntiles.as<int32_t>(), c.tstart.as<int32_t>(), nact, N, c.tleaf.as<int32_t>(),
                        nullptr, c.tx.as<double>(), c.ty.as<double>(), c.tz.as<double>(), nullptr, phi, grad,
                        c.tile_order.as<int32_t>(), c.pairs.as<double>());
    } else {
        launch_p2p_direct(c, N, nact, c.tx.as<double>(), c.ty.as<double>(), c.tz.as<double>(), c.tmesh.as<int32_t>(),
                          nullptr, phi, grad, 3, c.pairs.as<double>());
    }
    launch_newton_update(c, N, tau, phi, grad);
    launch_compact_active(c, N);
}

// Capture `count` Newton iterations into an executable graph.  The capture
// runs on a stream of the context's own (default priority); the graph is then
// launched on the context stream.
hipGraphExec_t capture_newton(Ctx &c, int64_t N, double tau, double *phi, double *grad, int count) {
    if (!c.capture_stream) LSS_HIP(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
    hipStream_t saved = c.stream;
    c.stream = c.capture_stream;
    hipGraph_t graph = nullptr;
    LSS_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < count; ++k) newton_iteration(c, N, tau, phi, grad);
    } catch (...) {
        (void)hipStreamEndCapture(c.stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        c.stream = saved;
        throw;
    }
    hipError_t e = hipStreamEndCapture(c.stream, &graph);
    c.stream = saved;
    if (e != hipSuccess) fail(LSS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) fail(LSS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return exec;
}

constexpr int kNewtonChunk = 8;   // iterations per graph launch between host checks

// Everything the captured iterations bake in: the address of every buffer
// their kernels touch, the sizes and scalars passed by value, and the options
// that choose kernels.  A graph captured for an equal key is reused.
std::vector<uint64_t> newton_key(const Ctx &c, int64_t N, double tau, int maxit, int chunk) {
    const NewtonState &s = c.ns;
    const Tree &t = c.tree;
    uint64_t tb;
    std::memcpy(&tb, &tau, 8);
    std::vector<uint64_t> k = {(uint64_t)N, tb, (uint64_t)maxit, (uint64_t)chunk, (uint64_t)c.opt.precision,
                               (uint64_t)c.opt.far_field, (uint64_t)c.opt.tile, (uint64_t)c.opt.count_useful,
                               (uint64_t)c.nnodes, (uint64_t)c.nmesh, (uint64_t)t.nboxes, (uint64_t)t.p,
                               (uint64_t)t.ncp, (uint64_t)t.K, (uint64_t)t.nroot, (uint64_t)t.bits};
    const DBuf *bufs[] = {&s.T, &s.H, &s.h, &s.lo, &s.hi, &s.sig, &s.mesh, &s.orig, &s.status, &s.iters, &s.seen,
                          &s.active, &s.active2, &s.flag, &s.blocksum, &s.nact, &s.hist, &s.phi, &s.grad,
                          &c.tx, &c.ty, &c.tz, &c.tmesh, &c.tleaf, &c.tstart, &c.ntiles, &c.tflag, &c.tpos,
                          &c.tile_order, &c.tile_bucket, &c.tile_queue, &c.pairs, &c.src, &c.node_off, &c.verts,
                          &c.tris, &c.vH, &c.sigma, &c.tri_off, &t.p2p_beg, &t.p2p_end, &t.p2p_val2, &t.nb, &t.ne,
                          &t.level, &t.ijk, &t.src, &t.L, &t.M, &t.m2p_beg, &t.m2p_end, &t.m2p_val2, &t.root,
                          &t.bmesh, &t.child, &t.parent, &t.rmax, &t.near_cnt};
    for (const DBuf *b : bufs) k.push_back((uint64_t)(uintptr_t)b->p);
    return k;
}

void drop_newton_graph(NewtonState &s) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    s.exec = nullptr;
    s.exec_key.clear();
}

void project(Ctx &c, const double *uv, int32_t np, double *h, double *xout, int8_t *st, int8_t *it, unsigned flags) {
    if (np <= 0) fail(LSS_EINVAL, "lss_project: np must be >= 1");
    if (!uv || !h) fail(LSS_EINVAL, "lss_project: chart_uv and h must be non-null");
    build(c);
    const int64_t N = c.ntris * (int64_t)np;
    if (N > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_project: ntris * np exceeds 2^31-1");
    const bool dev = flags & LSS_PTR_DEVICE;
    DBuf duv, dh, dx, dst, dit;
    upload(c, duv, uv, sizeof(double) * 2 * np, flags);
    const double tau = c.opt.newton_tau > 0 ? c.opt.newton_tau : (c.opt.precision == LSS_MIXED ? 1e-6 : 1e-12);
    const int maxit = c.opt.newton_max_iter > 0 ? c.opt.newton_max_iter : kMaxIterDefault;
    launch_chart_init(c, duv.as<double>(), np, N);
    ensure_targets(c, N);
    if (c.opt.far_field == LSS_FAR_FMM) ensure_tiles(c, N);
    NewtonState &s = c.ns;
    DBuf &phi = s.phi, &grad = s.grad;
    phi.ensure(sizeof(double) * N);
    grad.ensure(sizeof(double) * 3 * N);
    LSS_HIP(hipMemsetAsync(c.pairs.p, 0, 4 * sizeof(double), c.stream));
    // Iterations run in captured chunks; a node leaves the active list when it
    // converges or reaches maxit, so iterations past the last active one are
    // empty launches and the host only checks the count between chunks.  The
    // chunk is captured once and relaunched by later calls whose key matches.
    const bool fmm = c.opt.far_field == LSS_FAR_FMM;
    const int chunk = std::min(maxit, kNewtonChunk);
    std::vector<uint64_t> key = newton_key(c, N, tau, maxit, chunk);
    if (!s.exec || key != s.exec_key) {
        drop_newton_graph(s);
        s.exec = capture_newton(c, N, tau, phi.as<double>(), grad.as<double>(), chunk);
        s.exec_key = std::move(key);
    }
    hipGraphExec_t exec = s.exec;
    c.ev_reset();
    try {
        int done = 0;
        if (fmm && maxit > 1) {     // first step from the chart points, then re-bin by leaf
            c.ev_begin();
            newton_iteration(c, N, tau, phi.as<double>(), grad.as<double>());
            c.ev_end();
            done = 1;
        }
        for (; done < maxit; done += chunk) {
            int32_t nact = 0;
            LSS_HIP(hipMemcpyAsync(&nact, s.nact.p, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
            LSS_HIP(hipStreamSynchronize(c.stream));
            if (nact == 0) break;
            if (fmm && done > 0) rebin_active(c, N, nact);
            c.ev_begin();
            LSS_HIP(hipGraphLaunch(exec, c.stream));
            c.ev_end();
        }
        LSS_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
        (void)hipStreamSynchronize(c.stream);
        drop_newton_graph(s);
        throw;
    }
    double *oh = h, *ox = xout;
    int8_t *ost = st, *oit = it;
    if (!dev) {
        dh.ensure(sizeof(double) * N);
        oh = dh.as<double>();
        if (xout) { dx.ensure(sizeof(double) * 3 * N); ox = dx.as<double>(); }
        if (st) { dst.ensure(N); ost = dst.as<int8_t>(); }
        if (it) { dit.ensure(N); oit = dit.as<int8_t>(); }
    }
    launch_newton_output(c, N, oh, ox, ost, oit);
    c.pairs_pending = true;
    if (!dev) {
        LSS_HIP(hipMemcpyAsync(h, oh, sizeof(double) * N, hipMemcpyDeviceToHost, c.stream));
        if (xout) LSS_HIP(hipMemcpyAsync(xout, ox, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c.stream));
        if (st) LSS_HIP(hipMemcpyAsync(st, ost, N, hipMemcpyDeviceToHost, c.stream));
        if (it) LSS_HIP(hipMemcpyAsync(it, oit, N, hipMemcpyDeviceToHost, c.stream));
    }
    int32_t cnt[4] = {0, 0, 0, 0};
    std::vector<int32_t> hist(kHistCap, 0);
    LSS_HIP(hipMemcpyAsync(cnt, s.nact.p, sizeof(cnt), hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipMemcpyAsync(hist.data(), s.hist.p, sizeof(int32_t) * kHistCap, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    int64_t evals = 0;
    for (int k = 0; k < cnt[3] && k < kHistCap; ++k) evals += hist[k];
    c.stats.last_targets = evals;
    c.stats.newton_iters = cnt[3];
}

// Chart geometry at given chart distances (section 3.1, eq. u_vector to eq. da):
// the chart points x = T + h H, one evaluation of grad Phi there, then the
// tangents, area element and outward unit normal per node.
void chart_geometry(Ctx &c, const double *uv, int32_t np, const double *h, double *xu, double *xv, double *da,
                    double *nrm, unsigned flags) {
    if (np <= 0) fail(LSS_EINVAL, "lss_chart_geometry: np must be >= 1");
    if (!uv || !h) fail(LSS_EINVAL, "lss_chart_geometry: chart_uv and h must be non-null");
    build(c);
    const int64_t N = c.ntris * (int64_t)np;
    if (N > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_chart_geometry: ntris * np exceeds 2^31-1");
    if (N == 0) return;
    const bool dev = flags & LSS_PTR_DEVICE;
    DBuf duv, dh, x, xm, phi, grad, oxu, oxv, oda, onr;
    upload(c, duv, uv, sizeof(double) * 2 * np, flags);
    const double *ph = h;
    if (!dev) {
        upload(c, dh, h, sizeof(double) * N, 0);
        ph = dh.as<double>();
    }
    x.ensure(sizeof(double) * 3 * N);
    if (c.nmesh > 1) xm.ensure(sizeof(int32_t) * N);
    launch_chart_points(c, duv.as<double>(), np, N, ph, x.as<double>(), c.nmesh > 1 ? xm.as<int32_t>() : nullptr);
    phi.ensure(sizeof(double) * N);
    grad.ensure(sizeof(double) * 3 * N);
    eval(c, x.as<double>(), c.nmesh > 1 ? xm.as<int32_t>() : nullptr, N, phi.as<double>(), grad.as<double>(),
         LSS_PTR_DEVICE);
    double *qxu = xu, *qxv = xv, *qda = da, *qnr = nrm;
    if (!dev) {
        if (xu) { oxu.ensure(sizeof(double) * 3 * N); qxu = oxu.as<double>(); }
        if (xv) { oxv.ensure(sizeof(double) * 3 * N); qxv = oxv.as<double>(); }
        if (da) { oda.ensure(sizeof(double) * N); qda = oda.as<double>(); }
        if (nrm) { onr.ensure(sizeof(double) * 3 * N); qnr = onr.as<double>(); }
    }
    launch_chart_geometry(c, duv.as<double>(), np, N, ph, grad.as<double>(), qxu, qxv, qda, qnr);
    if (!dev) {
        if (xu) LSS_HIP(hipMemcpyAsync(xu, qxu, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c.stream));
        if (xv) LSS_HIP(hipMemcpyAsync(xv, qxv, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c.stream));
        if (da) LSS_HIP(hipMemcpyAsync(da, qda, sizeof(double) * N, hipMemcpyDeviceToHost, c.stream));
        if (nrm) LSS_HIP(hipMemcpyAsync(nrm, qnr, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c.stream));
    }
    // the temporaries are freed on return: wait for the kernels that use them
    LSS_HIP(hipStreamSynchronize(c.stream));
}

// Hessian (and Phi, grad Phi) by the direct sum over the target's mesh
void eval_hessian(Ctx &c, const double *x, const int32_t *xm, int64_t n, double *phi, double *grad, double *hess,
                  unsigned flags) {
    if (n < 0) fail(LSS_EINVAL, "lss_eval_hessian: n < 0");
    if (n == 0) return;
    if (n > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_eval_hessian: n exceeds 2^31-1");
    if (!x || !hess) fail(LSS_EINVAL, "lss_eval_hessian: x and hess must be non-null");
    if (c.nmesh > 1 && !xm) fail(LSS_EINVAL, "lss_eval_hessian: x_mesh is required for a batch of meshes");
    build(c);
    const bool dev = flags & LSS_PTR_DEVICE;
    DBuf hx, hxm, hphi, hgrad, hhess;
    const double *dx = x;
    const int32_t *dxm = c.nmesh > 1 ? xm : nullptr;
    double *dphi = phi, *dgrad = grad, *dhess = hess;
    if (!dev) {
        upload(c, hx, x, sizeof(double) * 3 * n, 0);
        dx = hx.as<double>();
        if (dxm) {
            upload(c, hxm, xm, sizeof(int32_t) * n, 0);
            dxm = hxm.as<int32_t>();
        }
        if (phi) { hphi.ensure(sizeof(double) * n); dphi = hphi.as<double>(); }
        if (grad) { hgrad.ensure(sizeof(double) * 3 * n); dgrad = hgrad.as<double>(); }
        hhess.ensure(sizeof(double) * 6 * n);
        dhess = hhess.as<double>();
    }
    if (dxm) {
        DBuf bad;
        bad.ensure(8);
        LSS_HIP(hipMemsetAsync(bad.p, 0, 8, c.stream));
        hipLaunchKernelGGL(k_check_mesh_ids, dim3(grid_for(n)), dim3(256), 0, c.stream, n, dxm, c.nmesh,
                           bad.as<unsigned long long>());
        unsigned long long nb = 0;
        LSS_HIP(hipMemcpyAsync(&nb, bad.p, 8, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (nb) fail(LSS_EINVAL, "lss_eval_hessian: x_mesh values outside [0, nmesh)");
    }
    if (c.opt.far_field == LSS_FAR_FMM) {       // near lists + expansions of the context's tree
        const EvalBufs b = eval_bufs_ctx(c, n);
        c.ev_reset();
        launch_soa(c, dx, n, b.tx, b.ty, b.tz);
        if (dxm) LSS_HIP(hipMemcpyAsync(b.tmesh, dxm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        eval_fmm_bufs(c, b, n, dphi, dgrad, dhess);
    } else {
        launch_hessian_direct(c, n, dx, dxm, dphi, dgrad, dhess);
    }
    if (!dev) {
        if (phi) LSS_HIP(hipMemcpyAsync(phi, dphi, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
        if (grad) LSS_HIP(hipMemcpyAsync(grad, dgrad, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipMemcpyAsync(hess, dhess, sizeof(double) * 6 * n, hipMemcpyDeviceToHost, c.stream));
    }
    LSS_HIP(hipStreamSynchronize(c.stream));
}

// Phi, grad Phi with the target-attached width sigma(x)
void eval_multiscale(Ctx &c, double lambda, double sigma0, const double *x, const int32_t *xm, int64_t n, double *phi,
                     double *grad, double *sig, unsigned flags) {
    if (!c.have_sources) fail(LSS_ESTATE, "lss_eval_multiscale: no sources (call lss_set_sources)");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) fail(LSS_EINVAL, "lss_eval_multiscale: lambda must be positive");
    if (!(sigma0 >= 0.0) || !std::isfinite(sigma0)) fail(LSS_EINVAL, "lss_eval_multiscale: sigma0 must be >= 0");
    if (n < 0) fail(LSS_EINVAL, "lss_eval_multiscale: n < 0");
    if (n == 0) return;
    if (n > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_eval_multiscale: n exceeds 2^31-1");
    if (!x || !phi) fail(LSS_EINVAL, "lss_eval_multiscale: x and phi must be non-null");
    if (c.nmesh > 1 && !xm) fail(LSS_EINVAL, "lss_eval_multiscale: x_mesh is required for a batch of meshes");
    const bool dev = flags & LSS_PTR_DEVICE;
    // centroids, sigma_j and sigma0 per mesh (sqrt(5) max_j D_j when sigma0 == 0)
    DBuf cen, D, s0, raw, cbox;
    cen.ensure(sizeof(Cen) * c.ntris);
    D.ensure(sizeof(double) * c.ntris);
    launch_centroids(c, lambda, cen.as<Cen>(), D.as<double>());
    cbox.ensure(sizeof(double) * 6 * ((c.ntris + 255) / 256));
    launch_cen_boxes(c, cen.as<Cen>(), cbox.as<double>());
    std::vector<double> hD(c.ntris), hs0(c.nmesh);
    LSS_HIP(hipMemcpyAsync(hD.data(), D.p, sizeof(double) * c.ntris, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    for (int32_t m = 0; m < c.nmesh; ++m) {
        double dmax = 0.0;
        for (int64_t j = c.h_tri_off[m]; j < c.h_tri_off[m + 1]; ++j) dmax = std::max(dmax, hD[j]);
        hs0[m] = sigma0 > 0.0 ? sigma0 : std::sqrt(5.0) * dmax;
        if (c.h_tri_off[m + 1] > c.h_tri_off[m] && !(hs0[m] > 0.0) )
            fail(LSS_EINVAL, "lss_eval_multiscale: a mesh has only zero-size triangles");
    }
    upload(c, s0, hs0.data(), sizeof(double) * c.nmesh, 0);
    DBuf hx, hxm, hphi, hgrad, hsig;
    const double *dx = x;
    const int32_t *dxm = c.nmesh > 1 ? xm : nullptr;
    double *dphi = phi, *dgrad = grad, *dsig = sig;
    if (!dev) {
        upload(c, hx, x, sizeof(double) * 3 * n, 0);
        dx = hx.as<double>();
        if (dxm) {
            upload(c, hxm, xm, sizeof(int32_t) * n, 0);
            dxm = hxm.as<int32_t>();
        }
        hphi.ensure(sizeof(double) * n);
        dphi = hphi.as<double>();
        if (grad) { hgrad.ensure(sizeof(double) * 3 * n); dgrad = hgrad.as<double>(); }
        if (sig) { hsig.ensure(sizeof(double) * n); dsig = hsig.as<double>(); }
    }
    if (dxm) {
        DBuf bad;
        bad.ensure(8);
        LSS_HIP(hipMemsetAsync(bad.p, 0, 8, c.stream));
        hipLaunchKernelGGL(k_check_mesh_ids, dim3(grid_for(n)), dim3(256), 0, c.stream, n, dxm, c.nmesh,
                           bad.as<unsigned long long>());
        unsigned long long nb = 0;
        LSS_HIP(hipMemcpyAsync(&nb, bad.p, 8, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (nb) fail(LSS_EINVAL, "lss_eval_multiscale: x_mesh values outside [0, nmesh)");
    }
    if (c.opt.far_field == LSS_FAR_FMM) {
        // sigma(x) and grad sigma at the targets; sigma at the centroids sizes
        // the leaves (built in place of the caller's sigma, which is put back
        // afterwards: the built state is then stale and rebuilt on use); the
        // lists are built for these targets, with cut * sigma(x) as the
        // radius every far interaction must clear
        DBuf sall, gall, xall, xmall, cpt, cxm, saved;
        const int64_t nt = c.ntris, na = n + nt;
        sall.ensure(sizeof(double) * na);
        gall.ensure(sizeof(double) * 3 * na);
        cpt.ensure(sizeof(double) * 3 * nt);
        cxm.ensure(sizeof(int32_t) * nt);
        hipLaunchKernelGGL(k_cen_points, dim3(grid_for(nt)), dim3(256), 0, c.stream, nt, cen.as<Cen>(),
                           c.tri_off.as<int64_t>(), c.nmesh, cpt.as<double>(), cxm.as<int32_t>());
        LSS_CHECK_LAUNCH("k_cen_points");
        // one pass over the targets and the centroids together: the
        // interpolation cells then serve both
        bool done = false;
        if (c.opt.sigma_interp != 1) {
            xall.ensure(sizeof(double) * 3 * na);
            LSS_HIP(hipMemcpyAsync(xall.p, dx, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, c.stream));
            LSS_HIP(hipMemcpyAsync(xall.as<double>() + 3 * n, cpt.p, sizeof(double) * 3 * nt, hipMemcpyDeviceToDevice,
                                   c.stream));
            if (dxm) {
                xmall.ensure(sizeof(int32_t) * na);
                LSS_HIP(hipMemcpyAsync(xmall.p, dxm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
                LSS_HIP(hipMemcpyAsync(xmall.as<int32_t>() + n, cxm.p, sizeof(int32_t) * nt, hipMemcpyDeviceToDevice,
                                       c.stream));
            }
            done = sigma_field_interp(c, na, xall.as<double>(), dxm ? xmall.as<int32_t>() : nullptr, cen.as<Cen>(),
                                      cbox.as<double>(), s0.as<double>(), hs0.data(), sall.as<double>(),
                                      gall.as<double>(), c.opt.sigma_interp == 2);
        }
        if (!done) {
            launch_sigma_field(c, n, dx, dxm, cen.as<Cen>(), cbox.as<double>(), s0.as<double>(), sall.as<double>(),
                               gall.as<double>());
            launch_sigma_field(c, nt, cpt.as<double>(), c.nmesh > 1 ? cxm.as<int32_t>() : nullptr, cen.as<Cen>(),
                               cbox.as<double>(), s0.as<double>(), sall.as<double>() + n, gall.as<double>() + 3 * n);
        }
        double *tsig = sall.as<double>(), *tgs = gall.as<double>(), *csig = sall.as<double>() + n;
        std::vector<double> hcs(c.ntris);
        LSS_HIP(hipMemcpyAsync(hcs.data(), csig, sizeof(double) * c.ntris, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        double mn = INFINITY, mx = 0.0;
        for (double v : hcs) { mn = std::min(mn, v); mx = std::max(mx, v); }
        if (!(mn > 0.0) || !std::isfinite(mx)) fail(LSS_EINVAL, "lss_eval_multiscale: sigma at a centroid is not positive");
        struct Restore {
            Ctx &c;
            DBuf &saved;
            bool had;
            double lo, hi;
            ~Restore() {
                if (had) (void)hipMemcpyAsync(c.sigma.p, saved.p, sizeof(double) * c.ntris, hipMemcpyDeviceToDevice,
                                              c.stream);
                (void)hipStreamSynchronize(c.stream);
                c.have_sigma = had;
                c.sigma_min = lo;
                c.sigma_max = hi;
                c.built = false;
                c.target_widths = nullptr;
            }
        } restore{c, saved, c.have_sigma, c.sigma_min, c.sigma_max};
        if (c.have_sigma) {
            saved.ensure(sizeof(double) * c.ntris);
            LSS_HIP(hipMemcpyAsync(saved.p, c.sigma.p, sizeof(double) * c.ntris, hipMemcpyDeviceToDevice, c.stream));
        }
        c.sigma.ensure(sizeof(double) * c.ntris);
        LSS_HIP(hipMemcpyAsync(c.sigma.p, csig, sizeof(double) * c.ntris, hipMemcpyDeviceToDevice, c.stream));
        c.have_sigma = true;
        c.sigma_min = mn;
        c.sigma_max = mx;
        c.built = false;
        const TargetWidths tw{dx, dxm, tsig, n};
        c.target_widths = &tw;
        build(c);
        c.target_widths = nullptr;
        const EvalBufs b = eval_bufs_ctx(c, n);
        c.ev_reset();
        launch_soa(c, dx, n, b.tx, b.ty, b.tz);
        if (dxm) LSS_HIP(hipMemcpyAsync(b.tmesh, dxm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        const double cut = c.opt.cut_factor > 0 ? c.opt.cut_factor
                                                 : (c.opt.precision == LSS_MIXED ? kCutMixed : kCutFP64);
        const MsArgs ms{tsig, tgs, 0.5 * cut * cut};
        eval_fmm_bufs(c, b, n, dphi, dgrad, nullptr, &ms);
        if (dsig) LSS_HIP(hipMemcpyAsync(dsig, tsig, sizeof(double) * n, hipMemcpyDeviceToDevice, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
    } else {
        raw.ensure(sizeof(RawNode) * c.ntris * c.nq);
        launch_prep_raw(c, raw.as<RawNode>());
        launch_eval_multiscale(c, n, dx, dxm, cen.as<Cen>(), cbox.as<double>(), raw.as<RawNode>(), s0.as<double>(),
                               dphi, dgrad, dsig);
    }
    if (!dev) {
        LSS_HIP(hipMemcpyAsync(phi, dphi, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
        if (grad) LSS_HIP(hipMemcpyAsync(grad, dgrad, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c.stream));
        if (sig) LSS_HIP(hipMemcpyAsync(sig, dsig, sizeof(double) * n, hipMemcpyDeviceToHost, c.stream));
    }
    LSS_HIP(hipStreamSynchronize(c.stream));
}

void chart_curvature(Ctx &c, const double *uv, int32_t np, const double *h, double *xuu, double *xuv, double *xvv,
                     double *gauss, double *mean, unsigned flags) {
    if (np <= 0) fail(LSS_EINVAL, "lss_chart_curvature: np must be >= 1");
    if (!uv || !h) fail(LSS_EINVAL, "lss_chart_curvature: chart_uv and h must be non-null");
    build(c);
    const int64_t N = c.ntris * (int64_t)np;
    if (N > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_chart_curvature: ntris * np exceeds 2^31-1");
    if (N == 0) return;
    const bool dev = flags & LSS_PTR_DEVICE;
    DBuf duv, dh, x, xm, grad, hess, o[5];
    upload(c, duv, uv, sizeof(double) * 2 * np, flags);
    const double *ph = h;
    if (!dev) {
        upload(c, dh, h, sizeof(double) * N, 0);
        ph = dh.as<double>();
    }
    x.ensure(sizeof(double) * 3 * N);
    if (c.nmesh > 1) xm.ensure(sizeof(int32_t) * N);
    launch_chart_points(c, duv.as<double>(), np, N, ph, x.as<double>(), c.nmesh > 1 ? xm.as<int32_t>() : nullptr);
    grad.ensure(sizeof(double) * 3 * N);
    hess.ensure(sizeof(double) * 6 * N);
    eval_hessian(c, x.as<double>(), c.nmesh > 1 ? xm.as<int32_t>() : nullptr, N, nullptr, grad.as<double>(),
                 hess.as<double>(), LSS_PTR_DEVICE);
    double *out[5] = {xuu, xuv, xvv, gauss, mean};
    const int width[5] = {3, 3, 3, 1, 1};
    double *q[5];
    for (int k = 0; k < 5; ++k) {
        q[k] = out[k];
        if (!dev && out[k]) {
            o[k].ensure(sizeof(double) * width[k] * N);
            q[k] = o[k].as<double>();
        }
    }
    launch_chart_curvature(c, duv.as<double>(), np, N, ph, grad.as<double>(), hess.as<double>(), q[0], q[1], q[2],
                           q[3], q[4]);
    if (!dev)
        for (int k = 0; k < 5; ++k)
            if (out[k])
                LSS_HIP(hipMemcpyAsync(out[k], q[k], sizeof(double) * width[k] * N, hipMemcpyDeviceToHost,
                                       c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
}

// ------------------------------------------------------------- autotuner
std::string tune_key(const Ctx &c) {
    hipDeviceProp_t prop;
    std::string dev = "gfx";
    if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) dev = prop.gcnArchName;
    std::ostringstream k;
    k << dev << "/tris=" << c.ntris << "/nq=" << c.nq << "/mesh=" << c.nmesh << "/prec=" << c.opt.precision
      << "/far=" << c.opt.far_field << "/p=" << c.opt.fmm_order << "/cut=" << c.opt.cut_factor
      << "/smin=" << c.sigma_min << "/smax=" << c.sigma_max;
    return k.str();
}

bool tune_lookup(const char *path, const std::string &key, lss_options &o) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    auto num = [](const std::string &l, const char *name, double &v) {
        const std::string tag = std::string("\"") + name + "\":";
        const size_t at = l.find(tag);
        if (at == std::string::npos) return false;
        v = atof(l.c_str() + at + tag.size());
        return true;
    };
    while (std::getline(f, line)) {
        const std::string tag = "\"key\": \"" + key + "\"";
        if (line.find(tag) == std::string::npos) continue;
        double v;
        if (num(line, "leaf_shrink", v)) o.leaf_shrink = v;
        if (num(line, "leaf_capacity", v)) o.leaf_capacity = (int32_t)v;
        if (num(line, "tile", v)) o.tile = (int32_t)v;
        if (num(line, "admissibility", v)) o.admissibility = (int32_t)v;
        if (num(line, "fmm_order", v)) o.fmm_order = (int32_t)v;
        found = true;               // the last matching line wins
    }
    return found;
}

void autotune(Ctx &c, const double *x, int64_t n, unsigned flags, double w, const char *path, lss_options *out) {
    if (!c.have_sources || !c.have_sigma) fail(LSS_ESTATE, "lss_autotune: set sources and sigma first");
    if (!x || n < 1) fail(LSS_EINVAL, "lss_autotune: need n >= 1 targets");
    if (n > (int64_t)INT32_MAX) fail(LSS_EINVAL, "lss_autotune: n exceeds 2^31-1");
    if (!(w > 0.0) || !std::isfinite(w)) fail(LSS_EINVAL, "lss_autotune: eval_weight must be positive");
    if (c.nmesh > 1) fail(LSS_EINVAL, "lss_autotune: tunes one mesh at a time (the targets carry no mesh ids)");
    const lss_options base = c.opt;
    const std::string key = tune_key(c);
    lss_options best = base;
    if (tune_lookup(path, key, best)) {
        validate_options(best);
        c.opt = best;
        c.built = false;
        if (out) *out = best;
        return;
    }
    DBuf dx, phi, grad;
    upload(c, dx, x, sizeof(double) * 3 * n, flags);
    phi.ensure(sizeof(double) * n);
    grad.ensure(sizeof(double) * 3 * n);
    // accuracy subset: at most 16384 targets spread evenly over the input,
    // against the exact discrete sum (direct FP64 path). The errors of a
    // truncated expansion are heavy-tailed (a few targets at the edge of an
    // admissible pair), so the subset is large: a few hundred targets have
    // missed a worst case four times their own maximum.
    const int64_t ns = std::min<int64_t>(n, 16384);
    std::vector<double> hx(3 * (size_t)n), hs(3 * (size_t)ns);
    LSS_HIP(hipMemcpyAsync(hx.data(), dx.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c.stream));
    LSS_HIP(hipStreamSynchronize(c.stream));
    for (int64_t i = 0; i < ns; ++i)
        for (int k = 0; k < 3; ++k) hs[3 * i + k] = hx[3 * (i * n / ns) + k];
    std::vector<double> rp(ns), rg(3 * ns), cp(ns), cg(3 * ns);
    c.opt = base;
    c.opt.far_field = LSS_FAR_DIRECT;
    c.opt.precision = LSS_FP64;
    c.built = false;
    eval(c, hs.data(), nullptr, ns, rp.data(), rg.data(), 0);
    double mp = 0.0, mg = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
        mp = std::max(mp, std::fabs(rp[i]));
        mg = std::max(mg, std::sqrt(rg[3 * i] * rg[3 * i] + rg[3 * i + 1] * rg[3 * i + 1] + rg[3 * i + 2] * rg[3 * i + 2]));
    }
    const double bar = 0.25 * (base.precision == LSS_MIXED ? 1e-6 : 1e-12);
    hipEvent_t e0, e1, e2;
    LSS_HIP(hipEventCreate(&e0));
    LSS_HIP(hipEventCreate(&e1));
    LSS_HIP(hipEventCreate(&e2));
    double best_cost = 1e300;
    // cost of one candidate (build + weighted evaluation), or infinity when it
    // misses the accuracy bar on the subset
    auto trial = [&](const lss_options &o) {
        c.opt = o;
        c.built = false;
        LSS_HIP(hipEventRecord(e0, c.stream));
        build(c);
        LSS_HIP(hipEventRecord(e1, c.stream));
        eval(c, dx.as<double>(), nullptr, n, phi.as<double>(), grad.as<double>(), LSS_PTR_DEVICE);
        LSS_HIP(hipEventRecord(e2, c.stream));
        LSS_HIP(hipEventSynchronize(e2));
        float tb = 0, te = 0;
        LSS_HIP(hipEventElapsedTime(&tb, e0, e1));
        LSS_HIP(hipEventElapsedTime(&te, e1, e2));
        eval(c, hs.data(), nullptr, ns, cp.data(), cg.data(), 0);
        double ep = 0.0, eg = 0.0;
        for (int64_t i = 0; i < ns; ++i) {
            ep = std::max(ep, std::fabs(cp[i] - rp[i]));
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) d2 += (cg[3 * i + k] - rg[3 * i + k]) * (cg[3 * i + k] - rg[3 * i + k]);
            eg = std::max(eg, std::sqrt(d2));
        }
        const bool ok = ep <= bar * mp && eg <= bar * mg;
        const double cost = ok ? tb + w * te : 1e300;
        if (cost < best_cost) {
            best_cost = cost;
            best = o;
        }
        return cost;
    };
    try {
        if (base.far_field == LSS_FAR_FMM) {
            const bool mixed = base.precision == LSS_MIXED;
            const int p0 = mixed ? 20 : 26, K0 = mixed ? 4 : 7;
            // stage 1: leaves (shrink over [1, 3], capacity) and tile at the default K and p
            // (written out, so that the choice names them)
            for (double sh : {1.0, 1.25, 1.5, 2.0, 2.5, 3.0})
                for (int cp_ : {64, 256})
                    for (int tl : mixed ? std::vector<int>{64} : std::vector<int>{64, 128}) {
                        lss_options o = base;
                        o.fmm_order = p0;
                        o.admissibility = K0;
                        o.leaf_shrink = sh;
                        o.leaf_capacity = cp_;
                        o.tile = tl;
                        trial(o);
                    }
            // stage 2: admissibility K and order p at the best leaves (order
            // outermost: the translation operators are rebuilt per order)
            const lss_options leaves = best;
            for (int dp : {-4, -2, 0, 2})
                for (int dK : {-1, 0, 2, 4}) {
                    if (dp == 0 && dK == 0) continue;     // timed in stage 1
                    if (K0 + dK < 4) continue;            // below the option's range
                    lss_options o = leaves;
                    o.fmm_order = p0 + dp;
                    o.admissibility = K0 + dK;
                    trial(o);
                }
        } else {
            for (int tl : {64, 128, 256}) {
                lss_options o = base;
                o.tile = tl;
                trial(o);
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        c.opt = base;
        c.built = false;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    if (best_cost >= 1e300) best = base;     // nothing met the bar: keep the caller's options
    c.opt = best;
    c.built = false;
    if (path && best_cost < 1e300) {
        std::ofstream f(path, std::ios::app);
        if (f) {
            char buf[320];
            snprintf(buf, sizeof(buf),
                     ", \"leaf_shrink\": %.3f, \"leaf_capacity\": %d, \"tile\": %d, \"admissibility\": %d, "
                     "\"fmm_order\": %d, \"cost_ms\": %.3f}",
                     best.leaf_shrink, best.leaf_capacity, best.tile, best.admissibility, best.fmm_order, best_cost);
            f << "{\"key\": \"" << key << "\"" << buf << "\n";
        }
    }
    if (out) *out = best;
}

template <class F> int guarded(lss_ctx *ctx, F &&f) {
    if (!ctx) return LSS_EINVAL;
    try {
        LSS_HIP(hipSetDevice(ctx->c.device));
        f(ctx->c);
        ctx->c.err.clear();
        return LSS_OK;
    } catch (const Error &e) {
        ctx->c.err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->c.err = "host allocation failed";
        return LSS_ENOMEM;
    } catch (...) {
        ctx->c.err = "unexpected internal error";
        return LSS_EHIP;
    }
}

}  // namespace
}  // namespace lss

using lss::Ctx;
using lss::DBuf;
using lss::fail;
using lss::upload;

namespace {
thread_local std::string g_create_err;   // message of the last failed lss_create on this thread
}

extern "C" {

int32_t lss_default_rule(double *out, int32_t cap) {
    double r[3 * lss::kDefaultRuleNodes];
    lss::default_rule(r);
    if (out && cap > 0) std::memcpy(out, r, sizeof(double) * 3 * (size_t)std::min<int32_t>(cap, lss::kDefaultRuleNodes));
    return lss::kDefaultRuleNodes;
}

int lss_create(lss_ctx **out, int hip_device, void *hip_stream) {
    g_create_err.clear();
    if (!out) { g_create_err = "lss_create: out is null"; return LSS_EINVAL; }
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        g_create_err = std::string("lss_create: hipGetDeviceCount: ") + hipGetErrorString(e) +
                       " (devices: " + std::to_string(ndev) + ")";
        return LSS_EHIP;
    }
    if (hip_device < 0 || hip_device >= ndev) { g_create_err = "lss_create: device index out of range"; return LSS_EINVAL; }
    // look up the allocation-free path's scratch array on this device now (a
    // failure is reported by lss_eval_noalloc, not here)
    if (hipSetDevice(hip_device) == hipSuccess) (void)lss::noalloc_scratch(hip_device, nullptr);
    lss_ctx *ctx = new (std::nothrow) lss_ctx;
    if (!ctx) return LSS_ENOMEM;
    ctx->c.device = hip_device;
    ctx->c.stream = static_cast<hipStream_t>(hip_stream);
    *out = ctx;
    return LSS_OK;
}

void lss_destroy(lss_ctx *ctx) {
    if (!ctx) return;
    Ctx &c = ctx->c;
    (void)hipSetDevice(c.device);
    (void)hipStreamSynchronize(c.stream);
    DBuf *bufs[] = {&c.verts, &c.tris, &c.tris6, &c.tri_off, &c.node_off, &c.rule, &c.sigma, &c.src, &c.vH, &c.tkey,
                    &c.tkey2, &c.tperm, &c.tperm2, &c.tx, &c.ty, &c.tz, &c.tmesh, &c.sort_tmp, &c.pairs, &c.tile_queue, &c.tile_order, &c.tile_bucket,
                    &c.tflag, &c.tpos, &c.tstart, &c.ntiles, &c.tleaf,
                    &c.ns.T, &c.ns.H, &c.ns.h, &c.ns.lo, &c.ns.hi, &c.ns.sig, &c.ns.mesh, &c.ns.orig,
                    &c.ns.status, &c.ns.iters, &c.ns.seen, &c.ns.active, &c.ns.active2, &c.ns.flag, &c.ns.blocksum,
                    &c.ns.nact, &c.ns.hist};
    lss::drop_newton_graph(c.ns);
    for (DBuf *b : bufs) b->release();
    if (c.capture_stream) (void)hipStreamDestroy(c.capture_stream);
    if (c.aux_stream) (void)hipStreamDestroy(c.aux_stream);
    for (hipEvent_t e : c.aux_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c.ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : c.ev_stop) (void)hipEventDestroy(e);
    delete ctx;
}

const char *lss_last_error(const lss_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_create_err.c_str(); }

int lss_synchronize(lss_ctx *ctx) {
    return lss::guarded(ctx, [&](Ctx &c) { LSS_HIP(hipStreamSynchronize(c.stream)); });
}

int lss_set_sources(lss_ctx *ctx, const double *verts, int64_t nverts, const int32_t *tris, int64_t ntris,
                    const int64_t *mesh_tri_offsets, int32_t nmesh, const double *rule_uvw, int32_t nq,
                    unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) {
        if (!verts || !tris) fail(LSS_EINVAL, "lss_set_sources: null pointer");
        if (!rule_uvw && nq != 0 && nq != lss::kDefaultRuleNodes)
            fail(LSS_EINVAL, "lss_set_sources: rule_uvw == NULL (default rule) needs nq 0 or 12");
        if (!rule_uvw) nq = lss::kDefaultRuleNodes;
        if (nverts < 3 || ntris < 1 || nq < 1) fail(LSS_EINVAL, "lss_set_sources: need nverts >= 3, ntris >= 1, nq >= 1");
        if (nverts > (int64_t)INT32_MAX || ntris * (int64_t)nq > ((int64_t)1 << 40))
            fail(LSS_EINVAL, "lss_set_sources: mesh too large");
        if (mesh_tri_offsets == nullptr && nmesh > 1) fail(LSS_EINVAL, "lss_set_sources: nmesh > 1 needs offsets");
        if (nmesh < 0) fail(LSS_EINVAL, "lss_set_sources: nmesh < 0");
        const bool dev = flags & LSS_PTR_DEVICE;
        const bool quad = flags & LSS_TRI6;
        const int nvt = quad ? 6 : 3;
        c.have_sources = false;
        c.have_sigma = false;
        c.built = false;
        // mesh offsets: validated on the host (copied there if on the device)
        int32_t nm = (mesh_tri_offsets && nmesh >= 1) ? nmesh : 1;
        std::vector<int64_t> off(nm + 1);
        if (mesh_tri_offsets && nmesh >= 1) {
            LSS_HIP(hipMemcpy(off.data(), mesh_tri_offsets, sizeof(int64_t) * (nm + 1),
                              dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
        } else {
            off[0] = 0;
            off[1] = ntris;
        }
        if (off[0] != 0 || off[nm] != ntris) fail(LSS_EINVAL, "lss_set_sources: offsets must start at 0 and end at ntris");
        for (int32_t m = 0; m < nm; ++m)
            if (off[m + 1] < off[m]) fail(LSS_EINVAL, "lss_set_sources: offsets must be non-decreasing");
        std::vector<double> hrule(3 * (size_t)nq);
        if (rule_uvw)
            LSS_HIP(hipMemcpy(hrule.data(), rule_uvw, sizeof(double) * 3 * nq,
                              dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
        else
            lss::default_rule(hrule.data());
        for (int m = 0; m < nq; ++m)
            if (!std::isfinite(hrule[3 * m]) || !std::isfinite(hrule[3 * m + 1]) || !std::isfinite(hrule[3 * m + 2]))
                fail(LSS_EINVAL, "lss_set_sources: rule entries must be finite");
        upload(c, c.verts, verts, sizeof(double) * 3 * nverts, flags);
        if (quad) {
            upload(c, c.tris6, tris, sizeof(int32_t) * 6 * ntris, flags);
            c.tris.ensure(sizeof(int32_t) * 3 * ntris);
            hipLaunchKernelGGL(lss::k_corners, dim3(lss::grid_for(ntris)), dim3(256), 0, c.stream, ntris,
                               c.tris6.as<int32_t>(), c.tris.as<int32_t>());
            LSS_CHECK_LAUNCH("k_corners");
        } else {
            upload(c, c.tris, tris, sizeof(int32_t) * 3 * ntris, flags);
            c.tris6.release();
        }
        upload(c, c.rule, hrule.data(), sizeof(double) * 3 * nq, 0);
        c.tri_off.ensure(sizeof(int64_t) * (nm + 1));
        LSS_HIP(hipMemcpyAsync(c.tri_off.p, off.data(), sizeof(int64_t) * (nm + 1), hipMemcpyHostToDevice, c.stream));
        std::vector<int64_t> noff(nm + 1);
        for (int32_t m = 0; m <= nm; ++m) noff[m] = off[m] * nq;
        c.node_off.ensure(sizeof(int64_t) * (nm + 1));
        LSS_HIP(hipMemcpyAsync(c.node_off.p, noff.data(), sizeof(int64_t) * (nm + 1), hipMemcpyHostToDevice, c.stream));
        // index and coordinate checks on the device
        DBuf bad;
        bad.ensure(16);
        LSS_HIP(hipMemsetAsync(bad.p, 0, 16, c.stream));
        hipLaunchKernelGGL(lss::k_check_tris, dim3(lss::grid_for(nvt * ntris)), dim3(256), 0, c.stream, nvt * ntris,
                           (quad ? c.tris6 : c.tris).as<int32_t>(), nverts, bad.as<unsigned long long>());
        hipLaunchKernelGGL(lss::k_check_verts, dim3(lss::grid_for(3 * nverts)), dim3(256), 0, c.stream, 3 * nverts,
                           c.verts.as<double>(), bad.as<unsigned long long>() + 1);
        unsigned long long nb[2] = {0, 0};
        LSS_HIP(hipMemcpyAsync(nb, bad.p, 16, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (nb[0]) fail(LSS_EINVAL, "lss_set_sources: triangle vertex index outside [0, nverts)");
        if (nb[1]) fail(LSS_EINVAL, "lss_set_sources: non-finite vertex coordinate");
        c.nverts = nverts;
        c.ntris = ntris;
        c.nmesh = nm;
        c.nq = nq;
        c.quadratic = quad;
        c.h_tri_off = off;
        std::vector<double> vol;
        int64_t ndeg = 0;
        double vmin = lss::launch_check_orientation(c, vol, ndeg);
        c.stats = lss_stats{};
        c.stats.n_degenerate = ndeg;
        if (!(vmin > 0.0)) fail(LSS_EORIENT, "lss_set_sources: a mesh has non-positive signed volume (inward orientation?)");
        c.have_sources = true;
        ++c.sources_gen;
    });
}

int lss_set_sigma(lss_ctx *ctx, const double *sigma, int64_t n, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) {
        if (!c.have_sources) fail(LSS_ESTATE, "lss_set_sigma: call lss_set_sources first");
        if (!sigma) fail(LSS_EINVAL, "lss_set_sigma: null pointer");
        if (n != 1 && n != c.ntris) fail(LSS_EINVAL, "lss_set_sigma: n must be 1 or ntris");
        c.have_sigma = false;
        c.built = false;
        DBuf in, stat;
        upload(c, in, sigma, sizeof(double) * n, flags);
        c.sigma.ensure(sizeof(double) * c.ntris);
        stat.ensure(24);
        unsigned long long init[3] = {0ull, ~0ull, 0ull};
        LSS_HIP(hipMemcpyAsync(stat.p, init, 24, hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(lss::k_sigma_set, dim3(lss::grid_for(c.ntris)), dim3(256), 0, c.stream, c.ntris,
                           in.as<double>(), n, c.sigma.as<double>(), stat.as<unsigned long long>());
        LSS_CHECK_LAUNCH("k_sigma_set");
        unsigned long long h[3];
        LSS_HIP(hipMemcpyAsync(h, stat.p, 24, hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (h[0]) fail(LSS_EINVAL, "lss_set_sigma: sigma must be positive and finite");
        double mn, mx;
        std::memcpy(&mn, &h[1], 8);
        std::memcpy(&mx, &h[2], 8);
        c.sigma_min = mn;
        c.sigma_max = mx;
        c.have_sigma = true;
    });
}

int lss_set_options(lss_ctx *ctx, const lss_options *opt) {
    return lss::guarded(ctx, [&](Ctx &c) {
        lss_options o{};
        if (opt) o = *opt;
        lss::validate_options(o);
        if (o.precision != c.opt.precision || o.far_field != c.opt.far_field || o.fmm_order != c.opt.fmm_order ||
            o.leaf_capacity != c.opt.leaf_capacity || o.cut_factor != c.opt.cut_factor ||
            o.leaf_shrink != c.opt.leaf_shrink || o.admissibility != c.opt.admissibility ||
            o.curved_charts != c.opt.curved_charts)
            c.built = false;
        c.opt = o;
    });
}

int lss_get_options(const lss_ctx *ctx, lss_options *out) {
    if (!ctx || !out) return LSS_EINVAL;
    *out = ctx->c.opt;
    return LSS_OK;
}

int lss_build(lss_ctx *ctx) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::build(c); });
}

int lss_eval(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n, double *phi, double *grad,
             unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::eval(c, x, x_mesh, n, phi, grad, flags); });
}

int lss_eval_noalloc(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n, double *phi, double *grad,
                     unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::eval_noalloc(c, x, x_mesh, n, phi, grad, flags); });
}

int lss_project(lss_ctx *ctx, const double *chart_uv, int32_t np, double *h, double *xout, int8_t *status,
                int8_t *iters, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::project(c, chart_uv, np, h, xout, status, iters, flags); });
}

int lss_eval_hessian(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n, double *phi, double *grad,
                     double *hess, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::eval_hessian(c, x, x_mesh, n, phi, grad, hess, flags); });
}

int lss_eval_multiscale(lss_ctx *ctx, double lambda, double sigma0, const double *x, const int32_t *x_mesh,
                        int64_t n, double *phi, double *grad, double *sigma_x, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) {
        lss::eval_multiscale(c, lambda, sigma0, x, x_mesh, n, phi, grad, sigma_x, flags);
    });
}

int lss_chart_curvature(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *h, double *xuu,
                        double *xuv, double *xvv, double *gauss, double *mean, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) {
        lss::chart_curvature(c, chart_uv, np, h, xuu, xuv, xvv, gauss, mean, flags);
    });
}

int lss_chart_geometry(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *h, double *xu, double *xv,
                       double *da, double *normal, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::chart_geometry(c, chart_uv, np, h, xu, xv, da, normal, flags); });
}

int lss_chart_interp(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *f, int32_t ncomp,
                     const double *eval_uv, int32_t ne, double *out, unsigned flags) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::chart_interp(c, chart_uv, np, f, ncomp, eval_uv, ne, out, flags); });
}

int lss_autotune(lss_ctx *ctx, const double *x, int64_t n, unsigned flags, double eval_weight,
                 const char *cache_path, lss_options *out) {
    return lss::guarded(ctx, [&](Ctx &c) { lss::autotune(c, x, n, flags, eval_weight, cache_path, out); });
}

int lss_get_stats(const lss_ctx *ctx, lss_stats *out) {
    if (!ctx || !out) return LSS_EINVAL;
    Ctx &c = const_cast<lss_ctx *>(ctx)->c;
    if (c.ev_pending) {
        (void)hipSetDevice(c.device);
        double ms = 0.0;
        for (int k = 0; k < c.ev_used; ++k) {
            float t = 0.0f;
            if (hipEventSynchronize(c.ev_stop[k]) != hipSuccess ||
                hipEventElapsedTime(&t, c.ev_start[k], c.ev_stop[k]) != hipSuccess) {
                c.err = "lss_get_stats: event timing failed";
                return LSS_EHIP;
            }
            ms += t;
        }
        c.stats.pair_kernel_ms = ms;
        c.stats.pair_kernel_launches = c.ev_used;
        c.ev_pending = false;
    }
    if (c.pairs_pending) {
        double pr[4] = {0.0, 0.0, 0.0, 0.0};
        (void)hipSetDevice(c.device);
        if (hipMemcpyAsync(pr, c.pairs.p, 4 * sizeof(double), hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
            hipStreamSynchronize(c.stream) != hipSuccess) {
            c.err = "lss_get_stats: reading the pair counter failed";
            return LSS_EHIP;
        }
        c.stats.last_pairs = pr[0];
        c.stats.lane_pairs = pr[1];
        c.stats.useful_pairs = c.opt.far_field == LSS_FAR_FMM ? pr[2] : pr[0];
        c.stats.dipole_pairs = c.opt.far_field == LSS_FAR_FMM ? pr[3] : 0.0;
        c.pairs_pending = false;
    }
    *out = c.stats;
    return LSS_OK;
}

}  // extern "C"
