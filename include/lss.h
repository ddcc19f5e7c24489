/*
 * lss.h -- C ABI of liblss, the MI355X (gfx950) evaluator of the smoothed
 * level-set function of a triangulated solid and of its chart projection.
 *
 * Method (Vico, Greengard, O'Neil, Rachh, "A fast boundary integral method
 * for high-order multiscale mesh generation"):
 *   Phi(x) is the Gaussian-smoothed indicator of the solid bounded by a flat
 *   skeleton triangulation (section 2, eq. basemodelg).  By the divergence
 *   theorem (section 4.1, eq. surf / kerpsi) it is a surface integral, and
 *   after quadrature on every triangle (section 4.3, eq. discrete_int)
 *
 *     Phi(x)  = sum_k  -(a_k . d_k) K_k(rho_k),        d_k = x - y_k, rho_k = |d_k|
 *     grad Phi(x) = sum_k [ -a_k K_k(rho_k) - (a_k . d_k) K_k'(rho_k)/rho_k d_k ]
 *
 *   over quadrature nodes y_k = P1 + u_m (P2-P1) + v_m (P3-P1) of triangle j,
 *   a_k = w_m (P2-P1) x (P3-P1), and
 *     K(rho) = erf(u)/(4 pi rho^3) - sqrt(2/pi) e^{-u^2}/(4 pi sigma rho^2),
 *     u = rho/(sqrt 2 sigma), sigma = sigma_j (width of the source triangle).
 *   Far from the node (rho >= 8 sigma) K is the Laplace dipole factor
 *   1/(4 pi rho^3) (section 4.4, eq. kerapprox / kerdecomp).
 *   The gradient is the exact derivative of the discrete sum (the paper's
 *   printed eq. gradPhi has a sign slip in its second term).
 *   Chart projection (section 3, eq. h / newton / newtonderiv; section 3.2,
 *   eq. newtoneq): for chart node (u_i, v_i) on triangle j, find h with
 *   Phi(T(u_i,v_i) + h H(u_i,v_i)) = 1/2 by Newton's method from h = 0, with
 *   T the flat triangle (eq. tparam) and H the linear pseudonormal field
 *   (eq. mkvertexpn, mkpseudovec).
 *
 * Conventions shared by every entry point
 *   - Every function returns LSS_OK (0) or a positive LSS_E* code; the
 *     message of the last failure on a context is lss_last_error(ctx).
 *     No C++ exception crosses this boundary.
 *   - Pointers are host memory unless LSS_PTR_DEVICE is set in `flags`, in
 *     which case every array argument of that call is HIP device memory of
 *     the context's device.  With host pointers a call is synchronous: it
 *     returns when outputs are written.  With device pointers the work is
 *     queued on the context's stream and the call returns without waiting
 *     (inputs must stay valid, outputs are defined, once the stream reaches
 *     that point; lss_synchronize() waits).
 *   - The caller owns every buffer it passes.  set_* calls copy their inputs
 *     into context-owned device memory, so caller buffers may be released
 *     after the call (host) or after the stream passes it (device).  The
 *     library never hands out memory for the caller to free.
 *   - A context is used by one host thread at a time.  Different contexts
 *     may run concurrently on different streams.
 *   - Row-major layouts: verts (nverts, 3) double; tris (ntris, 3) int32 with
 *     0-based indices, counter-clockwise seen from outside (outward
 *     orientation); targets (n, 3) double; grad (n, 3) double.
 */
#ifndef LSS_H
#define LSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lss_ctx lss_ctx;

/* return codes */
enum {
    LSS_OK = 0,
    LSS_EINVAL = 1,   /* bad argument: null pointer, negative or zero size, index out of range,
                         sigma <= 0 or not finite, unknown option value */
    LSS_ENOMEM = 2,   /* device or host allocation failed */
    LSS_EHIP = 3,     /* HIP runtime error (message names the call) */
    LSS_ESTATE = 4,   /* called out of order, e.g. lss_eval before lss_set_sources / lss_set_sigma */
    LSS_EORIENT = 5   /* a mesh has non-positive signed volume (inward or open orientation) */
};

/* arithmetic of the pair evaluations */
enum {
    LSS_FP64 = 0,     /* every pair, sum and update in FP64 (target: 1e-12 relative to the oracle) */
    LSS_MIXED = 1     /* pair kernel in FP32 with FP32 chunk sums folded by two-sum into
                         float-float accumulators; positions differenced in FP64 before rounding;
                         far field expansions, Newton update and bracketing in FP64
                         (target: 1e-6 relative to the oracle) */
};

/* far-field treatment */
enum {
    LSS_FAR_DIRECT = 0,  /* every (target, node) pair with the full kernel: exact discrete sum */
    LSS_FAR_FMM = 1      /* octree: pairs in adjacent leaves with the full kernel, the rest by a
                            Laplace-dipole fast multipole method (section 4.4, eq. kerdecomp) */
};

/* per chart node status written by lss_project */
enum {
    LSS_NODE_CONVERGED = 0,
    LSS_NODE_MAXITER = 1,     /* not converged after max_iter iterations */
    LSS_NODE_NOBRACKET = 2,   /* no root near the skeleton: a bisection step went past |h| > 3/4 hmax
                                 (hmax = 16 sigma_j/|H|) before Phi - 1/2 changed sign, or the
                                 iteration cap was reached with |h| > hmax/2 */
    LSS_NODE_DEGENERATE_H = 3 /* |H| < 1e-3: no usable pseudonormal direction */
};

#define LSS_PTR_DEVICE 1u
/* lss_set_sources: tris holds six indices per triangle (quadratic skeleton) */
#define LSS_TRI6 2u

typedef struct lss_options {
    int32_t precision;        /* LSS_FP64 (default) or LSS_MIXED */
    int32_t far_field;        /* LSS_FAR_DIRECT (default) or LSS_FAR_FMM */
    int32_t fmm_order;        /* multipole order p for LSS_FAR_FMM (M2L classes farther than the
                                 closest admissible one are translated at the lower order that
                                 reaches the same truncation error, plus two); 0 = default for the
                                 precision (26 FP64, 20 MIXED) */
    int32_t leaf_capacity;    /* octree: a box splits while more than this many of its nodes have a
                                 cut radius <= leaf_shrink x its children's side; 0 = default 64 */
    double  cut_factor;       /* near/far cut radius in units of the source sigma; the near list of
                                 a leaf covers every node within cut_factor * sigma_node;
                                 0 = default (8 for FP64, sqrt(40) for MIXED) */
    double  newton_tau;       /* converged when |h_k - h_{k-1}| <= newton_tau * sigma_j;
                                 0 = default (1e-12 FP64, 1e-6 MIXED) */
    int32_t newton_max_iter;  /* 0 = default 40 */
    int32_t tile;             /* targets per workgroup of the pair kernels: 64, 128 or 256; 0 = default
                                 (direct sum 256; FMM 64; the mixed FMM kernel always uses 64) */
    double  leaf_shrink;      /* LSS_FAR_FMM: boxes may be as narrow as (cut radius of their nodes) /
                                 leaf_shrink (see leaf_capacity); M2L needs a Euclidean gap between
                                 the boxes >= the source box's largest cut radius.
                                 0 = default (2 for FP64, 1.5 for MIXED); otherwise in [1, 3] */
    int32_t count_useful;     /* LSS_FAR_FMM: nonzero makes the evaluation kernels also count the
                                 pairs inside the cut (lss_stats.useful_pairs), at a small cost in
                                 speed; 0 = off (useful_pairs stays 0 for the FMM path) */
    int32_t admissibility;    /* LSS_FAR_FMM: K of the multipole-to-local criterion |v|^2 >= K for
                                 boxes v sides apart (a larger K needs a lower fmm_order for the
                                 same accuracy but leaves more pairs to the near lists);
                                 0 = default (4 MIXED, 7 FP64); otherwise in [4, 18] */
    int32_t curved_charts;    /* quadratic skeletons (LSS_TRI6): nonzero puts the chart bases on the
                                 curved patches (T(u,v) the quadratic patch, H linear in the
                                 vertex pseudonormals of the curved triangles: their corner
                                 normals y_u x y_v weighted by their corner angles); 0 = bases on
                                 the corner triangles.  No effect on flat skeletons. */
    int32_t sigma_interp;     /* how lss_eval_multiscale with LSS_FAR_FMM forms sigma(x): 0 = automatic
                                 (interpolated when the cells' nodes number under a quarter of the
                                 points, else the direct sum), 1 = always the direct sum, 2 =
                                 interpolated wherever the cell grid applies */
    int32_t reserved[2];      /* must be zero */
} lss_options;

typedef struct lss_stats {
    int64_t n_tris;           /* triangles of the current source set */
    int64_t n_nodes;          /* quadrature nodes (sources) = n_tris * nq */
    int32_t n_mesh;
    int32_t fmm_order;        /* order used by the last build (0 in direct mode) */
    int64_t n_leaves;         /* octree leaves (0 in direct mode) */
    int64_t n_boxes;          /* octree boxes */
    int64_t n_m2l;            /* multipole-to-local translations of the last build */
    int32_t tree_depth;
    int32_t newton_iters;     /* iterations run by the last lss_project */
    int64_t last_targets;     /* targets of the last lss_eval, or target evaluations summed over
                                 the iterations of the last lss_project */
    double  last_pairs;       /* pair-kernel evaluations of the last lss_eval / lss_project */
    int64_t n_degenerate;     /* zero-area triangles in the source set (they contribute nothing) */
    double  pair_kernel_ms;   /* device time from HIP events recorded on the context stream
                                 (reading it waits for them): for lss_eval, around the
                                 pair-kernel launches; for lss_project, around the launches of
                                 the captured Newton iterations (target update, evaluation,
                                 Newton step and compaction together) */
    int32_t pair_kernel_launches;  /* lss_eval: pair-kernel launches timed in pair_kernel_ms;
                                      lss_project: timed launches of Newton iterations (graphs of
                                      8 iterations; with LSS_FAR_FMM the first iteration runs on
                                      its own, and the active list is re-ordered by leaf before
                                      every graph launch) */
    int32_t pad0;
    double  lane_pairs;       /* pair evaluations the pair kernels spent, idle lanes of partly
                                 filled tiles included (last_pairs / lane_pairs = lane use) */
    int64_t n_m2p;            /* (leaf, box) pairs of the last build whose far field reaches the
                                 leaf's targets straight from the box's multipole expansion */
    double  useful_pairs;     /* pairs of the last lss_eval / lss_project whose distance is inside
                                 the cut of their node (rho < cut_factor * sigma): the work the
                                 method itself asks for (section 4.4: the near field is the ball of
                                 radius cut around the target).  LSS_FAR_DIRECT: every pair (the
                                 exact sum has no cut).  LSS_FAR_FMM: counted only with
                                 lss_options.count_useful, else 0.  last_pairs / useful_pairs is
                                 the overhead of evaluating whole leaves of the near lists. */
    double  dipole_pairs;     /* LSS_FAR_FMM with lss_options.count_useful (LSS_MIXED, or LSS_FP64
                                 with 64-target tiles): pairs of the last lss_eval / lss_project
                                 taken by the dipole-only loop (near-list nodes beyond their cut
                                 radius of every target of their tile, summed with the far kernel
                                 pair by pair); last_pairs - dipole_pairs went through the full
                                 kernel.  Otherwise 0. */
} lss_stats;

/* Create a context on HIP device `hip_device`, queuing work on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context or NULL on failure. */
int lss_create(lss_ctx **out, int hip_device, void *hip_stream);

/* Release the context and all its device memory (waits for its stream). NULL is a no-op. */
void lss_destroy(lss_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call on ctx.
 * With ctx == NULL: the message of the last failed lss_create on the calling thread. */
const char *lss_last_error(const lss_ctx *ctx);

/* Wait until all work queued on the context's stream has finished. */
int lss_synchronize(lss_ctx *ctx);

/* Set the skeleton mesh (section 3: water-tight, positively oriented flat
 * triangles) and the quadrature rule on T0 (section 4.3).
 *   verts (nverts,3), tris (ntris,3): see conventions; nverts, ntris >= 1.
 *   mesh_tri_offsets: CSR of length nmesh+1 splitting the triangles into
 *     independent meshes (a ragged batch); offsets[0] = 0, non-decreasing,
 *     offsets[nmesh] = ntris.  NULL (with nmesh 0 or 1) = one mesh.
 *   rule_uvw (nq,3): nodes (u_m, v_m) on T0 and weights w_m (sum 1/2), nq >= 1;
 *     NULL selects the default rule of lss_default_rule (Dunavant's 12-node
 *     degree-6 rule, standing in for the paper's Vioreanu-Rokhlin rules of
 *     section 4.3); nq must then be 0 or 12.
 * Indices outside [0, nverts) give LSS_EINVAL.  A mesh with signed volume
 * <= 0 gives LSS_EORIENT.  Invalidates sigma-dependent state: lss_set_sigma
 * must follow before lss_build / lss_eval / lss_project.
 * With LSS_TRI6 in flags the skeleton is quadratic (section on quadratic
 * skeletons: second-order curvilinear triangles): tris is (ntris,6), the
 * corners P1 P2 P3 in the order above, then the edge points P4 (edge P1P2),
 * P5 (P2P3), P6 (P3P1), shared by the two triangles of an edge.  The patch is
 * y(u,v) = sum_k N_k(u,v) P_k with the quadratic Lagrange shape functions
 * and each node carries w (y_u x y_v).  The orientation check uses the
 * corner triangles P1 P2 P3; the vertex pseudonormals and the chart bases of
 * lss_project / lss_chart_geometry / lss_chart_curvature use the corner
 * triangles too, or the curved patches with lss_options.curved_charts; Phi
 * sums the curved triangles. */
int lss_set_sources(lss_ctx *ctx,
                    const double *verts, int64_t nverts,
                    const int32_t *tris, int64_t ntris,
                    const int64_t *mesh_tri_offsets, int32_t nmesh,
                    const double *rule_uvw, int32_t nq,
                    unsigned flags);

/* The default source quadrature rule (section 4.3 asks for a high-order rule
 * for smooth functions on each triangle): the 12-node symmetric degree-6 rule
 * of Dunavant on T0, as rows (u_m, v_m, w_m) with sum w_m = 1/2, exact for
 * polynomials of total degree <= 6.  Writes min(cap, 12) rows to out (host
 * memory; NULL or cap <= 0 writes nothing) and returns 12.  Needs no device
 * and no context. */
int32_t lss_default_rule(double *out, int32_t cap);

/* Set the smoothing width (section 2: sigma_j attached to triangle j).
 *   n == 1: one constant sigma; n == ntris: one sigma per triangle.
 * Any sigma <= 0 or not finite gives LSS_EINVAL. */
int lss_set_sigma(lss_ctx *ctx, const double *sigma, int64_t n, unsigned flags);

/* Set options (NULL = all defaults).  Unknown values give LSS_EINVAL. */
int lss_set_options(lss_ctx *ctx, const lss_options *opt);
int lss_get_options(const lss_ctx *ctx, lss_options *out);

/* Prepare everything that depends only on sources, sigma and options:
 * quadrature nodes and folded constants, vertex pseudonormals, and for
 * LSS_FAR_FMM the octree, interaction lists, multipole and local expansions.
 * Idempotent; eval / project call it implicitly when state is stale. */
int lss_build(lss_ctx *ctx);

/* Phi and grad Phi at n targets x (n,3).  x_mesh (n) gives, for a batch
 * with nmesh > 1, the mesh whose nodes are summed for each target (NULL is
 * allowed only for nmesh == 1); values outside [0, nmesh) give LSS_EINVAL
 * (device arrays too: a check kernel runs and the call waits for it).
 * phi (n), grad (n,3) receive the results; grad may be NULL.  n == 0 is a
 * no-op.  Non-finite targets give NaN outputs.  With LSS_FAR_FMM a target
 * outside its mesh's root cube (the node bounding box padded by twice the
 * largest cut radius) gets its field from a walk of that mesh's tree:
 * multipole expansions of the boxes far enough from it, direct sums of the
 * leaves that are not. */
int lss_eval(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n,
             double *phi, double *grad, unsigned flags);

/* Allocation-free evaluation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): lss_eval's evaluation, same kernels in the same order, with
 * every per-call buffer (target copies, sort keys and workspace, tile lists)
 * in a static device array of the library (48 MiB per device, held until the
 * process ends) instead of context allocations.  Results equal lss_eval's bit
 * for bit.  Differences from lss_eval:
 *   - device pointers only: flags must contain LSS_PTR_DEVICE (else EINVAL);
 *   - n <= LSS_NOALLOC_MAX_TARGETS (else EINVAL; call lss_eval instead);
 *   - the context must already be built (lss_build, or any call that builds,
 *     after the last set_* call), else ESTATE: this call does not build;
 *   - lss_get_stats is not updated (no counters, no timing events);
 *   - every call on one device shares the array: calls that overlap on one
 *     device (contexts on different streams of that device) race; calls
 *     ordered on one stream do not.  The array keeps the last call's
 *     contents; what must start at zero is cleared by a kernel, not a memset.
 * It calls no hipMalloc / hipFree and no allocating library routine.  With a
 * batch (nmesh > 1) it checks x_mesh first and waits for that check, as
 * lss_eval does; otherwise it returns without waiting (outputs are defined
 * once the context stream passes the call).  Arguments as for lss_eval. */
#define LSS_NOALLOC_MAX_TARGETS 524288
int lss_eval_noalloc(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n, double *phi, double *grad,
                     unsigned flags);

/* Chart projection onto Phi = 1/2 for np chart nodes (u_i, v_i) on T0,
 * chart_uv (np,2), on every triangle.  Output index j*np + i (triangle
 * major): h (ntris*np) pseudonormal distance, xout (ntris*np, 3) projected
 * point T + h H, status (ntris*np) LSS_NODE_*, iters (ntris*np) Newton
 * iterations used.  xout, status and iters may be NULL.  Each iteration
 * evaluates Phi and grad Phi only at nodes that have not converged. */
int lss_project(lss_ctx *ctx, const double *chart_uv, int32_t np,
                double *h, double *xout, int8_t *status, int8_t *iters,
                unsigned flags);

/* Chart geometry at the chart nodes of every triangle (section 3.1: eq. chart,
 * u_vector, U_vector_2, v_vector, v_vector_2, eq. da), for distances h from
 * lss_project (index j * np + i, the same chart_uv).  With x = T + h H the
 * function evaluates grad Phi at x (as lss_eval, with the context's options)
 * and writes per node:
 *   xu, xv (N,3): x_u = T_u + h H_u + (dh/du) H with dh/du = -(T_u + h H_u) . grad Phi
 *                 / (H . grad Phi), and likewise in v (T and H are linear on the
 *                 triangle, so T_u = P2 - P1, H_u = H2 - H1, T_v = P3 - P1, H_v = H3 - H1);
 *   da (N):       |x_u x x_v|, the area element per du dv of the standard simplex;
 *   normal (N,3): the outward unit normal -grad Phi / |grad Phi| (Phi grows inward).
 * N = ntris * np.  Any output may be NULL.  Nodes with H . grad Phi = 0 or a
 * zero gradient get non-finite values.  Host or device arrays as for lss_project;
 * the call returns when the outputs are written. */
int lss_chart_geometry(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *h, double *xu, double *xv,
                       double *da, double *normal, unsigned flags);

/* Hessian of Phi (section 3.1: needed for the charts' second derivatives,
 * eq. uu_vector_aux1/aux2), with Phi and grad Phi from the same pass, at n
 * targets x (n,3); x_mesh as for lss_eval.  hess (n,6) receives the
 * symmetric matrix as xx, xy, xz, yy, yz, zz; phi (n) and grad (n,3) may be
 * NULL.  Pairs are summed in FP64 with the full kernel and its third radial
 * function G = F'(rho)/rho.  LSS_FAR_DIRECT: every (target, node) pair of the
 * target's mesh (cost n times the mesh's node count).  LSS_FAR_FMM: the
 * context's octree: the near lists with the full kernel, the M2P lists and
 * the leaf's local expansion with their second derivatives (targets outside
 * the root cube: every node of their mesh).  The accuracy follows the
 * context's cut and order: about 1e-13 relative with the FP64 settings,
 * 1e-7 with the mixed ones (whose cut and order are smaller); the
 * precision option does not change the pair arithmetic.  Host or device
 * arrays per flags; returns when the outputs are written. */
int lss_eval_hessian(lss_ctx *ctx, const double *x, const int32_t *x_mesh, int64_t n, double *phi, double *grad,
                     double *hess, unsigned flags);

/* Phi and grad Phi with the target-attached width of section 2 (eq.
 * basemodelk, convkernel, sigma2) instead of the per-triangle sigma of
 * lss_set_sigma: for a target x of mesh m,
 *   sigma(x) = sum_j sigma_j w_j / sum_j w_j,  w_j = exp(-|x - c_j|^2 / (2 sigma0^2)),
 * over the triangles j of mesh m, c_j the centroid and sigma_j = D_j / lambda
 * with D_j the diameter of the smallest ball enclosing the (corner) triangle;
 * sigma0 > 0 as given, or sigma0 == 0 for sqrt(5) max_j D_j of the mesh (the
 * paper's suggestion, with lambda about 2.5).  Phi sums every node of the
 * mesh with width sigma(x); grad Phi is the exact x-derivative, including
 * (dPhi/dsigma) grad sigma.  x (n,3), x_mesh as for lss_eval; phi (n); grad
 * (n,3) and sigma_x (n, receives sigma(x)) may be NULL.
 * LSS_FAR_DIRECT: sigma(x) is a direct FP64 sum over the centroids of the
 * target's mesh and Phi a direct FP64 sum over the mesh's nodes.
 * LSS_FAR_FMM: sigma(x) and grad sigma come from the direct sum, or (option
 * sigma_interp) from tensor Chebyshev interpolation of the weight sums
 * sum_j w_j, sum_j sigma_j w_j and their first moments in cells of side
 * 1.5 sigma0 (17 nodes per axis, each node value a direct FP64 sum; the
 * interpolation error is below the sums' own rounding), with the direct sum
 * for points outside the cells or farther than 3 sigma0 from every centroid.
 * The octree is built with leaves sized by sigma(x) at the centroids, the
 * near lists are cut per box at the largest sigma(x) of its targets and
 * summed at each target's width, and the far field comes from the
 * expansions (accuracy as for lss_eval with the same options); the
 * context's own sigma is left as it was, and its built state is rebuilt on
 * the next call that needs it.  Needs sources, not sigma (LSS_ESTATE
 * otherwise).
 * lambda <= 0, sigma0 < 0 or non-finite give LSS_EINVAL.  Host or device
 * arrays per flags; returns when the outputs are written. */
int lss_eval_multiscale(lss_ctx *ctx, double lambda, double sigma0, const double *x, const int32_t *x_mesh,
                        int64_t n, double *phi, double *grad, double *sigma_x, unsigned flags);

/* Second derivatives and curvatures of the charts x = T + h H at the chart
 * nodes (section 3.1, eq. uu_vector, uu_vector_aux1, uu_vector_aux2 and the
 * analogous uv, vv expressions), for distances h (ntris*np) from
 * lss_project.  T and H are linear on the (corner) triangle, so with
 * B = grad grad Phi (from lss_eval_hessian's sum), g = grad Phi, D = g.H and
 * x_u, x_v, h_u, h_v as in lss_chart_geometry:
 *   xuu (N,3) = 2 h_u H_u + h_uu H,  h_uu = -(x_u.B x_u + 2 h_u g.H_u)/D;
 *   xuv (N,3) = h_u H_v + h_v H_u + h_uv H,
 *               h_uv = -(x_u.B x_v + g.(h_u H_v + h_v H_u))/D;
 *   xvv (N,3) = 2 h_v H_v + h_vv H,  h_vv = -(x_v.B x_v + 2 h_v g.H_v)/D;
 *   gauss (N) = (LN - M^2)/(EG - F^2), mean (N) = -(EN - 2FM + GL)/(2(EG - F^2))
 *   (first and second fundamental forms with the outward normal -g/|g|, so
 *   a sphere of radius R has mean curvature 1/R).
 * N = ntris * np.  Any output may be NULL.  The cost is that of
 * lss_eval_hessian (with the context's far-field option) at the N chart points.  Host or device arrays as for
 * lss_project; returns when the outputs are written. */
int lss_chart_curvature(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *h, double *xuu,
                        double *xuv, double *xvv, double *gauss, double *mean, unsigned flags);

/* Interpolation of chart data between the chart nodes (section 3.3: a chart
 * is a polynomial of total degree p on the standard simplex, represented in
 * the orthogonal Koornwinder basis through its values at the p-th order
 * nodes).  chart_uv (np,2) are the nodes, np = (p+1)(p+2)/2, unisolvent for
 * degree p (else LSS_EINVAL); f (ntris*np, ncomp) the data at the nodes of
 * every triangle (index j * np + i, e.g. x or h from lss_project); eval_uv
 * (ne,2) points of the simplex; out (ntris*ne, ncomp) receives the value of
 * every triangle's degree-p interpolant at them (index j * ne + e).  The
 * interpolation matrix (ne x np) is formed on the host in FP64 by LU with
 * partial pivoting; one kernel applies it to all triangles.  Needs sources
 * (LSS_ESTATE otherwise), not sigma.  Host or device arrays as for
 * lss_project; returns when out is written. */
int lss_chart_interp(lss_ctx *ctx, const double *chart_uv, int32_t np, const double *f, int32_t ncomp,
                     const double *eval_uv, int32_t ne, double *out, unsigned flags);

/* Autotuner: choose the tile width and, for LSS_FAR_FMM, the near/far split
 * (leaf shrink over [1, 3], leaf capacity, admissibility K and order p) for
 * the current source set, sigma and precision by timing candidates on the
 * caller's targets: cost = (build time) + eval_weight * (time to evaluate x),
 * each from HIP events on the context stream.  A candidate is accepted only
 * if, on up to 16384 of the targets (spread evenly over x), its Phi and
 * grad Phi agree with the exact discrete sum (the direct FP64 path) to a
 * quarter of the precision's bar (1e-12 FP64, 1e-6 MIXED; maximum error relative to the
 * largest value).  The search first times leaf shrink x capacity (x tile)
 * at the default K and p, then K and p around their defaults at the best
 * leaves.  Pass a spatially compact subset of the real targets and
 * eval_weight = (all targets) / n to keep the local target density.
 * cache_path (may be NULL): a text file of one JSON object per line keyed by
 * device, sizes and precision; a matching line is reused without timing, a
 * new result is appended.  On return the best options are set on ctx and
 * written to *out (may be NULL).  x: (n,3), host or device per flags; n >= 1. */
int lss_autotune(lss_ctx *ctx, const double *x, int64_t n, unsigned flags, double eval_weight,
                 const char *cache_path, lss_options *out);

/* Counters of the context.  Waits for the events and counters of the last
 * lss_eval / lss_project (so it synchronises with those calls). */
int lss_get_stats(const lss_ctx *ctx, lss_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* LSS_H */
