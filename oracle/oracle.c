/*
 * Reference oracle for the smoothed-indicator level set (TEST INFRASTRUCTURE).
 *
 * This file is a plain, slow, FP64 CPU implementation of what the GPU path
 * computes.  It exists only to check that path: the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load it; the product library never
 * does.  It shares no code, header, table or constant with the GPU sources.
 *
 * What it computes (paper: Vico, Greengard, O'Neil, Rachh, "A fast boundary
 * integral method for high-order multiscale mesh generation"):
 *
 *  - quadrature nodes on each flat skeleton triangle (eq. tparam; discrete
 *    sum eq. discrete_int):  y = P1 + u (P2-P1) + v (P3-P1), with the
 *    area-weighted outward normal  J = (P2-P1) x (P3-P1)  so that
 *    N_hat da = J du dv;
 *  - on a quadratic (second-order curvilinear) skeleton triangle (section
 *    on quadratic skeletons) given by six points, the corners P1, P2, P3 and
 *    the edge points P4 (edge P1P2), P5 (P2P3), P6 (P3P1):
 *    y = sum_k N_k(u, v) P_k with the quadratic Lagrange shape functions of
 *    the six points, and J = y_u x y_v at the node (the paper names the
 *    element but not its node order or shape functions: these are the
 *    standard ones);
 *  - the level-set function as the direct discrete sum (eq. surf, kerpsi,
 *    discrete_int)  Phi(x) = sum_nodes w psi_sigma(x, y)  with
 *        psi da = -(J . d) K(rho) w du dv,   d = x - y,  rho = |d|,
 *        K(rho) = erf(u)/(4 pi rho^3) - sqrt(2/pi) exp(-u^2)/(4 pi sigma rho^2),
 *        u = rho / (sqrt(2) sigma);
 *    sigma is the width attached to the source triangle (constant or one per
 *    triangle);  for u < 1 the difference of the two singular terms is
 *    replaced by its Taylor series (section 4.4, eq. kerpsi_asymp), summed
 *    to 1e-18 relative instead of the printed five terms;
 *  - the gradient as the exact x-derivative of the same sum:
 *        grad psi da = [ -J K(rho) - (J . d) F(rho) d ] w du dv,
 *        F(rho) = K'(rho) / rho
 *    where F is the function the paper prints after eq. gradPhi.  (The paper's
 *    eq. gradPhi carries the opposite sign on its second term, and its small-u
 *    gradient series eq. kerpsi_asymp2 omits the (N.d) d term; the exact
 *    derivative is used here, and F also gets its own series for u < 1.)
 *    No cut-off and no far-field approximation: every pair uses the full
 *    kernel, accumulated with Neumaier compensation;
 *  - the Hessian of the same sum (for the charts' second derivatives,
 *    section 3.1 eq. uu_vector_aux1/aux2), with the third radial function
 *    G = F'(rho)/rho:
 *        grad grad psi da = [ -F (J d^T + d J^T) - (J.d) F I - (J.d) G d d^T ] w;
 *  - the paper's target-attached width (section 2, eq. basemodelk,
 *    convkernel, sigma2): sigma(x) = sum_j sigma_j w_j / sum_j w_j over the
 *    triangle centroids c_j, w_j = exp(-|x - c_j|^2 / (2 sigma0^2)),
 *    sigma_j = D_j / lambda (D_j the diameter of the smallest enclosing
 *    ball), and Phi, grad Phi with K(rho; sigma(x)) plus the chain-rule term
 *    (dPhi/dsigma) grad sigma;
 *  - vertex pseudonormals (eq. mkvertexpn) and the linear pseudonormal field
 *    on each triangle (eq. mkpseudovec);
 *  - the chart projection: for chart node (u_i, v_i) of triangle j, the root
 *    h of Phi(T + h H) = 1/2 (eq. newton) by Newton's iteration (eq. newtoneq,
 *    derivative eq. newtonderiv) from h = 0, safeguarded by bisection inside
 *    the bracket [lo, hi] the iterates establish, starting from
 *    [-hmax, hmax] with hmax = 16 sigma_j / |H| (Phi decreases along H near
 *    the level set, so g > 0 raises lo and g < 0 lowers hi; a Newton step that
 *    leaves (lo, hi) or has H.grad Phi >= 0 is replaced by the midpoint).
 *    Stop when |dh| <= tau sigma_j.  The safeguard, the scale-free stopping
 *    test and the status codes are additions to the paper's plain iteration.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 * (no -ffast-math: the order of floating-point operations is as written).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_NOBRACKET = 2, ST_DEGENERATE_H = 3 };

/* ------------------------------------------------------------------ sums */
typedef struct { double s, c; } nsum;           /* Neumaier compensated sum */

static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------ radial functions */
/* K(rho) and F(rho) = K'(rho)/rho for width sigma (see header). */
static void radial_KF(double rho, double sigma, double *K, double *F)
{
    const double u = rho / (sqrt(2.0) * sigma);
    if (u < 1.0) {
        /* K = [sum_n 2 (-1)^n u^2n / (n! (2n+3))] / (4 sqrt(2 pi^3) sigma^3)
         * F = -[sum_m 2 (-1)^m u^2m / (m! (2m+5))] / (4 sqrt(2 pi^3) sigma^5) */
        const double u2 = u * u;
        double p = 1.0;              /* (-1)^n u^2n / n! */
        double sk = 0.0, sf = 0.0;
        for (int n = 0; n < 40; ++n) {
            double tk = 2.0 * p / (2.0 * n + 3.0);
            double tf = 2.0 * p / (2.0 * n + 5.0);
            sk += tk;
            sf += tf;
            if (fabs(tk) < 1e-18 * fabs(sk) && fabs(tf) < 1e-18 * fabs(sf)) break;
            p *= -u2 / (double)(n + 1);
        }
        const double c = 1.0 / (4.0 * sqrt(2.0 * ORC_PI * ORC_PI * ORC_PI) * sigma * sigma * sigma);
        *K = c * sk;
        *F = -c * sf / (sigma * sigma);
    } else {
        const double e = exp(-u * u);
        const double er = erf(u);
        const double r2 = rho * rho, r3 = r2 * rho, r5 = r3 * r2;
        const double s2 = sigma * sigma, s3 = s2 * sigma;
        *K = er / (4.0 * ORC_PI * r3) - sqrt(2.0 / ORC_PI) * e / (4.0 * ORC_PI * sigma * r2);
        /* F as printed after eq. gradPhi */
        *F = (e * sqrt(2.0) * (r3 + 3.0 * rho * s2) - 3.0 * sqrt(ORC_PI) * s3 * er)
             / (4.0 * pow(ORC_PI, 1.5) * r5 * s3);
    }
}

/* G(rho) = F'(rho)/rho, the third radial function of the Hessian.  With
 * K = P(3/2, u^2)/(4 pi rho^3) (P the regularised lower incomplete gamma
 * function), d/drho [P(s, u^2)/rho^(2s)] = -2s P(s+1, u^2)/rho^(2s+1), so
 * F = -3 P(5/2, u^2)/(4 pi rho^5) and G = 15 P(7/2, u^2)/(4 pi rho^7), where
 * P(s+1, t) = P(s, t) - t^s e^-t / Gamma(s+1) takes P(3/2, t) = erf(u) -
 * 2 u e^-t / sqrt(pi) up to s = 7/2.  For u < 1.5 the same function by the
 * term-wise derivative of the F series:
 *   G = [sum_k 2 (-1)^k u^2k / (k! (2k+7))] / (4 sqrt(2 pi^3) sigma^7). */
static double radial_G(double rho, double sigma)
{
    const double u = rho / (sqrt(2.0) * sigma);
    if (u < 1.5) {
        const double u2 = u * u;
        double p = 1.0, s = 0.0;
        for (int k = 0; k < 60; ++k) {
            const double t = 2.0 * p / (2.0 * k + 7.0);
            s += t;
            if (fabs(t) < 1e-18 * fabs(s)) break;
            p *= -u2 / (double)(k + 1);
        }
        return s / (4.0 * sqrt(2.0 * ORC_PI * ORC_PI * ORC_PI) * pow(sigma, 7.0));
    }
    const double t = u * u, e = exp(-t);
    const double P32 = erf(u) - 2.0 * u * e / sqrt(ORC_PI);
    const double P52 = P32 - pow(t, 1.5) * e / (0.75 * sqrt(ORC_PI));          /* Gamma(5/2) */
    const double P72 = P52 - pow(t, 2.5) * e / (1.875 * sqrt(ORC_PI));         /* Gamma(7/2) */
    return 15.0 * P72 / (4.0 * ORC_PI * pow(rho, 7.0));
}

/* exported for the kernel-function checks: K, F at rho for one sigma */
void oracle_radial(const double *rho, int64_t n, double sigma, double *K, double *F)
{
    for (int64_t i = 0; i < n; ++i) radial_KF(rho[i], sigma, &K[i], &F[i]);
}

void oracle_radial_G(const double *rho, int64_t n, double sigma, double *G)
{
    for (int64_t i = 0; i < n; ++i) G[i] = radial_G(rho[i], sigma);
}

/* --------------------------------------------------------- quadrature nodes */
static void tri_node(const double *verts, const int32_t *tri, const double *uvw,
                     double y[3], double a[3])
{
    const double *P1 = verts + 3 * (int64_t)tri[0];
    const double *P2 = verts + 3 * (int64_t)tri[1];
    const double *P3 = verts + 3 * (int64_t)tri[2];
    double tu[3], tv[3];
    for (int c = 0; c < 3; ++c) {
        tu[c] = P2[c] - P1[c];
        tv[c] = P3[c] - P1[c];
        y[c] = P1[c] + uvw[0] * tu[c] + uvw[1] * tv[c];
    }
    a[0] = uvw[2] * (tu[1] * tv[2] - tu[2] * tv[1]);
    a[1] = uvw[2] * (tu[2] * tv[0] - tu[0] * tv[2]);
    a[2] = uvw[2] * (tu[0] * tv[1] - tu[1] * tv[0]);
}

/* Quadratic triangle: barycentrics l1 = 1-u-v, l2 = u, l3 = v;
 *   N1 = l1(2 l1 - 1), N2 = l2(2 l2 - 1), N3 = l3(2 l3 - 1),
 *   N4 = 4 l1 l2,      N5 = 4 l2 l3,      N6 = 4 l3 l1,
 * derivatives by the chain rule with dl/du = (-1, 1, 0), dl/dv = (-1, 0, 1). */
static void quad_node(const double *verts, const int32_t *tri, const double *uvw,
                      double y[3], double a[3])
{
    const double u = uvw[0], v = uvw[1];
    const double l1 = 1.0 - u - v, l2 = u, l3 = v;
    const double N[6] = {l1 * (2.0 * l1 - 1.0), l2 * (2.0 * l2 - 1.0), l3 * (2.0 * l3 - 1.0),
                         4.0 * l1 * l2, 4.0 * l2 * l3, 4.0 * l3 * l1};
    const double Nu[6] = {-(4.0 * l1 - 1.0), 4.0 * l2 - 1.0, 0.0,
                          4.0 * (l1 - l2), 4.0 * l3, -4.0 * l3};
    const double Nv[6] = {-(4.0 * l1 - 1.0), 0.0, 4.0 * l3 - 1.0,
                          -4.0 * l2, 4.0 * l2, 4.0 * (l1 - l3)};
    double yu[3] = {0, 0, 0}, yv[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) y[c] = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double *P = verts + 3 * (int64_t)tri[k];
        for (int c = 0; c < 3; ++c) {
            y[c] += N[k] * P[c];
            yu[c] += Nu[k] * P[c];
            yv[c] += Nv[k] * P[c];
        }
    }
    a[0] = uvw[2] * (yu[1] * yv[2] - yu[2] * yv[1]);
    a[1] = uvw[2] * (yu[2] * yv[0] - yu[0] * yv[2]);
    a[2] = uvw[2] * (yu[0] * yv[1] - yu[1] * yv[0]);
}

/* node m of triangle j; nvt = 3 (flat) or 6 (quadratic) indices per triangle */
static void src_node(const double *verts, const int32_t *tris, int32_t nvt, int64_t j,
                     const double *uvw, double y[3], double a[3])
{
    if (nvt == 6) quad_node(verts, tris + 6 * j, uvw, y, a);
    else tri_node(verts, tris + 3 * j, uvw, y, a);
}

/* all nodes y and weighted normals a = w J, node index = tri * nq + m */
void oracle_nodes(const double *verts, const int32_t *tris, int32_t nvt, int64_t ntris,
                  const double *rule, int32_t nq, double *y, double *a)
{
    for (int64_t j = 0; j < ntris; ++j)
        for (int m = 0; m < nq; ++m)
            src_node(verts, tris, nvt, j, rule + 3 * m, y + 3 * (j * nq + m), a + 3 * (j * nq + m));
}

/* ------------------------------------------------------------ evaluation */
typedef struct {
    const double *verts;
    const int32_t *tris;
    int32_t nvt;              /* indices per triangle: 3 flat, 6 quadratic */
    const int64_t *tri_off;   /* nmesh+1 or NULL */
    int64_t ntris;
    const double *sigma;      /* length 1 or ntris */
    int64_t nsigma;
    const double *rule;
    int32_t nq;
} srcset;

static void eval_point(const srcset *S, const double x[3], int32_t mesh,
                       double *phi, double grad[3], double *aphi, double *agrad)
{
    int64_t j0 = 0, j1 = S->ntris;
    if (S->tri_off) { j0 = S->tri_off[mesh]; j1 = S->tri_off[mesh + 1]; }
    nsum sp = {0, 0}, sg[3] = {{0, 0}, {0, 0}, {0, 0}}, ap = {0, 0}, ag = {0, 0};
    for (int64_t j = j0; j < j1; ++j) {
        const double sigma = S->nsigma == 1 ? S->sigma[0] : S->sigma[j];
        for (int m = 0; m < S->nq; ++m) {
            double y[3], a[3], d[3];
            src_node(S->verts, S->tris, S->nvt, j, S->rule + 3 * m, y, a);
            d[0] = x[0] - y[0]; d[1] = x[1] - y[1]; d[2] = x[2] - y[2];
            const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double K, F;
            radial_KF(rho, sigma, &K, &F);
            const double ad = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
            const double tphi = -ad * K;
            double tg[3];
            for (int c = 0; c < 3; ++c) tg[c] = -a[c] * K - ad * F * d[c];
            nsum_add(&sp, tphi);
            for (int c = 0; c < 3; ++c) nsum_add(&sg[c], tg[c]);
            nsum_add(&ap, fabs(tphi));
            nsum_add(&ag, sqrt(tg[0] * tg[0] + tg[1] * tg[1] + tg[2] * tg[2]));
        }
    }
    *phi = nsum_get(&sp);
    for (int c = 0; c < 3; ++c) grad[c] = nsum_get(&sg[c]);
    if (aphi) *aphi = nsum_get(&ap);
    if (agrad) *agrad = nsum_get(&ag);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Phi and grad Phi at n targets.  x_mesh (may be NULL) selects, per target,
 * the mesh (CSR range of tri_off) whose triangles are summed. aphi / agrad
 * (may be NULL) receive sum |term| and sum ||grad term||. */
void oracle_eval(const double *verts, const int32_t *tris, int32_t nvt, int64_t ntris,
                 const int64_t *tri_off, const double *sigma, int64_t nsigma,
                 const double *rule, int32_t nq,
                 const double *x, const int32_t *x_mesh, int64_t n,
                 double *phi, double *grad, double *aphi, double *agrad, int nthreads)
{
    srcset S = {verts, tris, nvt, tri_off, ntris, sigma, nsigma, rule, nq};
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i)
        eval_point(&S, x + 3 * i, x_mesh ? x_mesh[i] : 0, &phi[i], grad + 3 * i,
                   aphi ? &aphi[i] : NULL, agrad ? &agrad[i] : NULL);
}

/* Hessian of Phi at n targets (the second x-derivative of the same discrete
 * sum, needed for the second derivatives of the charts, section 3.1 eq.
 * uu_vector_aux1/aux2).  Per node, with a = w J, d = x - y:
 *   d2 psi / dx_i dx_j = -F (a_i d_j + a_j d_i) - (a.d) F delta_ij - (a.d) G d_i d_j.
 * Output hess (n, 6): xx, xy, xz, yy, yz, zz.  Full kernel for every pair. */
void oracle_hessian(const double *verts, const int32_t *tris, int32_t nvt, int64_t ntris,
                    const int64_t *tri_off, const double *sigma, int64_t nsigma,
                    const double *rule, int32_t nq,
                    const double *x, const int32_t *x_mesh, int64_t n, double *hess, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t mesh = x_mesh ? x_mesh[i] : 0;
        int64_t j0 = 0, j1 = ntris;
        if (tri_off) { j0 = tri_off[mesh]; j1 = tri_off[mesh + 1]; }
        nsum S[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) S[r][c].s = S[r][c].c = 0.0;
        for (int64_t j = j0; j < j1; ++j) {
            const double sg = nsigma == 1 ? sigma[0] : sigma[j];
            for (int m = 0; m < nq; ++m) {
                double y[3], a[3], d[3];
                src_node(verts, tris, nvt, j, rule + 3 * m, y, a);
                for (int c = 0; c < 3; ++c) d[c] = x[3 * i + c] - y[c];
                const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double K, F;
                radial_KF(rho, sg, &K, &F);
                const double G = radial_G(rho, sg);
                const double ad = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
                for (int r = 0; r < 3; ++r)
                    for (int c = r; c < 3; ++c)
                        nsum_add(&S[r][c], -F * (a[r] * d[c] + a[c] * d[r]) - (r == c ? ad * F : 0.0)
                                               - ad * G * d[r] * d[c]);
            }
        }
        double *o = hess + 6 * i;
        o[0] = nsum_get(&S[0][0]); o[1] = nsum_get(&S[0][1]); o[2] = nsum_get(&S[0][2]);
        o[3] = nsum_get(&S[1][1]); o[4] = nsum_get(&S[1][2]); o[5] = nsum_get(&S[2][2]);
    }
}

/* ------------------------------------------- multiscale sigma(x) (section 2) */
/* D_j: diameter of the smallest ball enclosing the triangle: the longest
 * edge when the triangle is right or obtuse (the ball on that edge holds the
 * third vertex), else twice the circumradius abc / (4 area). */
static double tri_diameter(const double *A, const double *B, const double *C)
{
    double a2 = 0, b2 = 0, c2 = 0, e1[3], e2[3], cr[3];
    for (int k = 0; k < 3; ++k) {
        a2 += (B[k] - C[k]) * (B[k] - C[k]);
        b2 += (C[k] - A[k]) * (C[k] - A[k]);
        c2 += (A[k] - B[k]) * (A[k] - B[k]);
        e1[k] = B[k] - A[k];
        e2[k] = C[k] - A[k];
    }
    double m = a2 > b2 ? a2 : b2;
    m = m > c2 ? m : c2;
    if (2.0 * m >= a2 + b2 + c2) return sqrt(m);          /* largest angle >= 90 degrees */
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double area2 = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);   /* twice the area */
    return sqrt(a2 * b2 * c2) / area2;                    /* 2 R = abc / (2 area) */
}

/* Centroids c_j and D_j of triangles j0..j1-1 (corners P1 P2 P3). */
static void tri_centroids(const double *verts, const int32_t *tris, int32_t nvt, int64_t j0, int64_t j1,
                          double *cen, double *D)
{
    for (int64_t j = j0; j < j1; ++j) {
        const int32_t *t = tris + nvt * j;
        const double *A = verts + 3 * (int64_t)t[0], *B = verts + 3 * (int64_t)t[1], *C = verts + 3 * (int64_t)t[2];
        for (int k = 0; k < 3; ++k) cen[3 * j + k] = (A[k] + B[k] + C[k]) / 3.0;
        D[j] = tri_diameter(A, B, C);
    }
}

/* sigma(x) of eq. sigma2 and its gradient
 *   grad sigma = -sum_j (sigma_j - sigma) w_j (x - c_j) / (sigma0^2 sum_j w_j),
 * w_j = exp(-|x - c_j|^2 / (2 sigma0^2)), all weights taken relative to the
 * largest one (the nearest centroid) so that none underflows to 0/0. */
static void sigma_blend(const double *cen, const double *sj, int64_t j0, int64_t j1, double s0,
                        const double x[3], double *sig, double g[3])
{
    double dmin = INFINITY;
    for (int64_t j = j0; j < j1; ++j) {
        const double dx = x[0] - cen[3 * j], dy = x[1] - cen[3 * j + 1], dz = x[2] - cen[3 * j + 2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < dmin) dmin = d2;
    }
    nsum num = {0, 0}, den = {0, 0};
    for (int64_t j = j0; j < j1; ++j) {
        const double dx = x[0] - cen[3 * j], dy = x[1] - cen[3 * j + 1], dz = x[2] - cen[3 * j + 2];
        const double w = exp(-(dx * dx + dy * dy + dz * dz - dmin) / (2.0 * s0 * s0));
        nsum_add(&num, sj[j] * w);
        nsum_add(&den, w);
    }
    const double s = nsum_get(&num) / nsum_get(&den);
    nsum gs[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t j = j0; j < j1; ++j) {
        const double d[3] = {x[0] - cen[3 * j], x[1] - cen[3 * j + 1], x[2] - cen[3 * j + 2]};
        const double w = exp(-(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - dmin) / (2.0 * s0 * s0));
        for (int k = 0; k < 3; ++k) nsum_add(&gs[k], -(sj[j] - s) * w * d[k]);
    }
    *sig = s;
    for (int k = 0; k < 3; ++k) g[k] = nsum_get(&gs[k]) / (s0 * s0 * nsum_get(&den));
}

/* sigma(x) (n), grad sigma (n,3), sigma_j (ntris) and the sigma0 used per
 * mesh, from the triangles' centroids and diameters: sigma_j = D_j / lambda,
 * sigma0 as given, or sqrt(5) max_j D_j over the target's mesh when
 * sigma0 <= 0. */
void oracle_sigma_field(const double *verts, const int32_t *tris, int32_t nvt, int64_t ntris,
                        const int64_t *tri_off, int32_t nmesh, double lambda, double sigma0,
                        const double *x, const int32_t *x_mesh, int64_t n, double *sig, double *gsig,
                        double *sj_out, double *s0_out)
{
    const int32_t nm = tri_off ? nmesh : 1;
    double *cen = (double *)malloc(sizeof(double) * 3 * (size_t)ntris);
    double *D = (double *)malloc(sizeof(double) * (size_t)ntris);
    tri_centroids(verts, tris, nvt, 0, ntris, cen, D);
    for (int64_t j = 0; j < ntris; ++j) sj_out[j] = D[j] / lambda;
    for (int32_t m = 0; m < nm; ++m) {
        const int64_t j0 = tri_off ? tri_off[m] : 0, j1 = tri_off ? tri_off[m + 1] : ntris;
        double dmax = 0.0;
        for (int64_t j = j0; j < j1; ++j) dmax = D[j] > dmax ? D[j] : dmax;
        s0_out[m] = sigma0 > 0.0 ? sigma0 : sqrt(5.0) * dmax;
    }
    for (int64_t i = 0; i < n; ++i) {
        const int32_t m = x_mesh ? x_mesh[i] : 0;
        const int64_t j0 = tri_off ? tri_off[m] : 0, j1 = tri_off ? tri_off[m + 1] : ntris;
        sigma_blend(cen, sj_out, j0, j1, s0_out[m], x + 3 * i, &sig[i], gsig + 3 * i);
    }
    free(cen);
    free(D);
}

/* Phi and grad Phi with the target-attached width sigma(x) of eq. basemodelk,
 * convkernel and sigma2: every node of the target's mesh with K(rho; sigma(x))
 * and F(rho; sigma(x)), and the chain-rule term (dPhi/dsigma) grad sigma with
 *   dK/dsigma = -exp(-rho^2 / (2 sigma^2)) / (2 sqrt(2) pi^1.5 sigma^4),
 *   dPhi/dsigma = sum (a.d) exp(-rho^2 / (2 sigma^2)) / (2 sqrt(2) pi^1.5 sigma^4).
 * (The printed eq. gradPhi has the opposite sign on this term, as on its
 * second one; the exact derivative is used.)  sig / gsig from
 * oracle_sigma_field. */
void oracle_eval_multiscale(const double *verts, const int32_t *tris, int32_t nvt, int64_t ntris,
                            const int64_t *tri_off, const double *rule, int32_t nq,
                            const double *x, const int32_t *x_mesh, int64_t n,
                            const double *sig, const double *gsig, double *phi, double *grad, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t mesh = x_mesh ? x_mesh[i] : 0;
        int64_t j0 = 0, j1 = ntris;
        if (tri_off) { j0 = tri_off[mesh]; j1 = tri_off[mesh + 1]; }
        if (j0 == j1) {             /* no triangles: an empty sum */
            phi[i] = 0.0;
            for (int c = 0; c < 3; ++c) grad[3 * i + c] = 0.0;
            continue;
        }
        const double s = sig[i];
        const double cs = 1.0 / (2.0 * sqrt(2.0) * pow(ORC_PI, 1.5) * s * s * s * s);
        nsum sp = {0, 0}, sg[3] = {{0, 0}, {0, 0}, {0, 0}}, ss = {0, 0};
        for (int64_t j = j0; j < j1; ++j)
            for (int m = 0; m < nq; ++m) {
                double y[3], a[3], d[3];
                src_node(verts, tris, nvt, j, rule + 3 * m, y, a);
                for (int c = 0; c < 3; ++c) d[c] = x[3 * i + c] - y[c];
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                double K, F;
                radial_KF(sqrt(r2), s, &K, &F);
                const double ad = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
                nsum_add(&sp, -ad * K);
                for (int c = 0; c < 3; ++c) nsum_add(&sg[c], -a[c] * K - ad * F * d[c]);
                nsum_add(&ss, ad * exp(-r2 / (2.0 * s * s)) * cs);
            }
        phi[i] = nsum_get(&sp);
        const double dps = nsum_get(&ss);
        for (int c = 0; c < 3; ++c) grad[3 * i + c] = nsum_get(&sg[c]) + dps * gsig[3 * i + c];
    }
}

/* ----------------------------------------------------------- pseudonormals */
/* H(P) = sum_T theta_P(T) N_hat(T) / sum_T theta_P(T)  (eq. mkvertexpn). */
void oracle_pseudonormals(const double *verts, int64_t nverts, const int32_t *tris,
                          int64_t ntris, double *H)
{
    double *A = (double *)calloc((size_t)nverts, sizeof(double));
    for (int64_t i = 0; i < 3 * nverts; ++i) H[i] = 0.0;
    for (int64_t j = 0; j < ntris; ++j) {
        const int32_t *t = tris + 3 * j;
        const double *P[3] = {verts + 3 * (int64_t)t[0], verts + 3 * (int64_t)t[1], verts + 3 * (int64_t)t[2]};
        double e1[3], e2[3], N[3];
        for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
        N[0] = e1[1] * e2[2] - e1[2] * e2[1];
        N[1] = e1[2] * e2[0] - e1[0] * e2[2];
        N[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (nn == 0.0) continue;
        for (int k = 0; k < 3; ++k) {
            const double *A0 = P[k], *A1 = P[(k + 1) % 3], *A2 = P[(k + 2) % 3];
            double p[3], q[3], cr[3];
            for (int c = 0; c < 3; ++c) { p[c] = A1[c] - A0[c]; q[c] = A2[c] - A0[c]; }
            cr[0] = p[1] * q[2] - p[2] * q[1];
            cr[1] = p[2] * q[0] - p[0] * q[2];
            cr[2] = p[0] * q[1] - p[1] * q[0];
            const double theta = atan2(sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]),
                                       p[0] * q[0] + p[1] * q[1] + p[2] * q[2]);
            const int64_t v = t[k];
            for (int c = 0; c < 3; ++c) H[3 * v + c] += theta * N[c] / nn;
            A[v] += theta;
        }
    }
    for (int64_t v = 0; v < nverts; ++v)
        if (A[v] > 0.0)
            for (int c = 0; c < 3; ++c) H[3 * v + c] /= A[v];
    free(A);
}

/* Curved chart bases on quadratic skeleton triangles (the section on
 * quadratic skeletons: the pseudonormal construction carries over to the
 * curved triangles).  The quadratic Lagrange shape functions of the six
 * points (corners P1 P2 P3, edge points P4 on P1P2, P5 on P2P3, P6 on P3P1),
 * w = 1 - u - v:
 *   N1 = w (2w - 1), N2 = u (2u - 1), N3 = v (2v - 1), N4 = 4uw, N5 = 4uv, N6 = 4vw,
 * and their derivatives in u and v. */
static void quad_shape(double u, double v, double N[6], double Nu[6], double Nv[6])
{
    const double w = 1.0 - u - v;
    N[0] = w * (2.0 * w - 1.0); N[1] = u * (2.0 * u - 1.0); N[2] = v * (2.0 * v - 1.0);
    N[3] = 4.0 * u * w;         N[4] = 4.0 * u * v;         N[5] = 4.0 * v * w;
    Nu[0] = 1.0 - 4.0 * w; Nu[1] = 4.0 * u - 1.0; Nu[2] = 0.0;
    Nu[3] = 4.0 * (w - u); Nu[4] = 4.0 * v;       Nu[5] = -4.0 * v;
    Nv[0] = 1.0 - 4.0 * w; Nv[1] = 0.0;           Nv[2] = 4.0 * v - 1.0;
    Nv[3] = -4.0 * u;      Nv[4] = 4.0 * u;       Nv[5] = 4.0 * (w - v);
}

/* Point and tangents of triangle j's quadratic patch at (u, v). */
static void quad_point(const double *verts, const int32_t *t6, double u, double v, double y[3], double yu[3],
                       double yv[3])
{
    double N[6], Nu[6], Nv[6];
    quad_shape(u, v, N, Nu, Nv);
    for (int c = 0; c < 3; ++c) {
        y[c] = yu[c] = yv[c] = 0.0;
        for (int k = 0; k < 6; ++k) {
            const double P = verts[3 * (int64_t)t6[k] + c];
            y[c] += N[k] * P;
            yu[c] += Nu[k] * P;
            yv[c] += Nv[k] * P;
        }
    }
}

/* Vertex pseudonormals of a quadratic skeleton (eq. mkvertexpn on the curved
 * triangles): at each corner of each patch, the unit patch normal y_u x y_v
 * weighted by the angle between the patch's two edges there (their tangent
 * directions at the corner, from the edge directions (1,0), (0,1), (-1,1) of
 * T0), summed over the corners of the vertex and divided by the summed
 * angles, not renormalised. */
void oracle_pseudonormals_curved(const double *verts, int64_t nverts, const int32_t *tris6, int64_t ntris, double *H)
{
    static const double cuv[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    /* edge directions in (u, v) leaving each corner */
    static const double dir[3][2][2] = {{{1, 0}, {0, 1}}, {{-1, 1}, {-1, 0}}, {{0, -1}, {1, -1}}};
    double *A = (double *)calloc((size_t)nverts, sizeof(double));
    for (int64_t i = 0; i < 3 * nverts; ++i) H[i] = 0.0;
    for (int64_t j = 0; j < ntris; ++j) {
        const int32_t *t6 = tris6 + 6 * j;
        for (int k = 0; k < 3; ++k) {
            double y[3], yu[3], yv[3], N[3], p[3], q[3], cr[3];
            quad_point(verts, t6, cuv[k][0], cuv[k][1], y, yu, yv);
            N[0] = yu[1] * yv[2] - yu[2] * yv[1];
            N[1] = yu[2] * yv[0] - yu[0] * yv[2];
            N[2] = yu[0] * yv[1] - yu[1] * yv[0];
            const double nn = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            if (nn == 0.0) continue;
            for (int c = 0; c < 3; ++c) {
                p[c] = dir[k][0][0] * yu[c] + dir[k][0][1] * yv[c];
                q[c] = dir[k][1][0] * yu[c] + dir[k][1][1] * yv[c];
            }
            cr[0] = p[1] * q[2] - p[2] * q[1];
            cr[1] = p[2] * q[0] - p[0] * q[2];
            cr[2] = p[0] * q[1] - p[1] * q[0];
            const double theta = atan2(sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]),
                                       p[0] * q[0] + p[1] * q[1] + p[2] * q[2]);
            const int64_t v = t6[k];
            for (int c = 0; c < 3; ++c) H[3 * v + c] += theta * N[c] / nn;
            A[v] += theta;
        }
    }
    for (int64_t v = 0; v < nverts; ++v)
        if (A[v] > 0.0)
            for (int c = 0; c < 3; ++c) H[3 * v + c] /= A[v];
    free(A);
}

/* ---------------------------------------------------------- Newton projection */
/* For each selected triangle j (sel[k], or k if sel is NULL) and each chart
 * node (u_i, v_i): T, H from eq. tparam / mkpseudovec, then the safeguarded
 * Newton iteration described in the header.  Output index k * np + i.
 * With quadratic sources (nvt = 6) Phi sums the curved triangles; the chart
 * base T and the pseudonormal field H come from their corner triangles
 * P1 P2 P3, or with `curved` from the patches themselves: T = the quadratic
 * patch at (u, v), H linear in the curved-vertex pseudonormals
 * (oracle_pseudonormals_curved). */
void oracle_project(const double *verts, int64_t nverts, const int32_t *tris, int32_t nvt, int64_t ntris,
                    const int64_t *tri_off, int32_t nmesh,
                    const double *sigma, int64_t nsigma, const double *rule, int32_t nq,
                    const double *chart_uv, int32_t np, const int64_t *sel, int64_t nsel,
                    double tau, int32_t max_iter, int32_t curved,
                    double *h_out, double *x_out, int8_t *status, int8_t *iters,
                    int nthreads)
{
    srcset S = {verts, tris, nvt, tri_off, ntris, sigma, nsigma, rule, nq};
    const int cur = curved && nvt == 6;
    int32_t *corner = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)ntris);
    for (int64_t j = 0; j < ntris; ++j)
        for (int k = 0; k < 3; ++k) corner[3 * j + k] = tris[nvt * j + k];
    double *Hv = (double *)malloc(sizeof(double) * 3 * (size_t)nverts);
    if (cur) oracle_pseudonormals_curved(verts, nverts, tris, ntris, Hv);
    else oracle_pseudonormals(verts, nverts, corner, ntris, Hv);
    set_threads(nthreads);
    const int64_t total = nsel * (int64_t)np;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t idx = 0; idx < total; ++idx) {
        const int64_t k = idx / np;
        const int i = (int)(idx % np);
        const int64_t j = sel ? sel[k] : k;
        int32_t mesh = 0;
        if (tri_off) {           /* mesh holding triangle j */
            int32_t lo = 0, hi = nmesh;
            while (hi - lo > 1) { int32_t mid = (lo + hi) / 2; if (tri_off[mid] <= j) lo = mid; else hi = mid; }
            mesh = lo;
        }
        const double u = chart_uv[2 * i], v = chart_uv[2 * i + 1];
        const int32_t *t = corner + 3 * j;
        double T[3], H[3];
        for (int c = 0; c < 3; ++c) {
            const double p1 = verts[3 * (int64_t)t[0] + c], p2 = verts[3 * (int64_t)t[1] + c], p3 = verts[3 * (int64_t)t[2] + c];
            const double h1 = Hv[3 * (int64_t)t[0] + c], h2 = Hv[3 * (int64_t)t[1] + c], h3 = Hv[3 * (int64_t)t[2] + c];
            T[c] = p1 + u * (p2 - p1) + v * (p3 - p1);
            H[c] = h1 + u * (h2 - h1) + v * (h3 - h1);
        }
        if (cur) {
            double yu[3], yv[3];
            quad_point(verts, tris + 6 * j, u, v, T, yu, yv);
        }
        const double sj = nsigma == 1 ? sigma[0] : sigma[j];
        const double nH = sqrt(H[0] * H[0] + H[1] * H[1] + H[2] * H[2]);
        double h = 0.0;
        int st = ST_MAXITER, it = 0;
        if (!(nH >= 1e-3)) {
            st = ST_DEGENERATE_H;
        } else {
            const double hmax = 16.0 * sj / nH;
            double lo = -hmax, hi = hmax;
            int done = 0, seen = 0;     /* bit 1: g > 0 seen, bit 2: g < 0 seen */
            for (int k2 = 1; k2 <= max_iter; ++k2) {
                double x[3], phi, g[3];
                for (int c = 0; c < 3; ++c) x[c] = T[c] + h * H[c];
                eval_point(&S, x, mesh, &phi, g, NULL, NULL);
                const double gv = phi - 0.5;
                const double gp = H[0] * g[0] + H[1] * g[1] + H[2] * g[2];
                it = k2;
                if (gv > 0.0) { lo = h; seen |= 1; }
                else if (gv < 0.0) { hi = h; seen |= 2; }
                else { st = ST_CONVERGED; done = 1; break; }
                double hn = (gp < 0.0) ? h - gv / gp : NAN;
                const int newton = hn > lo && hn < hi;
                if (!newton) hn = 0.5 * (lo + hi);
                const double dh = hn - h;
                h = hn;
                /* a bisection step into the outer quarter of the search range
                 * without a sign change of g: no root near the skeleton */
                if (!newton && seen != 3 && fabs(h) > 0.75 * hmax) { st = ST_NOBRACKET; done = 1; break; }
                if (fabs(dh) <= tau * sj) { st = ST_CONVERGED; done = 1; break; }
            }
            /* not converged: NOBRACKET when the iterates were driven into the
             * outer half of the search range |h| <= hmax (no root near the
             * skeleton), MAXITER otherwise */
            if (!done) st = (fabs(h) > 0.5 * hmax) ? ST_NOBRACKET : ST_MAXITER;
        }
        h_out[idx] = h;
        for (int c = 0; c < 3; ++c) x_out[3 * idx + c] = T[c] + h * H[c];
        status[idx] = (int8_t)st;
        iters[idx] = (int8_t)it;
    }
    free(Hv);
    free(corner);
}
