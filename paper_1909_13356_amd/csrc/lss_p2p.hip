// Pair kernels of liblss (gfx950): the direct sum of the smoothed-indicator
// kernel over quadrature nodes (section 4.3, eq. discrete_int; kernel
// section 4.1, eq. kerpsi; exact gradient of the discrete sum).
//
// Per pair, with d = x - y, x = |d|^2 s2 (s2 = 1/(2 sigma^2)) and the folded
// dipole vector a' = c(sigma) w J:
//     Phi      -= (a'.d) S(x)
//     grad Phi += 2 s2 (a'.d) T(x) d - a' S(x)
// S(x) = gamma(3/2,x)/x^1.5, T(x) = gamma(5/2,x)/x^2.5 come from the rational
// fits of kfit_tables.h below the cut x = X (8 sigma in FP64, 6.32 sigma in
// FP32) and from the Laplace dipole S = (sqrt(pi)/2) x^-1.5, T = 1.5 S/x
// beyond it (section 4.4: the kernel equals the double-layer kernel there to
// the tail bound of the cut).
//
// Mixed path: the FP64 differences to a tile origin are carried as float-float
// (hi + lo) so that d keeps FP32 relative accuracy at any distance from it.
//
// Layout: one target per lane, TILE targets per workgroup (targets sorted by
// mesh, then Morton order); quadrature nodes are streamed through LDS in
// chunks of TILE packed records; each lane sums the nodes of its own mesh
// (per-lane node range, so a tile may straddle meshes of a ragged batch).
// Chunk partial sums are folded into compensated totals (two-sum).
#include <algorithm>
#include <cstring>
#include <hip/hip_runtime.h>

#include "fmm_math.h"
#include "kfit_tables.h"
#include "lss_internal.h"
#include "radial_exact.h"

namespace lss {

namespace {

constexpr double kSqrtPiHalf = 0.88622692545275801365;
// Staged node records carry the far-form constants: a' times kFoldA and 2 s2
// times kFoldT (SrcF, fold_src), so that the pair kernels work with
// S / (sqrt(pi)/2) and T / (1.5 sqrt(pi)/2); the fits below the cut
// (kfit_tables.h) are generated for these quotients.
constexpr double kFoldA = kSqrtPiHalf, kFoldT = 1.5;

// FP64 node record as staged in LDS: the far-form constants folded in as in
// SrcF (a' times sqrt(pi)/2, 2 s2 times 1.5)
__device__ __forceinline__ Src fold_src(Src f) {
    f.ax *= kFoldA;
    f.ay *= kFoldA;
    f.az *= kFoldA;
    f.s2x2 *= kFoldT;
    return f;
}

// Padding records (chunks are filled to whole node groups): zero dipole
// vector, placed so far away that every target sees them beyond the cut
// (the dipole branch, whose terms underflow to zero), so they neither
// contribute nor pull a node group into the near-branch evaluation.
__device__ __forceinline__ Src pad_src() {
    Src f;
    f.yx = f.yy = f.yz = 1.0e150;
    f.ax = f.ay = f.az = f.s2x2 = 0.0;
    f.s2 = 1.0;
    return f;
}

__device__ __forceinline__ SrcF pad_srcf() {
    SrcF f;
    f.yx = f.yy = f.yz = 1.0e18f;
    f.lx = f.ly = f.lz = 0.0f;
    f.ax = f.ay = f.az = f.s2x2 = 0.0f;
    f.s2 = 1.0f;
    f.pad = 0.0f;
    return f;
}

__device__ __forceinline__ void two_sum(double &s, double &e, double v) {
    double t = s + v;
    double bp = t - s;
    e += (s - (t - bp)) + (v - bp);
    s = t;
}

__device__ __forceinline__ void two_sum_f(float &s, float &e, float v) {
    float t = s + v;
    float bp = t - s;
    e += (s - (t - bp)) + (v - bp);
    s = t;
}

// S / (sqrt(pi)/2) and T / (1.5 sqrt(pi)/2) in FP64, for folded records (fold_src)
__device__ __forceinline__ void kfun64(double x, double &S, double &T) {
    if (x < KF64_X) {
        // power basis with shared powers t^k (t = x / X in [0, 1)): the
        // coefficients are the multiplicands, which the per-pair kernels keep
        // as scalar operands; Horner's addends are hoisted into vector
        // registers there, costing a wave per SIMD.  The coefficients are of
        // one sign but for a few small ones, so the sums stay well conditioned.
        const double t = x * KF64_INV_X;
        double ps = kf64_ps[0], pt = kf64_pt[0], q = kf64_q[0], tk = 1.0;
#pragma unroll
        for (int k = 1; k <= KF64_Q_DEG; ++k) {
            tk *= t;
            ps = fma(kf64_ps[k], tk, ps);
            pt = fma(kf64_pt[k], tk, pt);
            q = fma(kf64_q[k], tk, q);
        }
        double r = __builtin_amdgcn_rcp(q);
        const double er = fma(-q, r, 1.0);      // third-order correction of 1/q
        r = fma(r, fma(er, er, er), r);
        S = ps * r;
        T = pt * r;
    } else {
        const double r = rsq64(x);
        const double r2 = r * r;
        S = r2 * r;
        T = S * r2;
    }
}

// S / (sqrt(pi)/2) and T / (1.5 sqrt(pi)/2) in FP32, for SrcF records
__device__ __forceinline__ void kfun32(float x, float &S, float &T) {
    if (x < (float)KF32_X) {
        const float t = x * (float)KF32_INV_X;
        float ps = kf32_ps[KF32_PS_DEG], pt = kf32_pt[KF32_PT_DEG], q = kf32_q[KF32_Q_DEG];
#pragma unroll
        for (int k = KF32_Q_DEG - 1; k >= 0; --k) {
            ps = fmaf(ps, t, kf32_ps[k]);
            pt = fmaf(pt, t, kf32_pt[k]);
            q = fmaf(q, t, kf32_q[k]);
        }
        const float r = __builtin_amdgcn_rcpf(q);
        S = ps * r;
        T = pt * r;
    } else {
        const float r = __builtin_amdgcn_rsqf(x);
        const float r2 = r * r;
        S = r2 * r;
        T = S * r2;
    }
}

__device__ __forceinline__ void pair64(const Src &s, double x, double y, double z, double &p, double &gx,
                                       double &gy, double &gz) {
    const double dx = x - s.yx, dy = y - s.yy, dz = z - s.yz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ad = fma(s.ax, dx, fma(s.ay, dy, s.az * dz));
    double S, T;
    kfun64(r2 * s.s2, S, T);
    p = fma(-ad, S, p);
    const double g = ad * T * s.s2x2;
    gx = fma(g, dx, fma(-s.ax, S, gx));
    gy = fma(g, dy, fma(-s.ay, S, gy));
    gz = fma(g, dz, fma(-s.az, S, gz));
}

// K consecutive FP64 records against one target (see nodes32 below); with
// COUNT the pairs inside the cut are added to *cnt
template <int K, bool COUNT = false>
__device__ __forceinline__ void nodes64(const Src *sh, double x, double y, double z, double &p, double &gx,
                                        double &gy, double &gz, uint32_t *cnt = nullptr) {
    double dx[K], dy[K], dz[K], u[K], ad[K], S[K], T[K];
    double umin = 1.0e300;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const Src s = sh[k];
        dx[k] = x - s.yx;
        dy[k] = y - s.yy;
        dz[k] = z - s.yz;
        const double r2 = fma(dx[k], dx[k], fma(dy[k], dy[k], dz[k] * dz[k]));
        ad[k] = fma(s.ax, dx[k], fma(s.ay, dy[k], s.az * dz[k]));
        u[k] = r2 * s.s2;
        umin = fmin(umin, u[k]);
        const double ux = fmax(u[k], KF64_X);
        const double r = rsq64(ux);
        const double rr = r * r;
        S[k] = rr * r;                      // folded far form (see fold_src)
        T[k] = S[k] * rr;
    }
    if (umin < KF64_X) {                    // some pair of the group inside the cut
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double t = fmin(u[k], KF64_X) * KF64_INV_X;
            double ps = kf64_ps[KF64_Q_DEG], pt = kf64_pt[KF64_Q_DEG], q = kf64_q[KF64_Q_DEG];
#pragma unroll
            for (int i = KF64_Q_DEG - 1; i >= 0; --i) {
                ps = fma(ps, t, kf64_ps[i]);
                pt = fma(pt, t, kf64_pt[i]);
                q = fma(q, t, kf64_q[i]);
            }
            double r = __builtin_amdgcn_rcp(q);
            const double er = fma(-q, r, 1.0);      // third-order correction of 1/q
            r = fma(r, fma(er, er, er), r);
            const bool nr = u[k] < KF64_X;
            S[k] = nr ? ps * r : S[k];
            T[k] = nr ? pt * r : T[k];
            if (COUNT) *cnt += nr ? 1u : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const Src &s = sh[k];
        p = fma(-ad[k], S[k], p);
        const double g = ad[k] * T[k] * s.s2x2;
        gx = fma(g, dx[k], fma(-s.ax, S[k], gx));
        gy = fma(g, dy[k], fma(-s.ay, S[k], gy));
        gz = fma(g, dz[k], fma(-s.az, S[k], gz));
    }
}

constexpr int kNodeGroup64 = 4;

// FP64 record of a node beyond the cut of every target of a tile: position
// and a'' = (sqrt(pi)/2) a' s2^(-3/2)
struct alignas(16) FarD {
    double yx, yy, yz, ax, ay, az;
};

__device__ __forceinline__ FarD pad_fard() {
    FarD f;
    f.yx = f.yy = f.yz = 1.0e150;
    f.ax = f.ay = f.az = 0.0;
    return f;
}

// number of set bits of a wave mask below this lane
__device__ __forceinline__ int below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// K consecutive FP64 far records against one target: the Laplace dipole with
// the width moved into a'' and the gradient summed in two parts, as
// nodes32_far; 1/sqrt refined to FP64 (rsq64)
template <int K>
__device__ __forceinline__ void nodes64_far(const FarD *sh, double x, double y, double z, double &p, double &gx,
                                            double &gy, double &gz, double &hx, double &hy, double &hz) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const FarD s = sh[k];
        const double dx = x - s.yx, dy = y - s.yy, dz = z - s.yz;
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double r = rsq64(r2);
        const double rr = r * r, S = rr * r;
        const double ad = fma(s.ax, dx, fma(s.ay, dy, s.az * dz));
        p = fma(-ad, S, p);
        const double h = ad * S * rr;
        gx = fma(h, dx, gx);
        gy = fma(h, dy, gy);
        gz = fma(h, dz, gz);
        hx = fma(s.ax, S, hx);
        hy = fma(s.ay, S, hy);
        hz = fma(s.az, S, hz);
    }
}

// One FP64 far record against one target, the gradient accumulated whole
// (four accumulators instead of the seven of nodes64_far):
//   Phi -= (a''.d) S,  grad += 3 (a''.d) S |d|^-2 d - a'' S,  S = |d|^-3
__device__ __forceinline__ void pair_far64(const FarD &s, double x, double y, double z, double &p, double &gx,
                                           double &gy, double &gz) {
    const double dx = x - s.yx, dy = y - s.yy, dz = z - s.yz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double r = rsq64(r2);
    const double rr = r * r, S = rr * r;
    const double ad = fma(s.ax, dx, fma(s.ay, dy, s.az * dz));
    p = fma(-ad, S, p);
    const double h = 3.0 * ad * S * rr;
    gx = fma(h, dx, fma(-s.ax, S, gx));
    gy = fma(h, dy, fma(-s.ay, S, gy));
    gz = fma(h, dz, fma(-s.az, S, gz));
}

constexpr int kNodeGroup = 4;

template <int K, bool COUNT = false>
__device__ __forceinline__ void nodes32(const SrcF *sh, float x, float y, float z, float xl, float yl, float zl,
                                        float &p, float &gx, float &gy, float &gz, uint32_t *cnt = nullptr) {
    float dx[K], dy[K], dz[K], u[K], ad[K], S[K], T[K];
    float umin = 3.0e38f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const SrcF s = sh[k];
        dx[k] = (x - s.yx) + (xl - s.lx);
        dy[k] = (y - s.yy) + (yl - s.ly);
        dz[k] = (z - s.yz) + (zl - s.lz);
        const float r2 = fmaf(dx[k], dx[k], fmaf(dy[k], dy[k], dz[k] * dz[k]));
        ad[k] = fmaf(s.ax, dx[k], fmaf(s.ay, dy[k], s.az * dz[k]));
        u[k] = r2 * s.s2;
        umin = fminf(umin, u[k]);
        const float r = __builtin_amdgcn_rsqf(fmaxf(u[k], (float)KF32_X));
        const float rr = r * r;
        S[k] = rr * r;                      // folded far form (see SrcF)
        T[k] = S[k] * rr;
    }
    if (umin < (float)KF32_X) {             // some pair of the group inside the cut
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float t = fminf(u[k], (float)KF32_X) * (float)KF32_INV_X;
            float ps = kf32_ps[KF32_PS_DEG], pt = kf32_pt[KF32_PT_DEG], q = kf32_q[KF32_Q_DEG];
#pragma unroll
            for (int i = KF32_Q_DEG - 1; i >= 0; --i) {
                ps = fmaf(ps, t, kf32_ps[i]);
                pt = fmaf(pt, t, kf32_pt[i]);
                q = fmaf(q, t, kf32_q[i]);
            }
            const float rq = __builtin_amdgcn_rcpf(q);
            const bool nr = u[k] < (float)KF32_X;
            S[k] = nr ? ps * rq : S[k];
            T[k] = nr ? pt * rq : T[k];
            if (COUNT) *cnt += nr ? 1u : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const SrcF &s = sh[k];
        const float g = ad[k] * T[k] * s.s2x2;
        p = fmaf(-ad[k], S[k], p);
        gx = fmaf(g, dx[k], fmaf(-s.ax, S[k], gx));
        gy = fmaf(g, dy[k], fmaf(-s.ay, S[k], gy));
        gz = fmaf(g, dz[k], fmaf(-s.az, S[k], gz));
    }
}


// One (target, node) pair of a near list with the target's own width (see
// pair_ms), the node record's a' rescaled to a' s2^(-3/2) when staged (the
// caller multiplies the sums by s2x^(3/2) once): inside the cut and the FP64 fit's range the radial functions come
// from the fit (k1 = (sqrt(pi)/2) S, k2 = -(3 sqrt(pi)/2) s2x T) and exp(-t)
// from exp; inside the cut beyond that range from the exact forms (radial3);
// beyond the cut the kernel is the Laplace dipole, as in the far field
// (k1 = (sqrt(pi)/2) t^-3/2, k2 = -(3 sqrt(pi)/2) s2x t^-5/2, exp(-t) below
// the cut's truncation).
__device__ __forceinline__ void pair_ms_cut(const Src &s, double px, double py, double pz, double s2x, double tcut,
                                            MsAcc &A) {
    const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
    const double t = (dx * dx + dy * dy + dz * dz) * s2x;
    double k1, k2, et = 0.0;
    if (t < tcut && t < KF64_X) {
        const double tt = t * KF64_INV_X;
        double ps = kf64_ps[0], pt = kf64_pt[0], q = kf64_q[0], tk = 1.0;     // power basis (see kfun64)
#pragma unroll
        for (int i = 1; i <= KF64_Q_DEG; ++i) {
            tk *= tt;
            ps = fma(kf64_ps[i], tk, ps);
            pt = fma(kf64_pt[i], tk, pt);
            q = fma(kf64_q[i], tk, q);
        }
        double r = __builtin_amdgcn_rcp(q);
        const double er = fma(-q, r, 1.0);      // third-order correction of 1/q
        r = fma(r, fma(er, er, er), r);
        k1 = (0.5 * kSqrtPi) * (ps * r);
        k2 = -(1.5 * kSqrtPi) * s2x * (pt * r);
        et = exp(-t);
    } else if (t < tcut) {
        double k3;
        radial3(t, s2x, k1, k2, k3, et);
    } else {
        const double iu = rsq64(t);
        const double iu3 = iu * iu * iu;
        k1 = (0.5 * kSqrtPi) * iu3;
        k2 = -(1.5 * kSqrtPi) * s2x * iu3 * iu * iu;
    }
    const double ad = s.ax * dx + s.ay * dy + s.az * dz;
    A.f += ad * k1;
    const double adk2 = ad * k2;
    A.gx += s.ax * k1 + adk2 * dx;
    A.gy += s.ay * k1 + adk2 * dy;
    A.gz += s.az * k1 + adk2 * dz;
    A.e += ad * et;
}

// pair_hess for the octree's near lists: inside the cut the three radial
// functions come from one rational fit (kf64h: fit error near FP64 rounding),
// beyond the cut (x >= tcut) they are those of the Laplace double layer, as in
// the far field: k1 = (sqrt(pi)/2) x^-3/2, k2 = -(3 sqrt(pi)/2) s2 x^-5/2,
// k3 = (15 sqrt(pi)/2) s2^2 x^-7/2.
static_assert(KF64H_PS_DEG == KF64H_Q_DEG && KF64H_PT_DEG == KF64H_Q_DEG && KF64H_PU_DEG == KF64H_Q_DEG,
              "pair_hess_cut evaluates the Hessian fit's numerators in one loop");
__device__ __forceinline__ void pair_hess_cut(const Src &s, double px, double py, double pz, double tcut,
                                              HessAcc &A) {
    const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
    const double t = (dx * dx + dy * dy + dz * dz) * s.s2;
    double k1, k2, k3;
    if (t < tcut && t < KF64H_X) {
        // S, T, U from one rational fit (power basis, as kfun64):
        // k1 = S, k2 = -2 s2 T, k3 = 4 s2^2 U
        const double tt = t * KF64H_INV_X;
        double ps = kf64h_ps[0], pt = kf64h_pt[0], pu = kf64h_pu[0], q = kf64h_q[0], tk = 1.0;
#pragma unroll
        for (int i = 1; i <= KF64H_Q_DEG; ++i) {
            tk *= tt;
            ps = fma(kf64h_ps[i], tk, ps);
            pt = fma(kf64h_pt[i], tk, pt);
            pu = fma(kf64h_pu[i], tk, pu);
            q = fma(kf64h_q[i], tk, q);
        }
        double r = __builtin_amdgcn_rcp(q);
        const double er = fma(-q, r, 1.0);      // third-order correction of 1/q
        r = fma(r, fma(er, er, er), r);
        k1 = ps * r;
        k2 = -2.0 * s.s2 * (pt * r);
        k3 = 4.0 * s.s2 * s.s2 * (pu * r);
    } else if (t < tcut) {
        double et;
        radial3(t, s.s2, k1, k2, k3, et);
    } else {
        const double iu = rsq64(t);
        const double iu2 = iu * iu, iu3 = iu2 * iu, iu5 = iu3 * iu2;
        k1 = (0.5 * kSqrtPi) * iu3;
        k2 = -(1.5 * kSqrtPi) * s.s2 * iu5;
        k3 = (7.5 * kSqrtPi) * s.s2 * s.s2 * iu5 * iu2;
    }
    const double ad = s.ax * dx + s.ay * dy + s.az * dz;
    A.f -= ad * k1;
    const double adk2 = ad * k2, adk3 = ad * k3;
    A.gx -= s.ax * k1 + adk2 * dx;
    A.gy -= s.ay * k1 + adk2 * dy;
    A.gz -= s.az * k1 + adk2 * dz;
    const double ex = adk3 * dx, ey = adk3 * dy, ez = adk3 * dz;
    A.hxx -= 2.0 * k2 * s.ax * dx + adk2 + ex * dx;
    A.hyy -= 2.0 * k2 * s.ay * dy + adk2 + ey * dy;
    A.hzz -= 2.0 * k2 * s.az * dz + adk2 + ez * dz;
    A.hxy -= k2 * (s.ax * dy + s.ay * dx) + ex * dy;
    A.hxz -= k2 * (s.ax * dz + s.az * dx) + ex * dz;
    A.hyz -= k2 * (s.ay * dz + s.az * dy) + ey * dz;
}

// One (target, node) pair with the node beyond the cut of every target of the
// tile: pair_hess_cut's far form with the width folded into the record,
// a'' = (sqrt(pi)/2) a' s2^(-3/2) (FarD), S = |d|^-3, q = 3 S |d|^-2:
//   Phi -= (a''.d) S,  grad -= a'' S - q (a''.d) d,
//   Hess += q (a'' d^T + d a''^T) + q (a''.d) I - 5 q (a''.d) |d|^-2 d d^T
__device__ __forceinline__ void pair_hess_far(const FarD &s, double px, double py, double pz, HessAcc &A) {
    const double dx = px - s.yx, dy = py - s.yy, dz = pz - s.yz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ir = rsq64(r2);
    const double ir2 = ir * ir, S = ir2 * ir;
    const double ad = fma(s.ax, dx, fma(s.ay, dy, s.az * dz));
    A.f = fma(-ad, S, A.f);
    const double q = 3.0 * S * ir2;
    const double h = q * ad;
    A.gx = fma(h, dx, fma(-s.ax, S, A.gx));
    A.gy = fma(h, dy, fma(-s.ay, S, A.gy));
    A.gz = fma(h, dz, fma(-s.az, S, A.gz));
    const double e = 5.0 * h * ir2;
    const double ux = q * s.ax, uy = q * s.ay, uz = q * s.az;
    const double vx = e * dx, vy = e * dy, vz = e * dz;
    A.hxx = fma(fma(2.0, ux, -vx), dx, A.hxx + h);
    A.hyy = fma(fma(2.0, uy, -vy), dy, A.hyy + h);
    A.hzz = fma(fma(2.0, uz, -vz), dz, A.hzz + h);
    A.hxy = fma(ux - vx, dy, fma(uy, dx, A.hxy));
    A.hxz = fma(ux - vx, dz, fma(uz, dx, A.hxz));
    A.hyz = fma(uy - vy, dz, fma(uz, dy, A.hyz));
}

// FP32 record of a node that lies beyond the cut of every target of a tile:
// offset from the tile origin (no low part) and a'' = (sqrt(pi)/2) a' s2^(-3/2)
struct alignas(16) FarF {
    float yx, yy, yz, pad0;
    float ax, ay, az, pad1;
};

// Padding record of the far ring: zero vector, placed so far away that its
// terms underflow to zero.
__device__ __forceinline__ FarF pad_farf() {
    FarF f;
    f.yx = f.yy = f.yz = 1.0e18f;
    f.ax = f.ay = f.az = 0.0f;
    f.pad0 = f.pad1 = 0.0f;
    return f;
}

// K consecutive far records against one target: every node is beyond the cut
// of every target of the tile, so the kernel is the Laplace dipole.  With the
// width moved into a'' and r2 = |d|^2,
//   Phi -= (a''.d) r2^(-3/2),  grad Phi += 3 (a''.d) r2^(-5/2) d - a'' r2^(-3/2);
// the two gradient terms are summed apart (G += (a''.d) r2^(-5/2) d,
// H += a'' r2^(-3/2); the caller forms 3G - H once per run).  Positions are
// the FP32 offsets from the tile origin without the low parts: at |d| beyond
// the cut the rounding of the offsets is a relative error of a few units of
// FP32 rounding in d.
template <int K>
__device__ __forceinline__ void nodes32_far(const FarF *sh, float x, float y, float z, float &p, float &gx, float &gy,
                                            float &gz, float &hx, float &hy, float &hz) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const FarF s = sh[k];
        const float dx = x - s.yx, dy = y - s.yy, dz = z - s.yz;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float r = __builtin_amdgcn_rsqf(r2);
        const float rr = r * r, S = rr * r;
        const float ad = fmaf(s.ax, dx, fmaf(s.ay, dy, s.az * dz));
        p = fmaf(-ad, S, p);
        const float h = ad * S * rr;
        gx = fmaf(h, dx, gx);
        gy = fmaf(h, dy, gy);
        gz = fmaf(h, dz, gz);
        hx = fmaf(s.ax, S, hx);
        hy = fmaf(s.ay, S, hy);
        hz = fmaf(s.az, S, hz);
    }
}

__device__ __forceinline__ void pair32(const SrcF &s, float x, float y, float z, float xl, float yl, float zl,
                                       float &p, float &gx, float &gy, float &gz) {
    // d = (x_hi - y_hi) + (x_lo - y_lo): positions carried as float-float
    const float dx = (x - s.yx) + (xl - s.lx), dy = (y - s.yy) + (yl - s.ly), dz = (z - s.yz) + (zl - s.lz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ad = fmaf(s.ax, dx, fmaf(s.ay, dy, s.az * dz));
    float S, T;
    kfun32(r2 * s.s2, S, T);
    p = fmaf(-ad, S, p);
    const float g = ad * T * s.s2x2;
    gx = fmaf(g, dx, fmaf(-s.ax, S, gx));
    gy = fmaf(g, dy, fmaf(-s.ay, S, gy));
    gz = fmaf(g, dz, fmaf(-s.az, S, gz));
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------- FP64
template <int TILE>
__global__ __launch_bounds__(TILE) void k_p2p_direct_f64(
    int64_t nmax, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
    const double *__restrict__ ty, const double *__restrict__ tz, const int32_t *__restrict__ tmesh,
    const int64_t *__restrict__ node_off, const Src *__restrict__ src, const int32_t *__restrict__ out_idx,
    double *__restrict__ phi, double *__restrict__ grad, double *__restrict__ pairs) {
    __shared__ Src sh[TILE];
    const int64_t n = n_dev ? (int64_t)*n_dev : nmax;
    const int64_t t0 = (int64_t)blockIdx.x * TILE;
    if (t0 >= n) return;
    const int lane = threadIdx.x;
    const int64_t i = t0 + lane;
    const bool valid = i < n;
    const int64_t ii = valid ? i : n - 1;
    const double x = tx[ii], y = ty[ii], z = tz[ii];
    const int32_t m = tmesh[ii];
    const int64_t b = node_off[m], e = node_off[m + 1];
    // targets are sorted by mesh: the tile's node range runs from the first
    // target's mesh to the last target's mesh
    const int64_t tl = (t0 + TILE < n ? t0 + TILE : n) - 1;
    const int64_t lo = node_off[tmesh[t0]], hi = node_off[tmesh[tl] + 1];

    double sp = 0, ep = 0, sx = 0, ex = 0, sy = 0, ey = 0, sz = 0, ez = 0;
    for (int64_t c0 = lo; c0 < hi; c0 += TILE) {
        const int cnt = (int)(hi - c0 < TILE ? hi - c0 : TILE);
        __syncthreads();
        if (lane < cnt) sh[lane] = fold_src(src[c0 + lane]);
        else sh[lane] = pad_src();              // pad the chunk to whole node groups
        __syncthreads();
        double p = 0, gx = 0, gy = 0, gz = 0;
        const bool full = c0 >= b && c0 + cnt <= e;
        if (__all(full)) {
            for (int j = 0; j < cnt; j += kNodeGroup64) nodes64<kNodeGroup64>(sh + j, x, y, z, p, gx, gy, gz);
        } else {
            const int jb = (int)(b - c0 > 0 ? (b - c0 < cnt ? b - c0 : cnt) : 0);
            const int je = (int)(e - c0 < cnt ? (e - c0 > 0 ? e - c0 : 0) : cnt);
            for (int j = jb; j < je; ++j) pair64(sh[j], x, y, z, p, gx, gy, gz);
        }
        two_sum(sp, ep, p);
        two_sum(sx, ex, gx);
        two_sum(sy, ey, gy);
        two_sum(sz, ez, gz);
    }
    if (valid) {
        const int64_t o = out_idx ? (int64_t)out_idx[i] : i;
        phi[o] = sp + ep;
        if (grad) {
            grad[3 * o] = sx + ex;
            grad[3 * o + 1] = sy + ey;
            grad[3 * o + 2] = sz + ez;
        }
    }
    if (pairs) {                            // [0] pairs of real targets, [1] lane slots spent
        const double w = wave_sum(valid ? (double)(e - b) : 0.0), wl = wave_sum((double)(hi - lo));
        if ((lane & 63) == 0) { atomicAdd(pairs, w); atomicAdd(pairs + 1, wl); }
    }
}

// ---------------------------------------------------------------- mixed
template <int TILE>
__global__ __launch_bounds__(TILE) void k_p2p_direct_mixed(
    int64_t nmax, const int32_t *__restrict__ n_dev, const double *__restrict__ tx,
    const double *__restrict__ ty, const double *__restrict__ tz, const int32_t *__restrict__ tmesh,
    const int64_t *__restrict__ node_off, const Src *__restrict__ src, const int32_t *__restrict__ out_idx,
    double *__restrict__ phi, double *__restrict__ grad, double *__restrict__ pairs) {
    __shared__ SrcF sh[TILE];
    const int64_t n = n_dev ? (int64_t)*n_dev : nmax;
    const int64_t t0 = (int64_t)blockIdx.x * TILE;
    if (t0 >= n) return;
    const int lane = threadIdx.x;
    const int64_t i = t0 + lane;
    const bool valid = i < n;
    const int64_t ii = valid ? i : n - 1;
    // tile origin: positions are differenced in FP64 against it, then rounded
    const double ox = tx[t0], oy = ty[t0], oz = tz[t0];
    const double dxo = tx[ii] - ox, dyo = ty[ii] - oy, dzo = tz[ii] - oz;
    const float x = (float)dxo, y = (float)dyo, z = (float)dzo;
    const float xl = (float)(dxo - (double)x), yl = (float)(dyo - (double)y), zl = (float)(dzo - (double)z);
    const int32_t m = tmesh[ii];
    const int64_t b = node_off[m], e = node_off[m + 1];
    const int64_t tl = (t0 + TILE < n ? t0 + TILE : n) - 1;
    const int64_t lo = node_off[tmesh[t0]], hi = node_off[tmesh[tl] + 1];

    float sp = 0, ep = 0, sx = 0, ex = 0, sy = 0, ey = 0, sz = 0, ez = 0;
    for (int64_t c0 = lo; c0 < hi; c0 += TILE) {
        const int cnt = (int)(hi - c0 < TILE ? hi - c0 : TILE);
        __syncthreads();
        {
            SrcF f;
            if (lane < cnt) {
                const Src s = src[c0 + lane];
                const double qx = s.yx - ox, qy = s.yy - oy, qz = s.yz - oz;
                f.yx = (float)qx;
                f.yy = (float)qy;
                f.yz = (float)qz;
                f.lx = (float)(qx - (double)f.yx);
                f.ly = (float)(qy - (double)f.yy);
                f.lz = (float)(qz - (double)f.yz);
                f.s2 = (float)s.s2;
                f.ax = (float)(kFoldA * s.ax);
                f.ay = (float)(kFoldA * s.ay);
                f.az = (float)(kFoldA * s.az);
                f.s2x2 = (float)(kFoldT * s.s2x2);
            } else {
                f = pad_srcf();
            }
            f.pad = 0.0f;
            sh[lane] = f;
        }
        __syncthreads();
        const bool full = c0 >= b && c0 + cnt <= e;
        const int jb = full ? 0 : (int)(b - c0 > 0 ? (b - c0 < cnt ? b - c0 : cnt) : 0);
        const int je = full ? cnt : (int)(e - c0 < cnt ? (e - c0 > 0 ? e - c0 : 0) : cnt);
        const bool wave_full = __all(full);
        // FP32 partials over sub-chunks of 32 nodes, folded by two-sum
        for (int j0 = 0; j0 < cnt; j0 += 32) {
            float p = 0, gx = 0, gy = 0, gz = 0;
            const int j1 = j0 + 32 < cnt ? j0 + 32 : cnt;
            if (wave_full) {                // chunk padded with zero records to whole node groups
                for (int j = j0; j < j1; j += kNodeGroup) nodes32<kNodeGroup>(sh + j, x, y, z, xl, yl, zl, p, gx, gy, gz);
            } else {
                const int a0 = j0 > jb ? j0 : jb, a1 = j1 < je ? j1 : je;
                for (int j = a0; j < a1; ++j) pair32(sh[j], x, y, z, xl, yl, zl, p, gx, gy, gz);
            }
            two_sum_f(sp, ep, p);
            two_sum_f(sx, ex, gx);
            two_sum_f(sy, ey, gy);
            two_sum_f(sz, ez, gz);
        }
    }
    if (valid) {
        const int64_t o = out_idx ? (int64_t)out_idx[i] : i;
        phi[o] = (double)sp + (double)ep;
        if (grad) {
            grad[3 * o] = (double)sx + (double)ex;
            grad[3 * o + 1] = (double)sy + (double)ey;
            grad[3 * o + 2] = (double)sz + (double)ez;
        }
    }
    if (pairs) {                            // [0] pairs of real targets, [1] lane slots spent
        const double w = wave_sum(valid ? (double)(e - b) : 0.0), wl = wave_sum((double)(hi - lo));
        if ((lane & 63) == 0) { atomicAdd(pairs, w); atomicAdd(pairs + 1, wl); }
    }
}


// ------------------------------------------------------------ FMM eval
// One tile = up to TILE targets of one octree leaf.  Near field: the full
// kernel over the node ranges of the leaf's direct list, streamed through
// LDS; far field: the leaf's local expansion (L2P with its gradient).  The
// grid is persistent: workgroups walk the tile list, whose length is read on
// the device.
struct FmmEvalArgs {
    const int32_t *ntiles_dev, *tile_start;
    int64_t n_max;
    const int32_t *n_dev;
    const int32_t *sleaf;       // leaf of each sorted target (nboxes + m: outside mesh m's root)
    // tiles [tile_start[k], tile_start[k+1]) (the last ends at the target count)
    // hold at most TILE targets of one leaf
    const int32_t *sidx;
    const double *tx, *ty, *tz;
    const int32_t *out_idx;
    double *phi, *grad;
    const int32_t *p2p_beg, *p2p_end, *p2p_src;
    const int64_t *nb, *ne;
    const int32_t *lev, *ijk;
    const Src *src;
    int64_t nnodes;
    int32_t nboxes;
    const double *L;
    const double *M;            // multipole expansions (for the M2P lists)
    const int32_t *m2p_beg, *m2p_end, *m2p_src;
    const int32_t *child, *parent;
    const double *rmax;         // largest cut radius of each box's nodes
    int K;                      // separation criterion of the M2P lists
    int p, ncp;
    double tcut;                // x = rho^2 s2 at the cut (beyond it the Hessian pairs take the dipole form)
    const double *root;         // per-mesh root cubes (corner xyz, side)
    const int32_t *bmesh;
    double *pairs;
    // tile queue: [0] next tile, [1] finished workgroups; zero between
    // launches (the last workgroup to finish clears both)
    unsigned int *queue;
    const int32_t *order;       // queue position -> tile (most expensive first)
};

// next tile for the workgroup (uniform); tiles are handed out in list order
__device__ __forceinline__ int next_tile(const FmmEvalArgs &a, int *slot) {
    __syncthreads();                    // everyone has read the previous slot value
    if (threadIdx.x == 0) *slot = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    return *slot;
}

__device__ __forceinline__ void queue_done(const FmmEvalArgs &a) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(a.queue + 1, 1u) == gridDim.x - 1) {
            atomicExch(a.queue, 0u);
            atomicExch(a.queue + 1, 0u);
        }
    }
}

// The near list of a tile (its leaf's source boxes) is streamed as one packed
// sequence: up to TILE ranges at a time are prefix-summed in LDS and each
// chunk of TILE nodes is filled across range boundaries, so no chunk is left
// partly empty at the end of a small box.
template <int TILE>
struct RangeBatch {
    int64_t beg[TILE];
    int64_t off[TILE + 1];
};

// load ranges [e, e + nr) of the leaf's direct list and prefix-sum their
// lengths; returns the packed length (uniform)
template <int TILE>
__device__ __forceinline__ int64_t load_ranges(const FmmEvalArgs &a, RangeBatch<TILE> &rb, int e, int nr) {
    const int t = threadIdx.x;
    int64_t len = 0;
    if (t < nr) {
        const int32_t S = a.p2p_src[e + t];
        rb.beg[t] = a.nb[S];
        len = a.ne[S] - a.nb[S];
    }
    rb.off[t + 1] = len;
    if (t == 0) rb.off[0] = 0;
    __syncthreads();
    for (int d = 1; d < TILE; d <<= 1) {      // inclusive scan of off[1..TILE]
        int64_t v = (t >= d) ? rb.off[t + 1 - d] : 0;
        __syncthreads();
        rb.off[t + 1] += v;
        __syncthreads();
    }
    return rb.off[nr];
}

// node index of packed position v (v < total)
template <int TILE>
__device__ __forceinline__ int64_t packed_node(const RangeBatch<TILE> &rb, int nr, int64_t v) {
    int lo = 0, hi = nr;                       // last r with off[r] <= v
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (rb.off[mid] <= v) lo = mid; else hi = mid;
    }
    return rb.beg[lo] + (v - rb.off[lo]);
}

// local expansion of leaf B staged in LDS by the whole workgroup (the caller
// synchronises before use)
__device__ __forceinline__ void stage_local(const FmmEvalArgs &a, int32_t B, double *Ls) {
    const double *src = a.L + (int64_t)B * a.ncp;
    for (int k = threadIdx.x; k < a.ncp; k += blockDim.x) Ls[k] = src[k];
}

__device__ __forceinline__ void fmm_l2p(const FmmEvalArgs &a, int32_t B, const double *Ls, double x, double y,
                                        double z, double &ph, double g[3]) {
    const double s = box_side(a.root, a.bmesh, B, a.lev[B]);
    const double *o = a.root + 4 * a.bmesh[B];
    const double cx = o[0] + (a.ijk[3 * B] + 0.5) * s, cy = o[1] + (a.ijk[3 * B + 1] + 0.5) * s,
                 cz = o[2] + (a.ijk[3 * B + 2] + 0.5) * s;
    const double inv = 1.0 / s;
    fmm::l2p(Ls, (x - cx) * inv, (y - cy) * inv, (z - cz) * inv, inv, a.p, ph, g);
}

// M2P list of leaf B at this lane's target: the multipole expansion of each
// listed box is staged in buf (ncp doubles) by the whole workgroup and
// evaluated at (x, y, z) (section 4.4: the far kernel is the Laplace double
// layer, so a box whose nodes are all beyond the cut of every target of B
// contributes through its expansion).  Uniform over the workgroup; buf is free
// again when it returns.
__device__ __forceinline__ void fmm_m2p_list(const FmmEvalArgs &a, int32_t B, double *buf, double x, double y,
                                             double z, double &ph, double g[3]) {
    const int e0 = a.m2p_beg[B], e1 = a.m2p_end[B];
    for (int e = e0; e < e1; ++e) {
        const int32_t S = a.m2p_src[e];
        __syncthreads();
        const double *src = a.M + (int64_t)S * a.ncp;
        for (int k = threadIdx.x; k < a.ncp; k += blockDim.x) buf[k] = src[k];
        __syncthreads();
        const double s = box_side(a.root, a.bmesh, S, a.lev[S]);
        const double *o = a.root + 4 * a.bmesh[S];
        const double cx = o[0] + (a.ijk[3 * S] + 0.5) * s, cy = o[1] + (a.ijk[3 * S + 1] + 0.5) * s,
                     cz = o[2] + (a.ijk[3 * S + 2] + 0.5) * s;
        const double inv = 1.0 / s;
        double p1, g1[3];
        fmm::m2p(buf, (x - cx) * inv, (y - cy) * inv, (z - cz) * inv, inv, a.p, p1, g1);
        ph += p1;
        g[0] += g1[0];
        g[1] += g1[1];
        g[2] += g1[2];
    }
    __syncthreads();
}

// Far field at a target outside its mesh's root cube (every node is then
// beyond the cut, the root cube being padded by twice the largest cut
// radius): one lane walks mesh m's tree depth first without a stack (the
// eight children of a box are consecutive, so the next box after a subtree is
// the next sibling of the first ancestor that is not an eighth child).  A box
// that passes the M2P test of the lists for this point is evaluated from its
// multipole expansion, a leaf that does not is summed directly, any other box
// is opened.  Returns the direct pairs spent.
__device__ __forceinline__ double fmm_outside(const FmmEvalArgs &a, int32_t m, double x, double y, double z, double &ph,
                              double g[3]) {
    double npair = 0.0, p = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    int32_t b = m;                                  // level-0 box of mesh m
    while (b >= 0) {
        bool open = false;
        const int64_t n0 = a.nb[b], n1 = a.ne[b];
        if (n1 > n0) {
            const double s = box_side(a.root, a.bmesh, b, a.lev[b]);
            const double *o = a.root + 4 * a.bmesh[b];
            const double lo[3] = {o[0] + a.ijk[3 * b] * s, o[1] + a.ijk[3 * b + 1] * s, o[2] + a.ijk[3 * b + 2] * s};
            const double pt[3] = {x, y, z};
            double dc = 0.0, gap = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double c = lo[d] + 0.5 * s, e = pt[d] - c;
                const double gd = fmax(fmax(lo[d] - pt[d], pt[d] - (lo[d] + s)), 0.0);
                dc += e * e;
                gap += gd * gd;
            }
            if (dc >= (double)a.K * s * s && gap >= a.rmax[b] * a.rmax[b]) {
                double p1, g1[3];
                const double inv = 1.0 / s;
                fmm::m2p(a.M + (int64_t)b * a.ncp, (x - lo[0]) * inv - 0.5, (y - lo[1]) * inv - 0.5,
                         (z - lo[2]) * inv - 0.5, inv, a.p, p1, g1);
                p += p1;
                gx += g1[0];
                gy += g1[1];
                gz += g1[2];
            } else if (a.child[b] < 0) {
                for (int64_t k = n0; k < n1; ++k) pair64(fold_src(a.src[k]), x, y, z, p, gx, gy, gz);
                npair += (double)(n1 - n0);
            } else {
                open = true;
            }
        }
        if (open) {
            b = a.child[b];
        } else {
            while (b != m && b == a.child[a.parent[b]] + 7) b = a.parent[b];
            b = b == m ? -1 : b + 1;
        }
    }
    ph = p;
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
    return npair;
}

// Targets outside their mesh's root cube (their tiles are skipped by the
// tile kernels): one thread per target over the sorted targets, both
// precisions in FP64.
__global__ __launch_bounds__(256) void k_eval_outside(FmmEvalArgs a) {
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    double npair = 0.0, lanes = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t B = a.sleaf[i];
        if (B < a.nboxes) continue;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[i] : i;
        double ph, g[3];
        const double np = fmm_outside(a, B - a.nboxes, a.tx[ti], a.ty[ti], a.tz[ti], ph, g);
        npair += np;
        lanes += np;
        const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
        a.phi[o] = ph;
        if (a.grad) {
            a.grad[3 * o] = g[0];
            a.grad[3 * o + 1] = g[1];
            a.grad[3 * o + 2] = g[2];
        }
    }
    if (a.pairs && npair > 0.0) {           // [0] pairs of real targets, [1] lane slots spent
        atomicAdd(a.pairs, npair);
        atomicAdd(a.pairs + 1, lanes);
    }
}

// ---------------------------------------------------------------- Hessian
// Phi, grad Phi and the Hessian through the same tree and lists (section
// 3.1 needs the Hessian for the charts' second derivatives): the near list
// with the full kernel and its third radial function inside the cut
// (pair_hess_cut: the double layer beyond it, as in the far field), the M2P
// list and the leaf's local expansion with their second derivatives
// (fmm::m2p_hess, fmm::l2p_hess).  Beyond the cut the kernel is the Laplace
// double layer to the truncation of the cut (8 sigma: P(7/2, 32) differs from
// 1 by 2e-11 relative, so the Hessian bar is looser than the field's).  FP64
// in either precision setting; the context's cut and order set the accuracy.
__device__ __forceinline__ void fmm_m2p_list_hess(const FmmEvalArgs &a, int32_t B, double *buf, double x, double y,
                                                  double z, double &ph, double g[3], double H[6]) {
    const int e0 = a.m2p_beg[B], e1 = a.m2p_end[B];
    for (int e = e0; e < e1; ++e) {
        const int32_t S = a.m2p_src[e];
        __syncthreads();
        const double *src = a.M + (int64_t)S * a.ncp;
        for (int k = threadIdx.x; k < a.ncp; k += blockDim.x) buf[k] = src[k];
        __syncthreads();
        const double s = box_side(a.root, a.bmesh, S, a.lev[S]);
        const double *o = a.root + 4 * a.bmesh[S];
        const double inv = 1.0 / s;
        const double rx = (x - (o[0] + (a.ijk[3 * S] + 0.5) * s)) * inv;
        const double ry = (y - (o[1] + (a.ijk[3 * S + 1] + 0.5) * s)) * inv;
        const double rz = (z - (o[2] + (a.ijk[3 * S + 2] + 0.5) * s)) * inv;
        double p1, g1[3], h1[6];
        fmm::m2p(buf, rx, ry, rz, inv, a.p, p1, g1);
        fmm::m2p_hess(buf, rx, ry, rz, inv, a.p, h1);
        ph += p1;
        for (int d = 0; d < 3; ++d) g[d] += g1[d];
        for (int d = 0; d < 6; ++d) H[d] += h1[d];
    }
    __syncthreads();
}

// one workgroup of TILE lanes per tile (the tiles of the evaluation, at most
// TILE targets of one leaf), tiles taken in a grid-stride loop.  With 64-lane
// tiles (one wave) every staged node is tested against the tile's target
// bounding box: nodes beyond the cut of every target of the tile take the
// folded far form (pair_hess_far), the others pair_hess_cut, which still
// chooses per pair.
template <int TILE>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(3))) void k_hess_fmm(FmmEvalArgs a, double *hess) {
    constexpr bool kSplit = TILE == 64;
    __shared__ Src sh[TILE];
    __shared__ FarD shf[kSplit ? TILE : 1];
    __shared__ double tbox[6];          // the tile's target bounding box
    __shared__ RangeBatch<TILE> rb;
    extern __shared__ double Ls[];      // local expansion of the tile's leaf (ncp doubles)
    const int ntiles = *a.ntiles_dev;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    const int lane = threadIdx.x;
    const double far_t = a.tcut * (1.0 + 1e-6);         // margin over the rounding of the box gap
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = a.tile_start[tile];
        const int32_t B = a.sleaf[s0];
        const int64_t s1 = tile + 1 < ntiles ? (int64_t)a.tile_start[tile + 1] : n;
        if (B >= a.nboxes) continue;        // outside the root cube: k_hess_outside
        const int64_t sp_ = s0 + lane;
        const bool valid = sp_ < s1;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[valid ? sp_ : s0] : (valid ? sp_ : s0);
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        const int e0 = a.p2p_beg[B], e1 = a.p2p_end[B];
        if (kSplit) {
            double blo[3] = {x, y, z}, bhi[3] = {x, y, z};      // lanes past the tile end hold its first target
            for (int off = 32; off > 0; off >>= 1)
                for (int c = 0; c < 3; ++c) {
                    blo[c] = fmin(blo[c], __shfl_xor(blo[c], off));
                    bhi[c] = fmax(bhi[c], __shfl_xor(bhi[c], off));
                }
            __syncthreads();                // the previous tile is done with tbox
            if (lane == 0)
                for (int c = 0; c < 3; ++c) {
                    tbox[c] = blo[c];
                    tbox[3 + c] = bhi[c];
                }
        }
        HessAcc A;
        for (int eb = e0; eb < e1; eb += TILE) {
            const int nr = e1 - eb < TILE ? e1 - eb : TILE;
            __syncthreads();
            const int64_t total = load_ranges<TILE>(a, rb, eb, nr);
            for (int64_t c0 = 0; c0 < total; c0 += TILE) {
                const int cnt = (int)(total - c0 < TILE ? total - c0 : TILE);
                __syncthreads();
                if (kSplit) {
                    Src sr;
                    bool isfar = false;
                    if (lane < cnt) {
                        sr = a.src[packed_node<TILE>(rb, nr, c0 + lane)];
                        const double gx_ = fmax(fmax(tbox[0] - sr.yx, sr.yx - tbox[3]), 0.0);
                        const double gy_ = fmax(fmax(tbox[1] - sr.yy, sr.yy - tbox[4]), 0.0);
                        const double gz_ = fmax(fmax(tbox[2] - sr.yz, sr.yz - tbox[5]), 0.0);
                        isfar = (gx_ * gx_ + gy_ * gy_ + gz_ * gz_) * sr.s2 >= far_t;
                    }
                    const uint64_t fm = __ballot(isfar), nm = __ballot(lane < cnt && !isfar);
                    if (lane < cnt && !isfar) {
                        sh[below(nm)] = sr;
                    } else if (isfar) {
                        const double fa = kFoldA / (sr.s2 * sqrt(sr.s2));     // a''
                        FarD f;
                        f.yx = sr.yx;
                        f.yy = sr.yy;
                        f.yz = sr.yz;
                        f.ax = fa * sr.ax;
                        f.ay = fa * sr.ay;
                        f.az = fa * sr.az;
                        shf[below(fm)] = f;
                    }
                    __syncthreads();
                    const int nn = __popcll(nm), nf = __popcll(fm);
                    for (int j = 0; j < nn; ++j) pair_hess_cut(sh[j], x, y, z, a.tcut, A);
                    for (int j = 0; j < nf; ++j) pair_hess_far(shf[j], x, y, z, A);
                } else {
                    if (lane < cnt) sh[lane] = a.src[packed_node<TILE>(rb, nr, c0 + lane)];
                    __syncthreads();
                    for (int j = 0; j < cnt; ++j) pair_hess_cut(sh[j], x, y, z, a.tcut, A);
                }
            }
        }
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0}, H[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        fmm_m2p_list_hess(a, B, Ls, x, y, z, ph, g, H);
        stage_local(a, B, Ls);
        __syncthreads();
        {
            double lp, lg[3];                // fmm_l2p writes (does not add) its outputs
            fmm_l2p(a, B, Ls, x, y, z, lp, lg);
            ph += lp;
            for (int d = 0; d < 3; ++d) g[d] += lg[d];
        }
        {
            const double s = box_side(a.root, a.bmesh, B, a.lev[B]);
            const double *o = a.root + 4 * a.bmesh[B];
            const double inv = 1.0 / s;
            double h1[6];
            fmm::l2p_hess(Ls, (x - (o[0] + (a.ijk[3 * B] + 0.5) * s)) * inv,
                          (y - (o[1] + (a.ijk[3 * B + 1] + 0.5) * s)) * inv,
                          (z - (o[2] + (a.ijk[3 * B + 2] + 0.5) * s)) * inv, inv, a.p, h1);
            for (int d = 0; d < 6; ++d) H[d] += h1[d];
        }
        __syncthreads();                    // everyone is done with Ls before the next tile
        if (valid) {
            const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
            if (a.phi) a.phi[o] = A.f + ph;
            if (a.grad) {
                a.grad[3 * o] = A.gx + g[0];
                a.grad[3 * o + 1] = A.gy + g[1];
                a.grad[3 * o + 2] = A.gz + g[2];
            }
            double *q = hess + 6 * o;
            q[0] = A.hxx + H[0];
            q[1] = A.hxy + H[1];
            q[2] = A.hxz + H[2];
            q[3] = A.hyy + H[3];
            q[4] = A.hyz + H[4];
            q[5] = A.hzz + H[5];
        }
    }
}

// targets outside their mesh's root cube: the direct sum over the mesh's
// nodes (the level-0 box m holds them all), one thread per target
__global__ __launch_bounds__(256) void k_hess_outside(FmmEvalArgs a, double *hess) {
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t B = a.sleaf[i];
        if (B < a.nboxes) continue;
        const int32_t m = B - a.nboxes;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[i] : i;
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        HessAcc A;
        for (int64_t k = a.nb[m]; k < a.ne[m]; ++k) pair_hess(a.src[k], x, y, z, A);
        const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
        if (a.phi) a.phi[o] = A.f;
        if (a.grad) {
            a.grad[3 * o] = A.gx;
            a.grad[3 * o + 1] = A.gy;
            a.grad[3 * o + 2] = A.gz;
        }
        double *q = hess + 6 * o;
        q[0] = A.hxx;
        q[1] = A.hxy;
        q[2] = A.hxz;
        q[3] = A.hyy;
        q[4] = A.hyz;
        q[5] = A.hzz;
    }
}

// ------------------------------------------------ target-attached width
// Phi and grad Phi with sigma(x) (section 2, eq. basemodelk, sigma2) through
// a tree whose lists were built for these targets: a box is admissible when
// its gap clears cut * sigma(x) of every target in it, so every pair within
// the cut of sigma(x) is in a near list.  Near pairs use the target's width
// (pair_ms, which carries c(sigma(x)) a); the far field (Laplace double
// layer) does not depend on the width.  grad Phi gains (dPhi/dsigma) grad
// sigma, dPhi/dsigma = (2 c(x) / sigma(x)) sum (a.d) exp(-t) over the near
// pairs (beyond the cut exp(-t) is below the cut's truncation).  FP64.
__device__ __forceinline__ void ms_finish(double sx, const MsAcc &A, const double *gs, double &ph, double g[3]) {
    // Phi = -sum (c(x) a.d) k1, grad = -sum (c(x) a k1 + (c(x) a.d) k2 d),
    // dPhi/dsigma = (2 / sigma(x)) sum (c(x) a.d) e^-t
    const double dps = 2.0 * A.e / sx;
    ph -= A.f;
    g[0] += -A.gx + dps * gs[0];
    g[1] += -A.gy + dps * gs[1];
    g[2] += -A.gz + dps * gs[2];
}

template <int TILE>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(3))) void k_multiscale_fmm(FmmEvalArgs a, MsArgs ms) {
    // with 64-lane tiles (one wave) nodes beyond the cut of every target of
    // the tile (the gap to the tile's bounding box against the tile's largest
    // sigma(x)) take the Laplace double layer (nodes64_far), the others
    // pair_ms_cut, which still chooses per pair
    constexpr bool kSplit = TILE == 64;
    __shared__ Src sh[TILE];
    __shared__ FarD shf[kSplit ? TILE : 1];
    __shared__ double tbox[7];          // the tile's target bounding box and smallest s2(x)
    __shared__ RangeBatch<TILE> rb;
    extern __shared__ double Ls[];
    const int ntiles = *a.ntiles_dev;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    const int lane = threadIdx.x;
    const double far_t = ms.tcut * (1.0 + 1e-6);        // margin over the rounding of the box gap
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = a.tile_start[tile];
        const int32_t B = a.sleaf[s0];
        const int64_t s1 = tile + 1 < ntiles ? (int64_t)a.tile_start[tile + 1] : n;
        if (B >= a.nboxes) continue;        // outside the root cube: k_multiscale_outside
        const int64_t sp_ = s0 + lane;
        const bool valid = sp_ < s1;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[valid ? sp_ : s0] : (valid ? sp_ : s0);
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        const double sx = ms.sig[ti], s2x = 0.5 / (sx * sx);
        const int e0 = a.p2p_beg[B], e1 = a.p2p_end[B];
        if (kSplit) {
            double blo[4] = {x, y, z, s2x}, bhi[3] = {x, y, z};     // lanes past the tile end hold its first target
            for (int off = 32; off > 0; off >>= 1) {
                for (int c = 0; c < 3; ++c) {
                    blo[c] = fmin(blo[c], __shfl_xor(blo[c], off));
                    bhi[c] = fmax(bhi[c], __shfl_xor(bhi[c], off));
                }
                blo[3] = fmin(blo[3], __shfl_xor(blo[3], off));
            }
            __syncthreads();                // the previous tile is done with tbox
            if (lane == 0) {
                for (int c = 0; c < 3; ++c) {
                    tbox[c] = blo[c];
                    tbox[3 + c] = bhi[c];
                }
                tbox[6] = blo[3];
            }
        }
        MsAcc A;
        double pf = 0.0, gfx = 0.0, gfy = 0.0, gfz = 0.0;  // the far nodes' double layer
        for (int eb = e0; eb < e1; eb += TILE) {
            const int nr = e1 - eb < TILE ? e1 - eb : TILE;
            __syncthreads();
            const int64_t total = load_ranges<TILE>(a, rb, eb, nr);
            for (int64_t c0 = 0; c0 < total; c0 += TILE) {
                const int cnt = (int)(total - c0 < TILE ? total - c0 : TILE);
                __syncthreads();
                if (kSplit) {
                    Src r;
                    bool isfar = false;
                    if (lane < cnt) {
                        r = a.src[packed_node<TILE>(rb, nr, c0 + lane)];
                        const double gx_ = fmax(fmax(tbox[0] - r.yx, r.yx - tbox[3]), 0.0);
                        const double gy_ = fmax(fmax(tbox[1] - r.yy, r.yy - tbox[4]), 0.0);
                        const double gz_ = fmax(fmax(tbox[2] - r.yz, r.yz - tbox[5]), 0.0);
                        isfar = (gx_ * gx_ + gy_ * gy_ + gz_ * gz_) * tbox[6] >= far_t;
                    }
                    const uint64_t fm = __ballot(isfar), nm = __ballot(lane < cnt && !isfar);
                    if (lane < cnt) {           // a' s2^(-3/2): the width moves to the target
                        const double f = 1.0 / (r.s2 * sqrt(r.s2));
                        if (!isfar) {
                            r.ax *= f;
                            r.ay *= f;
                            r.az *= f;
                            sh[below(nm)] = r;
                        } else {                // a'' = (sqrt(pi)/2) a' s2^(-3/2)
                            FarD q;
                            q.yx = r.yx;
                            q.yy = r.yy;
                            q.yz = r.yz;
                            q.ax = kFoldA * f * r.ax;
                            q.ay = kFoldA * f * r.ay;
                            q.az = kFoldA * f * r.az;
                            shf[below(fm)] = q;
                        }
                    }
                    __syncthreads();
                    const int nn = __popcll(nm), nf = __popcll(fm);
                    for (int j = 0; j < nn; ++j) pair_ms_cut(sh[j], x, y, z, s2x, ms.tcut, A);
                    for (int j = 0; j < nf; ++j) pair_far64(shf[j], x, y, z, pf, gfx, gfy, gfz);
                } else {
                    if (lane < cnt) {           // a' s2^(-3/2): the width moves to the target (pair_ms_cut)
                        Src r = a.src[packed_node<TILE>(rb, nr, c0 + lane)];
                        const double f = 1.0 / (r.s2 * sqrt(r.s2));
                        r.ax *= f;
                        r.ay *= f;
                        r.az *= f;
                        sh[lane] = r;
                    }
                    __syncthreads();
                    for (int j = 0; j < cnt; ++j) pair_ms_cut(sh[j], x, y, z, s2x, ms.tcut, A);
                }
            }
        }
        {
            const double fx = s2x * sqrt(s2x);
            A.f *= fx;
            A.gx *= fx;
            A.gy *= fx;
            A.gz *= fx;
            A.e *= fx;
        }
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0};
        if (a.m2p_end[B] > a.m2p_beg[B]) fmm_m2p_list(a, B, Ls, x, y, z, ph, g);
        stage_local(a, B, Ls);
        __syncthreads();
        {
            double lp, lg[3];
            fmm_l2p(a, B, Ls, x, y, z, lp, lg);
            ph += lp;
            for (int d = 0; d < 3; ++d) g[d] += lg[d];
        }
        __syncthreads();
        if (valid) {
            ms_finish(sx, A, ms.gsig + 3 * ti, ph, g);
            ph += pf;                       // the double layer of the far nodes
            g[0] += gfx;
            g[1] += gfy;
            g[2] += gfz;
            const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
            a.phi[o] = ph;
            if (a.grad) {
                a.grad[3 * o] = g[0];
                a.grad[3 * o + 1] = g[1];
                a.grad[3 * o + 2] = g[2];
            }
        }
    }
}

// targets outside their mesh's root cube: every node of the mesh
__global__ __launch_bounds__(256) void k_multiscale_outside(FmmEvalArgs a, MsArgs ms) {
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t B = a.sleaf[i];
        if (B < a.nboxes) continue;
        const int32_t m = B - a.nboxes;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[i] : i;
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        const double sx = ms.sig[ti], s2x = 0.5 / (sx * sx);
        MsAcc A;
        for (int64_t k = a.nb[m]; k < a.ne[m]; ++k) pair_ms(a.src[k], x, y, z, s2x, A);
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0};
        ms_finish(sx, A, ms.gsig + 3 * ti, ph, g);
        const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
        a.phi[o] = ph;
        if (a.grad) {
            a.grad[3 * o] = g[0];
            a.grad[3 * o + 1] = g[1];
            a.grad[3 * o + 2] = g[2];
        }
    }
}

// Four waves per SIMD: the compiler fits the kernel in 128 VGPRs with a few
// spills outside the chunk loop (1% faster on C5 than three waves at 139).
// COUNT: also count the pairs inside the cut (pairs[2]), for the statistics
template <int TILE, bool COUNT>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_fmm_f64(FmmEvalArgs a) {
    __shared__ Src sh[TILE];
    __shared__ RangeBatch<TILE> rb;
    extern __shared__ double Ls[];      // local expansion of the tile's leaf (ncp doubles)
    const int ntiles = *a.ntiles_dev;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    const int lane = threadIdx.x;
    __shared__ int slot;
    for (int q = next_tile(a, &slot); q < ntiles; q = next_tile(a, &slot)) {
        const int tile = a.order[q];
        const int64_t s0 = a.tile_start[tile];
        const int32_t leafk = a.sleaf[s0];
        const int64_t s1 = tile + 1 < ntiles ? (int64_t)a.tile_start[tile + 1] : n;   // tile = [s0, s1)
        const int64_t sp_ = s0 + lane;
        const bool valid = sp_ < s1;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[valid ? sp_ : s0] : (valid ? sp_ : s0);
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        const int32_t B = leafk;
        if (B >= a.nboxes) continue;        // outside the root cube: k_eval_outside
        const int e0 = a.p2p_beg[B], e1 = a.p2p_end[B];
        __syncthreads();                    // previous tile is done with Ls
        stage_local(a, B, Ls);
        double sp = 0, ep = 0, sx = 0, ex = 0, sy = 0, ey = 0, sz = 0, ez = 0;
        double npair = 0.0;
        uint32_t nuse = 0;
        for (int eb = e0; eb < e1; eb += TILE) {
            const int nr = e1 - eb < TILE ? e1 - eb : TILE;
            __syncthreads();
            const int64_t total = load_ranges<TILE>(a, rb, eb, nr);
            npair += (double)total;
            for (int64_t c0 = 0; c0 < total; c0 += TILE) {
                const int cnt = (int)(total - c0 < TILE ? total - c0 : TILE);
                __syncthreads();
                if (lane < cnt) sh[lane] = fold_src(a.src[packed_node<TILE>(rb, nr, c0 + lane)]);
                else sh[lane] = pad_src();      // pad the chunk to whole node groups
                __syncthreads();
                double p = 0, gx = 0, gy = 0, gz = 0;
                for (int j = 0; j < cnt; j += kNodeGroup64)
                    nodes64<kNodeGroup64, COUNT>(sh + j, x, y, z, p, gx, gy, gz, &nuse);
                two_sum(sp, ep, p);
                two_sum(sx, ex, gx);
                two_sum(sy, ey, gy);
                two_sum(sz, ez, gz);
            }
        }
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0}, mph = 0.0, mg[3] = {0.0, 0.0, 0.0};
        if (a.m2p_end[B] > a.m2p_beg[B]) {  // uniform: Ls is the M2P staging buffer, then L again
            fmm_m2p_list(a, B, Ls, x, y, z, mph, mg);
            stage_local(a, B, Ls);
        }
        __syncthreads();                    // Ls staged
        fmm_l2p(a, B, Ls, x, y, z, ph, g);
        ph += mph;
        g[0] += mg[0];
        g[1] += mg[1];
        g[2] += mg[2];
        if (valid) {
            const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
            a.phi[o] = (sp + ph) + ep;
            if (a.grad) {
                a.grad[3 * o] = (sx + g[0]) + ex;
                a.grad[3 * o + 1] = (sy + g[1]) + ey;
                a.grad[3 * o + 2] = (sz + g[2]) + ez;
            }
        }
        if (a.pairs) {                      // [0] pairs of real targets, [1] lane slots spent, [2] inside the cut
            const double w = wave_sum(valid ? npair : 0.0), wl = wave_sum(npair);
            const double wu = COUNT ? wave_sum(valid ? (double)nuse : 0.0) : 0.0;
            if ((lane & 63) == 0) {
                atomicAdd(a.pairs, w);
                atomicAdd(a.pairs + 1, wl);
                if (COUNT) atomicAdd(a.pairs + 2, wu);
            }
        }
    }
    queue_done(a);
}


// FP64 path with 64-target tiles: as the mixed kernel below, every staged
// node is tested against the tile's target bounding box and goes to the near
// ring (the general loop: the far form for every pair, the rational fit for
// node groups with a pair inside the cut) or to the far ring (the dipole-only
// loop).  Nodes are staged 32 at a time, so that the two rings (7 KB) leave
// room for the 16 workgroups of four waves per SIMD in a CU's LDS.
constexpr int kNodeGroupSplit = 2;       // node group of the split kernel (fewer registers than 4)
constexpr int kRun64 = 32;               // records per partial sum
constexpr int kRing64 = 64;              // kRun64 - 1 left over + 32 staged

constexpr size_t kF64RingBytes = kRing64 * (sizeof(Src) + sizeof(FarD));

template <bool COUNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_fmm_f64_split(FmmEvalArgs a) {
    constexpr int W = 64;
    __shared__ RangeBatch<W> rb;
    __shared__ double tbox[6];          // the tile's target bounding box
    // node rings while the pairs run, then the local expansion (ncp doubles)
    // and the M2P staging buffer
    extern __shared__ __attribute__((aligned(16))) double Ls[];
    Src *ring_n = reinterpret_cast<Src *>(Ls);
    FarD *ring_f = reinterpret_cast<FarD *>(ring_n + kRing64);
    const int ntiles = *a.ntiles_dev;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    const int lane = threadIdx.x;
    const double far_u = KF64_X * (1.0 + 1e-6);
    __shared__ int slot;
    for (int q = next_tile(a, &slot); q < ntiles; q = next_tile(a, &slot)) {
        const int tile = a.order[q];
        const int64_t s0 = a.tile_start[tile];
        const int32_t B = a.sleaf[s0];
        if (B >= a.nboxes) continue;        // outside the root cube: k_eval_outside
        const int64_t s1 = tile + 1 < ntiles ? (int64_t)a.tile_start[tile + 1] : n;   // tile = [s0, s1)
        const int64_t sp_ = s0 + lane;
        const bool valid = sp_ < s1;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[valid ? sp_ : s0] : (valid ? sp_ : s0);
        const double x = a.tx[ti], y = a.ty[ti], z = a.tz[ti];
        const int e0 = a.p2p_beg[B], e1 = a.p2p_end[B];
        {
            double blo[3] = {x, y, z}, bhi[3] = {x, y, z};      // lanes past the tile end hold its first target
            for (int off = 32; off > 0; off >>= 1)
                for (int c = 0; c < 3; ++c) {
                    blo[c] = fmin(blo[c], __shfl_xor(blo[c], off));
                    bhi[c] = fmax(bhi[c], __shfl_xor(bhi[c], off));
                }
            __syncthreads();                // the previous tile is done with tbox
            if (lane == 0)
                for (int c = 0; c < 3; ++c) {
                    tbox[c] = blo[c];
                    tbox[3 + c] = bhi[c];
                }
        }
        double sp = 0, ep = 0, sx = 0, ex = 0, sy = 0, ey = 0, sz = 0, ez = 0;
        double npair = 0.0, nfar = 0.0;
        uint32_t nuse = 0;
        int hn = 0, nn = 0, hf = 0, nf = 0;     // head and fill of each ring (uniform)
        int eb = e0, nr = 0;
        int64_t total = 0, c0 = 0;
        for (bool last = false; !last;) {
            while (c0 >= total && eb < e1) {    // next batch of the leaf's direct list
                nr = e1 - eb < W ? e1 - eb : W;
                __syncthreads();
                total = load_ranges<W>(a, rb, eb, nr);
                npair += (double)total;
                c0 = 0;
                eb += nr;
            }
            last = c0 >= total;             // every node is staged: pad the remainders
            const int cnt = last ? 0 : (int)(total - c0 < kRun64 ? total - c0 : kRun64);
            Src sr;
            bool isfar = false;
            if (lane < cnt) {
                sr = a.src[packed_node<W>(rb, nr, c0 + lane)];
                const double gx_ = fmax(fmax(tbox[0] - sr.yx, sr.yx - tbox[3]), 0.0);
                const double gy_ = fmax(fmax(tbox[1] - sr.yy, sr.yy - tbox[4]), 0.0);
                const double gz_ = fmax(fmax(tbox[2] - sr.yz, sr.yz - tbox[5]), 0.0);
                isfar = (gx_ * gx_ + gy_ * gy_ + gz_ * gz_) * sr.s2 >= far_u;
            }
            c0 += cnt;
            const uint64_t fm = __ballot(isfar), nm = __ballot(lane < cnt && !isfar);
            __syncthreads();                // the runs taken last are read
            if (lane < cnt && !isfar) {
                int pos = hn + nn + below(nm);
                if (pos >= kRing64) pos -= kRing64;
                ring_n[pos] = fold_src(sr);
            } else if (isfar) {
                int pos = hf + nf + below(fm);
                if (pos >= kRing64) pos -= kRing64;
                const double fa = kFoldA / (sr.s2 * sqrt(sr.s2));     // a'' (nodes64_far)
                FarD f;
                f.yx = sr.yx;
                f.yy = sr.yy;
                f.yz = sr.yz;
                f.ax = fa * sr.ax;
                f.ay = fa * sr.ay;
                f.az = fa * sr.az;
                ring_f[pos] = f;
            }
            nn += __popcll(nm);
            nf += __popcll(fm);
            if (COUNT) nfar += (double)__popcll(fm);
            // a full run of a ring, or at the end its remainder (< kRun64 records,
            // contiguous since the heads are multiples of kRun64) padded to whole
            // node groups
            const int ln = nn >= kRun64 ? kRun64 : (last ? (nn + kNodeGroupSplit - 1) / kNodeGroupSplit * kNodeGroupSplit : 0);
            const int lf = nf >= kRun64 ? kRun64 : (last ? (nf + kNodeGroupSplit - 1) / kNodeGroupSplit * kNodeGroupSplit : 0);
            if (last) {
                if (lane >= nn && lane < ln) ring_n[hn + lane] = pad_src();
                if (lane >= nf && lane < lf) ring_f[hf + lane] = pad_fard();
            }
            __syncthreads();
            if (ln > 0) {
                double p = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll 1
                for (int j = 0; j < ln; j += kNodeGroupSplit)
                    nodes64<kNodeGroupSplit, COUNT>(ring_n + hn + j, x, y, z, p, gx, gy, gz, &nuse);
                two_sum(sp, ep, p);
                two_sum(sx, ex, gx);
                two_sum(sy, ey, gy);
                two_sum(sz, ez, gz);
                hn = hn + kRun64 == kRing64 ? 0 : hn + kRun64;
                nn = nn > kRun64 ? nn - kRun64 : 0;
            }
            if (lf > 0) {
                double p = 0, gx = 0, gy = 0, gz = 0, hx = 0, hy = 0, hz = 0;
#pragma unroll 1
                for (int j = 0; j < lf; j += kNodeGroupSplit)
                    nodes64_far<kNodeGroupSplit>(ring_f + hf + j, x, y, z, p, gx, gy, gz, hx, hy, hz);
                gx = fma(3.0, gx, -hx);
                gy = fma(3.0, gy, -hy);
                gz = fma(3.0, gz, -hz);
                two_sum(sp, ep, p);
                two_sum(sx, ex, gx);
                two_sum(sy, ey, gy);
                two_sum(sz, ez, gz);
                hf = hf + kRun64 == kRing64 ? 0 : hf + kRun64;
                nf = nf > kRun64 ? nf - kRun64 : 0;
            }
        }
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0}, mph = 0.0, mg[3] = {0.0, 0.0, 0.0};
        if (a.m2p_end[B] > a.m2p_beg[B])    // uniform: Ls is the M2P staging buffer first
            fmm_m2p_list(a, B, Ls, x, y, z, mph, mg);
        __syncthreads();                    // the rings (or the M2P buffer) are done
        stage_local(a, B, Ls);
        __syncthreads();                    // Ls staged
        fmm_l2p(a, B, Ls, x, y, z, ph, g);
        ph += mph;
        g[0] += mg[0];
        g[1] += mg[1];
        g[2] += mg[2];
        if (valid) {
            const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
            a.phi[o] = (sp + ph) + ep;
            if (a.grad) {
                a.grad[3 * o] = (sx + g[0]) + ex;
                a.grad[3 * o + 1] = (sy + g[1]) + ey;
                a.grad[3 * o + 2] = (sz + g[2]) + ez;
            }
        }
        if (a.pairs) {                      // [0] pairs of real targets, [1] lane slots spent, [2] inside the cut,
                                            // [3] taken by the dipole-only loop
            const double w = wave_sum(valid ? npair : 0.0), wl = wave_sum(npair);
            const double wu = COUNT ? wave_sum(valid ? (double)nuse : 0.0) : 0.0;
            const double wf = COUNT ? wave_sum(valid ? nfar : 0.0) : 0.0;
            if (lane == 0) {
                atomicAdd(a.pairs, w);
                atomicAdd(a.pairs + 1, wl);
                if (COUNT) {
                    atomicAdd(a.pairs + 2, wu);
                    atomicAdd(a.pairs + 3, wf);
                }
            }
        }
    }
    queue_done(a);
}

// Mixed path: one wavefront per tile of 64 targets.  Each staged node is
// tested against the tile's target bounding box: a node whose distance to the
// box is beyond its cut radius (u >= KF32_X for every target of the tile)
// goes to the far ring and the dipole-only loop, every other node to the near
// ring and the general loop (float-float offsets, the rational fit for node
// groups with a pair inside the cut).  Each ring is drained in runs of kRun
// records, one compensated partial sum per run; the remainders are padded to
// whole node groups at the end of the tile.  The rings share the dynamic LDS
// with the local expansion, which is staged once the pairs are done.
constexpr int kRun = 32;                 // records per partial sum

constexpr int kRing = 96;                // ring capacity: kRun - 1 left over + 64 staged
constexpr size_t kMixedRingBytes = kRing * (sizeof(SrcF) + sizeof(FarF));

template <bool COUNT>
__global__ __launch_bounds__(64) void k_eval_fmm_mixed(FmmEvalArgs a) {
    constexpr int W = 64;
    __shared__ RangeBatch<W> rb;
    __shared__ double tbox[6];          // the tile's target bounding box (offsets from its origin)
    // node rings while the pairs run, then the local expansion (ncp doubles)
    // and the M2P staging buffer
    extern __shared__ __attribute__((aligned(16))) double Ls[];
    SrcF *ring_n = reinterpret_cast<SrcF *>(Ls);
    FarF *ring_f = reinterpret_cast<FarF *>(ring_n + kRing);
    const int ntiles = *a.ntiles_dev;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n_max;
    const int lane = threadIdx.x;
    const double far_u = (double)KF32_X * (1.0 + 1e-4);     // margin over the FP32 rounding of u
    __shared__ int slot;
    for (int q = next_tile(a, &slot); q < ntiles; q = next_tile(a, &slot)) {
        const int tile = a.order[q];
        const int64_t s0 = a.tile_start[tile];
        const int32_t B = a.sleaf[s0];
        if (B >= a.nboxes) continue;        // outside the root cube: k_eval_outside
        const int64_t s1 = tile + 1 < ntiles ? (int64_t)a.tile_start[tile + 1] : n;   // tile = [s0, s1)
        const int64_t sp_ = s0 + lane;
        const bool valid = sp_ < s1;
        const int64_t ti = a.sidx ? (int64_t)a.sidx[valid ? sp_ : s0] : (valid ? sp_ : s0);
        const int64_t t0 = a.sidx ? (int64_t)a.sidx[s0] : s0;
        const double ox = a.tx[t0], oy = a.ty[t0], oz = a.tz[t0];     // tile origin
        const double dxo = a.tx[ti] - ox, dyo = a.ty[ti] - oy, dzo = a.tz[ti] - oz;
        const float x = (float)dxo, y = (float)dyo, z = (float)dzo;
        const float xl = (float)(dxo - (double)x), yl = (float)(dyo - (double)y), zl = (float)(dzo - (double)z);
        const int e0 = a.p2p_beg[B], e1 = a.p2p_end[B];
        // bounding box of the tile's targets (offsets from the origin; the
        // lanes past the tile end hold the first target)
        double blo[3] = {dxo, dyo, dzo}, bhi[3] = {dxo, dyo, dzo};
        for (int off = 32; off > 0; off >>= 1)
            for (int c = 0; c < 3; ++c) {
                blo[c] = fmin(blo[c], __shfl_xor(blo[c], off));
                bhi[c] = fmax(bhi[c], __shfl_xor(bhi[c], off));
            }
        __syncthreads();                    // the previous tile is done with tbox
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                tbox[c] = blo[c];
                tbox[3 + c] = bhi[c];
            }
        float sp = 0, ep = 0, sx = 0, ex = 0, sy = 0, ey = 0, sz = 0, ez = 0;
        double npair = 0.0, nfar = 0.0;
        uint32_t nuse = 0;
        int hn = 0, nn = 0, hf = 0, nf = 0;     // head and fill of each ring (uniform)
        for (int eb = e0; eb < e1; eb += W) {
            const int nr = e1 - eb < W ? e1 - eb : W;
            __syncthreads();
            const int64_t total = load_ranges<W>(a, rb, eb, nr);
            npair += (double)total;
            for (int64_t c0 = 0; c0 < total; c0 += W) {
                const int cnt = (int)(total - c0 < W ? total - c0 : W);
                Src sr;
                double qx = 0.0, qy = 0.0, qz = 0.0;
                bool isfar = false;
                if (lane < cnt) {
                    sr = a.src[packed_node<W>(rb, nr, c0 + lane)];
                    qx = sr.yx - ox;
                    qy = sr.yy - oy;
                    qz = sr.yz - oz;
                    const double gx_ = fmax(fmax(tbox[0] - qx, qx - tbox[3]), 0.0);
                    const double gy_ = fmax(fmax(tbox[1] - qy, qy - tbox[4]), 0.0);
                    const double gz_ = fmax(fmax(tbox[2] - qz, qz - tbox[5]), 0.0);
                    isfar = (gx_ * gx_ + gy_ * gy_ + gz_ * gz_) * sr.s2 >= far_u;
                }
                const uint64_t fm = __ballot(isfar), nm = __ballot(lane < cnt && !isfar);
                __syncthreads();                // the runs taken last are read
                if (lane < cnt && !isfar) {
                    int pos = hn + nn + below(nm);
                    if (pos >= kRing) pos -= kRing;
                    SrcF f;
                    f.yx = (float)qx;
                    f.yy = (float)qy;
                    f.yz = (float)qz;
                    f.lx = (float)(qx - (double)f.yx);
                    f.ly = (float)(qy - (double)f.yy);
                    f.lz = (float)(qz - (double)f.yz);
                    f.s2 = (float)sr.s2;
                    f.ax = (float)(kFoldA * sr.ax);
                    f.ay = (float)(kFoldA * sr.ay);
                    f.az = (float)(kFoldA * sr.az);
                    f.s2x2 = (float)(kFoldT * sr.s2x2);
                    f.pad = 0.0f;
                    ring_n[pos] = f;
                } else if (isfar) {
                    int pos = hf + nf + below(fm);
                    if (pos >= kRing) pos -= kRing;
                    const double fa = kFoldA / (sr.s2 * sqrt(sr.s2));     // a'' (nodes32_far)
                    FarF f;
                    f.yx = (float)qx;
                    f.yy = (float)qy;
                    f.yz = (float)qz;
                    f.ax = (float)(fa * sr.ax);
                    f.ay = (float)(fa * sr.ay);
                    f.az = (float)(fa * sr.az);
                    f.pad0 = f.pad1 = 0.0f;
                    ring_f[pos] = f;
                }
                nn += __popcll(nm);
                nf += __popcll(fm);
                if (COUNT) nfar += (double)__popcll(fm);
                __syncthreads();
                for (; nn >= kRun; nn -= kRun) {
                    float p = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll 1
                    for (int j = 0; j < kRun; j += kNodeGroup)
                        nodes32<kNodeGroup, COUNT>(ring_n + hn + j, x, y, z, xl, yl, zl, p, gx, gy, gz, &nuse);
                    two_sum_f(sp, ep, p);
                    two_sum_f(sx, ex, gx);
                    two_sum_f(sy, ey, gy);
                    two_sum_f(sz, ez, gz);
                    hn = hn + kRun == kRing ? 0 : hn + kRun;
                }
                for (; nf >= kRun; nf -= kRun) {
                    float p = 0, gx = 0, gy = 0, gz = 0, hx = 0, hy = 0, hz = 0;
#pragma unroll 1
                    for (int j = 0; j < kRun; j += kNodeGroup)
                        nodes32_far<kNodeGroup>(ring_f + hf + j, x, y, z, p, gx, gy, gz, hx, hy, hz);
                    gx = fmaf(3.0f, gx, -hx);
                    gy = fmaf(3.0f, gy, -hy);
                    gz = fmaf(3.0f, gz, -hz);
                    two_sum_f(sp, ep, p);
                    two_sum_f(sx, ex, gx);
                    two_sum_f(sy, ey, gy);
                    two_sum_f(sz, ez, gz);
                    hf = hf + kRun == kRing ? 0 : hf + kRun;
                }
            }
        }
        if (nn > 0 || nf > 0) {             // remainders (< kRun each), padded to whole node groups
            const int pn = (nn + kNodeGroup - 1) / kNodeGroup * kNodeGroup;
            const int pf = (nf + kNodeGroup - 1) / kNodeGroup * kNodeGroup;
            __syncthreads();
            if (lane >= nn && lane < pn) ring_n[hn + lane] = pad_srcf();    // hn + kRun <= kRing
            if (lane >= nf && lane < pf) ring_f[hf + lane] = pad_farf();
            __syncthreads();
            if (nn > 0) {
                float p = 0, gx = 0, gy = 0, gz = 0;
                for (int j = 0; j < pn; j += kNodeGroup)
                    nodes32<kNodeGroup, COUNT>(ring_n + hn + j, x, y, z, xl, yl, zl, p, gx, gy, gz, &nuse);
                two_sum_f(sp, ep, p);
                two_sum_f(sx, ex, gx);
                two_sum_f(sy, ey, gy);
                two_sum_f(sz, ez, gz);
            }
            if (nf > 0) {
                float p = 0, gx = 0, gy = 0, gz = 0, hx = 0, hy = 0, hz = 0;
                for (int j = 0; j < pf; j += kNodeGroup)
                    nodes32_far<kNodeGroup>(ring_f + hf + j, x, y, z, p, gx, gy, gz, hx, hy, hz);
                gx = fmaf(3.0f, gx, -hx);
                gy = fmaf(3.0f, gy, -hy);
                gz = fmaf(3.0f, gz, -hz);
                two_sum_f(sp, ep, p);
                two_sum_f(sx, ex, gx);
                two_sum_f(sy, ey, gy);
                two_sum_f(sz, ez, gz);
            }
        }
        const double X = a.tx[ti], Y = a.ty[ti], Z = a.tz[ti];
        double ph = 0.0, g[3] = {0.0, 0.0, 0.0}, mph = 0.0, mg[3] = {0.0, 0.0, 0.0};
        if (a.m2p_end[B] > a.m2p_beg[B])    // uniform: Ls is the M2P staging buffer first
            fmm_m2p_list(a, B, Ls, X, Y, Z, mph, mg);
        __syncthreads();                    // the rings (or the M2P buffer) are done
        stage_local(a, B, Ls);
        __syncthreads();                    // Ls staged
        fmm_l2p(a, B, Ls, X, Y, Z, ph, g);
        ph += mph;
        g[0] += mg[0];
        g[1] += mg[1];
        g[2] += mg[2];
        if (valid) {
            const int64_t o = a.out_idx ? (int64_t)a.out_idx[ti] : ti;
            a.phi[o] = ((double)sp + (double)ep) + ph;
            if (a.grad) {
                a.grad[3 * o] = ((double)sx + (double)ex) + g[0];
                a.grad[3 * o + 1] = ((double)sy + (double)ey) + g[1];
                a.grad[3 * o + 2] = ((double)sz + (double)ez) + g[2];
            }
        }
        if (a.pairs) {                      // [0] pairs of real targets, [1] lane slots spent, [2] inside the cut,
                                            // [3] taken by the dipole-only loop
            const double w = wave_sum(valid ? npair : 0.0), wl = wave_sum(npair);
            const double wu = COUNT ? wave_sum(valid ? (double)nuse : 0.0) : 0.0;
            const double wf = COUNT ? wave_sum(valid ? nfar : 0.0) : 0.0;
            if (lane == 0) {
                atomicAdd(a.pairs, w);
                atomicAdd(a.pairs + 1, wl);
                if (COUNT) {
                    atomicAdd(a.pairs + 2, wu);
                    atomicAdd(a.pairs + 3, wf);
                }
            }
        }
        __syncthreads();                    // Ls is read before the next tile's rings overwrite it
    }
    queue_done(a);
}

template <int TILE>
void launch_tile(Ctx &c, int64_t n, const int32_t *n_dev, const double *tx, const double *ty, const double *tz,
                 const int32_t *tmesh, const int32_t *out_idx, double *phi, double *grad, double *pairs) {
    dim3 grid((unsigned)ceil_div(n, TILE)), block(TILE);
    if (c.opt.precision == LSS_MIXED)
        hipLaunchKernelGGL(k_p2p_direct_mixed<TILE>, grid, block, 0, c.stream, n, n_dev, tx, ty, tz, tmesh,
                           c.node_off.as<int64_t>(), c.src.as<Src>(), out_idx, phi, grad, pairs);
    else
        hipLaunchKernelGGL(k_p2p_direct_f64<TILE>, grid, block, 0, c.stream, n, n_dev, tx, ty, tz, tmesh,
                           c.node_off.as<int64_t>(), c.src.as<Src>(), out_idx, phi, grad, pairs);
    LSS_CHECK_LAUNCH("k_p2p_direct");
}

template <int TILE>
void launch_hess_tile(Ctx &c, unsigned grid, const FmmEvalArgs &a, double *hess) {
    const size_t shm = sizeof(double) * (size_t)a.ncp;
    hipLaunchKernelGGL(k_hess_fmm<TILE>, dim3(grid), dim3(TILE), shm, c.stream, a, hess);
    LSS_CHECK_LAUNCH("k_hess_fmm");
}

template <int TILE>
void launch_fmm_tile(Ctx &c, unsigned grid, const FmmEvalArgs &a) {
    if (TILE == 64) {
        const size_t shm = std::max(kF64RingBytes, sizeof(double) * (size_t)a.ncp);
        if (c.opt.count_useful)
            hipLaunchKernelGGL(k_eval_fmm_f64_split<true>, dim3(grid), dim3(64), shm, c.stream, a);
        else
            hipLaunchKernelGGL(k_eval_fmm_f64_split<false>, dim3(grid), dim3(64), shm, c.stream, a);
        LSS_CHECK_LAUNCH("k_eval_fmm_f64_split");
        return;
    }
    const size_t shm = sizeof(double) * (size_t)a.ncp;
    if (c.opt.count_useful)
        hipLaunchKernelGGL((k_eval_fmm_f64<TILE, true>), dim3(grid), dim3(TILE), shm, c.stream, a);
    else
        hipLaunchKernelGGL((k_eval_fmm_f64<TILE, false>), dim3(grid), dim3(TILE), shm, c.stream, a);
    LSS_CHECK_LAUNCH("k_eval_fmm");
}

}  // namespace

// FMM tiles: 0 = default 64 (narrow tiles keep the lanes of small leaves
// busy); the mixed kernel always takes 64-target tiles
int fmm_tile(const Ctx &c) {
    if (c.opt.precision == LSS_MIXED) return 64;
    if (c.opt.tile == 64 || c.opt.tile == 128 || c.opt.tile == 256) return c.opt.tile;
    return 64;
}

void launch_eval_fmm(Ctx &c, int64_t max_tiles, const int32_t *ntiles_dev, const int32_t *tile_start,
                     const int32_t *n_dev, int64_t n_max, const int32_t *sorted_leaf, const int32_t *sorted_idx,
                     const double *tx, const double *ty, const double *tz, const int32_t *out_idx, double *phi,
                     double *grad, const int32_t *order, double *pairs, double *hess, const MsArgs *ms) {
    const Tree &t = c.tree;
    FmmEvalArgs a;
    a.ntiles_dev = ntiles_dev;
    a.tile_start = tile_start;
    a.n_max = n_max;
    a.n_dev = n_dev;
    a.sleaf = sorted_leaf;
    a.sidx = sorted_idx;
    a.tx = tx; a.ty = ty; a.tz = tz;
    a.out_idx = out_idx;
    a.phi = phi;
    a.grad = grad;
    a.p2p_beg = t.p2p_beg.as<int32_t>();
    a.p2p_end = t.p2p_end.as<int32_t>();
    a.p2p_src = t.p2p_val2.as<int32_t>();
    a.nb = t.nb.as<int64_t>();
    a.ne = t.ne.as<int64_t>();
    a.lev = t.level.as<int32_t>();
    a.ijk = t.ijk.as<int32_t>();
    a.src = t.src.as<Src>();
    a.nnodes = c.nnodes;
    a.nboxes = (int32_t)t.nboxes;
    a.L = t.L.as<double>();
    a.M = t.M.as<double>();
    a.m2p_beg = t.m2p_beg.as<int32_t>();
    a.m2p_end = t.m2p_end.as<int32_t>();
    a.m2p_src = t.m2p_val2.as<int32_t>();
    a.p = t.p;
    a.ncp = t.ncp;
    a.root = t.root.as<double>();
    a.bmesh = t.bmesh.as<int32_t>();
    a.pairs = pairs;
    a.queue = c.tile_queue.as<unsigned int>();
    a.order = order;
    a.child = t.child.as<int32_t>();
    a.parent = t.parent.as<int32_t>();
    a.rmax = t.rmax.as<double>();
    a.K = t.K;
    {
        const double cut = c.opt.cut_factor > 0 ? c.opt.cut_factor
                                                 : (c.opt.precision == LSS_MIXED ? kCutMixed : kCutFP64);
        a.tcut = 0.5 * cut * cut;
    }
    int64_t g = max_tiles < 16384 ? max_tiles : 16384;
    unsigned grid = (unsigned)(g > 0 ? g : 1);
    if (ms) {                               // target-attached width (FP64)
        const size_t shm = sizeof(double) * (size_t)a.ncp;
        switch (fmm_tile(c)) {
            case 64: hipLaunchKernelGGL(k_multiscale_fmm<64>, dim3(grid), dim3(64), shm, c.stream, a, *ms); break;
            case 128: hipLaunchKernelGGL(k_multiscale_fmm<128>, dim3(grid), dim3(128), shm, c.stream, a, *ms); break;
            default: hipLaunchKernelGGL(k_multiscale_fmm<256>, dim3(grid), dim3(256), shm, c.stream, a, *ms); break;
        }
        LSS_CHECK_LAUNCH("k_multiscale_fmm");
        const int64_t go = ceil_div(n_max > 0 ? n_max : 1, 256);
        hipLaunchKernelGGL(k_multiscale_outside, dim3((unsigned)(go < 1024 ? go : 1024)), dim3(256), 0, c.stream, a,
                           *ms);
        LSS_CHECK_LAUNCH("k_multiscale_outside");
        return;
    }
    if (hess) {                             // Phi, grad Phi and the Hessian (FP64)
        switch (fmm_tile(c)) {
            case 64: launch_hess_tile<64>(c, grid, a, hess); break;
            case 128: launch_hess_tile<128>(c, grid, a, hess); break;
            default: launch_hess_tile<256>(c, grid, a, hess); break;
        }
        const int64_t go = ceil_div(n_max > 0 ? n_max : 1, 256);
        hipLaunchKernelGGL(k_hess_outside, dim3((unsigned)(go < 1024 ? go : 1024)), dim3(256), 0, c.stream, a, hess);
        LSS_CHECK_LAUNCH("k_hess_outside");
        return;
    }
    if (c.opt.precision == LSS_MIXED) {
        const size_t shm = std::max(kMixedRingBytes, sizeof(double) * (size_t)a.ncp);
        if (c.opt.count_useful)
            hipLaunchKernelGGL(k_eval_fmm_mixed<true>, dim3(grid), dim3(64), shm, c.stream, a);
        else
            hipLaunchKernelGGL(k_eval_fmm_mixed<false>, dim3(grid), dim3(64), shm, c.stream, a);
        LSS_CHECK_LAUNCH("k_eval_fmm_mixed");
    } else {
        switch (fmm_tile(c)) {
            case 64: launch_fmm_tile<64>(c, grid, a); break;
            case 128: launch_fmm_tile<128>(c, grid, a); break;
            default: launch_fmm_tile<256>(c, grid, a); break;
        }
    }
    const int64_t go = ceil_div(n_max > 0 ? n_max : 1, 256);
    hipLaunchKernelGGL(k_eval_outside, dim3((unsigned)(go < 1024 ? go : 1024)), dim3(256), 0, c.stream, a);
    LSS_CHECK_LAUNCH("k_eval_outside");
}

void launch_p2p_direct(Ctx &c, int64_t n, const int32_t *n_dev, const double *tx, const double *ty,
                       const double *tz, const int32_t *tmesh, const int32_t *out_idx, double *phi,
                       double *grad, int /*grad_stride*/, double *pairs) {
    if (n <= 0) return;
    switch (c.opt.tile) {
        case 64: launch_tile<64>(c, n, n_dev, tx, ty, tz, tmesh, out_idx, phi, grad, pairs); break;
        case 128: launch_tile<128>(c, n, n_dev, tx, ty, tz, tmesh, out_idx, phi, grad, pairs); break;
        default: launch_tile<256>(c, n, n_dev, tx, ty, tz, tmesh, out_idx, phi, grad, pairs); break;
    }
}

}  // namespace lss
