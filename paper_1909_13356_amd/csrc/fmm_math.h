// Solid harmonics and translation operators of the Laplace fast multipole
// method used for the far field of the smoothed-indicator sum (section 4.4,
// eq. kerdecomp: beyond the cut the kernel is the Laplace double layer, whose
// sum the FMM evaluates).  Host + device, header only.
//
// Conventions (complex, m = -n..n):
//   regular   U_n^m(r):  U_0^0 = 1,  U_m^m = -(x+iy)/(2m) U_{m-1}^{m-1},
//                        U_n^m = ((2n-1) z U_{n-1}^m - r^2 U_{n-2}^m) / ((n+m)(n-m))
//   irregular T_n^m(r):  T_0^0 = 1/r, T_m^m = -(2m-1)(x+iy)/r^2 T_{m-1}^{m-1},
//                        T_n^m = ((2n-1) z T_{n-1}^m - (n-1+m)(n-1-m) T_{n-2}^m) / r^2
//   U_n^{-m} = (-1)^m conj(U_n^m), same for T.  With these
//     1/|x-y|        = sum conj(U_n^m(y)) T_n^m(x)                 (|y| < |x|)
//     U_n^m(a+b)     = sum_{k,l} U_k^l(a) U_{n-k}^{m-l}(b)
//     T_n^m(x-y)     = sum_{k,l} conj(U_k^l(y)) T_{n+k}^{m+l}(x)   (|y| < |x|)
//     dz U_n^m = U_{n-1}^m,  (dx+i dy) U_n^m = U_{n-1}^{m+1},  (dx-i dy) U_n^m = -U_{n-1}^{m-1}.
//
// Expansions of a box of side s, centre c, are stored scaled, real layout:
//   multipole  M~_n^m = M_n^m / s^n,   Phi(x) = sum M_n^m T_n^m(x - c)
//   local      L~_k^l = L_k^l s^k,     Phi(x) = sum L_k^l U_k^l(x - c)
// Real layout of coefficient (n, m >= 0): Re at n^2 (m = 0) or n^2 + 2m - 1,
// Im at n^2 + 2m; (p+1)^2 reals per expansion.  The m < 0 half follows from
// the symmetry of a real potential, M_n^{-m} = (-1)^m conj(M_n^m).
//
// Translations in scaled form are level independent:
//   M2M (child c -> parent):  M~_n^m(P) = sum 2^{-n} conj(U_{n-k}^{m-l}(w)) M~_k^l(c)
//   M2L (source S -> target T, same side s, v = (c_T - c_S)/s):
//                             L~_k^l(T) = (1/s) (-1)^{k+l} sum T_{n+k}^{m-l}(v) M~_n^m(S)
//   L2L (parent -> child):    L~_j^q(c) = sum 2^{-k} U_{k-j}^{l-q}(w) L~_k^l(P)
// with w = (c_child - c_parent)/s_child in {-1/2, 1/2}^3.
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define LSS_HD __host__ __device__ inline
#else
#define LSS_HD inline
#endif

namespace lss {
namespace fmm {

LSS_HD int ncoef(int p) { return (p + 1) * (p + 1); }
LSS_HD int ire(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
LSS_HD int iim(int n, int m) { return n * n + 2 * m; }
LSS_HD int tri(int n, int m) { return n * (n + 1) / 2 + m; }   // triangular table index, m >= 0

struct cd {
    double re, im;
};
LSS_HD cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
LSS_HD cd cconj(cd a) { return {a.re, -a.im}; }
LSS_HD cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
LSS_HD cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
LSS_HD cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }

// U_n^m (m >= 0, n <= p) into a triangular table
LSS_HD void regular_table(double x, double y, double z, int p, cd *U) {
    const double r2 = x * x + y * y + z * z;
    cd diag = {1.0, 0.0};
    for (int m = 0; m <= p; ++m) {
        if (m > 0) diag = cscale(cmul(diag, cd{x, y}), -1.0 / (2.0 * m));
        U[tri(m, m)] = diag;
        cd um2 = {0.0, 0.0}, um1 = diag;
        for (int n = m + 1; n <= p; ++n) {
            const double inv = 1.0 / ((double)(n + m) * (double)(n - m));
            cd un = {((2 * n - 1) * z * um1.re - r2 * um2.re) * inv, ((2 * n - 1) * z * um1.im - r2 * um2.im) * inv};
            U[tri(n, m)] = un;
            um2 = um1;
            um1 = un;
        }
    }
}

// T_n^m (m >= 0, n <= p) into a triangular table (r > 0)
LSS_HD void irregular_table(double x, double y, double z, int p, cd *T) {
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    cd diag = {sqrt(ir2), 0.0};
    for (int m = 0; m <= p; ++m) {
        if (m > 0) diag = cscale(cmul(diag, cd{x, y}), -(2.0 * m - 1.0) * ir2);
        T[tri(m, m)] = diag;
        cd tm2 = {0.0, 0.0}, tm1 = diag;
        for (int n = m + 1; n <= p; ++n) {
            const double a = (2 * n - 1) * z, b = (double)(n - 1 + m) * (double)(n - 1 - m);
            cd tn = {(a * tm1.re - b * tm2.re) * ir2, (a * tm1.im - b * tm2.im) * ir2};
            T[tri(n, m)] = tn;
            tm2 = tm1;
            tm1 = tn;
        }
    }
}

// table access with any m in [-n, n] (0 outside)
LSS_HD cd tget(const cd *tab, int n, int m) {
    if (n < 0 || m > n || m < -n) return cd{0.0, 0.0};
    if (m >= 0) return tab[tri(n, m)];
    cd v = cconj(tab[tri(n, -m)]);
    return (m & 1) ? cscale(v, -1.0) : v;
}

// Real-basis entry of a complex coefficient map L_k^l = sum_{n,m} A(k,l,n,m) M_n^m
// acting on the real layouts: output row (k, l>=0, Re/Im), input column (n, m>=0, Re/Im).
template <class F>
LSS_HD double folded_entry(const F &A, int k, int l, bool out_im, int n, int m, bool in_im) {
    cd c;
    if (m == 0) {
        if (in_im) return 0.0;
        c = A(k, l, n, 0);
    } else {
        cd ap = A(k, l, n, m), am = A(k, l, n, -m);
        if (m & 1) am = cscale(am, -1.0);
        if (!in_im) c = cadd(ap, am);
        else {
            cd d = csub(ap, am);
            c = cd{-d.im, d.re};   // i * d
        }
    }
    return out_im ? c.im : c.re;
}

// decode a real-layout index into (n, m, is_im)
LSS_HD void decode(int idx, int &n, int &m, bool &im) {
    n = (int)sqrt((double)idx);
    while (n * n > idx) --n;
    while ((n + 1) * (n + 1) <= idx) ++n;
    int r = idx - n * n;
    if (r == 0) { m = 0; im = false; }
    else { m = (r + 1) / 2; im = (r % 2) == 0; }
}

// operator entry functors --------------------------------------------------
struct M2LMap {           // A(k,l,n,m) = (-1)^{k+l} T_{n+k}^{m-l}(v)   (table up to 2p)
    const cd *Tv;
    LSS_HD cd operator()(int k, int l, int n, int m) const {
        cd t = tget(Tv, n + k, m - l);
        return ((k + l) & 1) ? cscale(t, -1.0) : t;
    }
};
struct M2MMap {           // A(n,m,k,l) = 2^{-n} conj(U_{n-k}^{m-l}(w))
    const cd *Uw;
    LSS_HD cd operator()(int n, int m, int k, int l) const {
        if (k > n) return cd{0.0, 0.0};
        cd u = cconj(tget(Uw, n - k, m - l));
        return cscale(u, ldexp(1.0, -n));
    }
};
struct L2LMap {           // A(j,q,k,l) = 2^{-k} U_{k-j}^{l-q}(w)
    const cd *Uw;
    LSS_HD cd operator()(int j, int q, int k, int l) const {
        if (k < j) return cd{0.0, 0.0};
        return cscale(tget(Uw, k - j, l - q), ldexp(1.0, -k));
    }
};

// P2M of one dipole a at scaled position rt (relative to the box centre, in
// units of the box side s): adds to M~ (real layout) the coefficients of
// -(a . grad_y) 1/(4 pi |x - y|).  U is a scratch table of tri(p, p)+1 entries.
LSS_HD void p2m_dipole(double rx, double ry, double rz, double ax, double ay, double az, double inv4pis, int p,
                       cd *U, double *M) {
    regular_table(rx, ry, rz, p, U);
    for (int n = 1; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            cd up = tget(U, n - 1, m + 1), dn = tget(U, n - 1, m - 1), zz = tget(U, n - 1, m);
            // (a . grad) U_n^m = 1/2 (ax - i ay) U^{m+1} - 1/2 (ax + i ay) U^{m-1} + az U^m
            cd t = cadd(cadd(cmul(cd{0.5 * ax, -0.5 * ay}, up), cmul(cd{-0.5 * ax, -0.5 * ay}, dn)), cscale(zz, az));
            t = cscale(cconj(t), -inv4pis);
            M[ire(n, m)] += t.re;
            if (m > 0) M[iim(n, m)] += t.im;
        }
}

// L2P: Phi and grad Phi of a local expansion at scaled position (rx,ry,rz)
// (in units of the box side s); grad is returned in physical units (divided by s).
// L is the real layout (any memory; on the device the caller stages it in LDS).
//   Phi          = sum_{j, m>=0} w_m Re(L_j^m U_j^m)                  (w_0 = 1, w_m = 2)
//   dPhi/dz      = sum_{j, m>=0} w_m Re(L_{j+1}^m U_j^m)
//   (dx + i dy)Phi = sum_{j, s} L_{j+1}^{s-1} U_j^s
//                 = sum_{j, m>=0} L_{j+1}^{m-1} U_j^m - [m > 0] conj(L_{j+1}^{m+1} U_j^m)
LSS_HD void l2p(const double *L, double rx, double ry, double rz, double inv_s, int p, double &phi, double g[3]) {
    const double r2 = rx * rx + ry * ry + rz * rz;
    double ph = 0.0, gz = 0.0, Are = 0.0, Aim = 0.0;
    cd diag = {1.0, 0.0};
    for (int m = 0; m <= p; ++m) {
        if (m > 0) diag = cscale(cmul(diag, cd{rx, ry}), -0.5 / (double)m);
        const double w = m == 0 ? 1.0 : 2.0;
        cd um2 = {0.0, 0.0}, u = diag;
        for (int j = m; j <= p; ++j) {
            if (j > m) {
                const double den = (double)((j + m) * (j - m));
                const double inv = 1.0 / den;
                cd un = {((2 * j - 1) * rz * u.re - r2 * um2.re) * inv, ((2 * j - 1) * rz * u.im - r2 * um2.im) * inv};
                um2 = u;
                u = un;
            }
            const double Lre = L[ire(j, m)], Lim = m ? L[iim(j, m)] : 0.0;
            ph += w * (Lre * u.re - Lim * u.im);
            if (j < p) {
                const int j1 = j + 1;
                const double zre = L[ire(j1, m)], zim = m ? L[iim(j1, m)] : 0.0;
                gz += w * (zre * u.re - zim * u.im);
                double are, aim;                       // L_{j+1}^{m-1}; L^{-1} = -conj(L^1)
                if (m >= 1) { are = L[ire(j1, m - 1)]; aim = (m - 1) ? L[iim(j1, m - 1)] : 0.0; }
                else { are = -L[ire(j1, 1)]; aim = L[iim(j1, 1)]; }
                Are += are * u.re - aim * u.im;
                Aim += are * u.im + aim * u.re;
                if (m > 0) {                           // - conj(L_{j+1}^{m+1} U_j^m)
                    const double bre = L[ire(j1, m + 1)], bim = L[iim(j1, m + 1)];
                    Are -= bre * u.re - bim * u.im;
                    Aim += bre * u.im + bim * u.re;
                }
            }
        }
    }
    phi = ph;
    g[0] = Are * inv_s;
    g[1] = Aim * inv_s;
    g[2] = gz * inv_s;
}

// M2P: Phi and grad Phi of a multipole expansion M~ (real layout) of a box of
// side s, centre c, at the scaled position (rx,ry,rz) = (x - c)/s, outside the
// sphere around the box.  It is the degree-0 and degree-1 part of the M2L of M~
// to a box of side s centred at x (see M2L above), so
//   Phi            = (1/s)   sum_{n,m} T_n^m(r) M~_n^m
//   dPhi/dz        = -(1/s^2) sum_{n,m} T_{n+1}^m(r) M~_n^m
//   (dx + i dy)Phi = -(1/s^2) conj(A),  A = sum_{n,m} T_{n+1}^{m-1}(r) M~_n^m.
// The m < 0 halves fold as in l2p: T_{n+1}^{-m} M_n^{-m} = conj(T_{n+1}^m M_n^m),
// and in A the terms of M_n^{m'} with m' <= 0 are -conj(T_{n+1}^{|m'|+1} M_n^{|m'|}).
// T_j^m is generated column by column (m = 0..p+1, j = m..p+1) and consumed at
// once, as T_j^m M_j^m, T_j^m M_{j-1}^m, T_j^m M_{j-1}^{m+1} and -conj(T_j^m M_{j-1}^{m-1}).
LSS_HD void m2p(const double *M, double rx, double ry, double rz, double inv_s, int p, double &phi, double g[3]) {
    const double r2 = rx * rx + ry * ry + rz * rz, ir2 = 1.0 / r2;
    double s0 = 0.0, s1 = 0.0, Are = 0.0, Aim = 0.0;
    cd diag = {sqrt(ir2), 0.0};
    for (int m = 0; m <= p + 1; ++m) {
        if (m > 0) diag = cscale(cmul(diag, cd{rx, ry}), -(2.0 * m - 1.0) * ir2);
        const double w = m == 0 ? 1.0 : 2.0;
        cd tm2 = {0.0, 0.0}, t = diag;
        for (int j = m; j <= p + 1; ++j) {
            if (j > m) {
                const double a = (2 * j - 1) * rz, b = (double)(j - 1 + m) * (double)(j - 1 - m);
                cd tn = {(a * t.re - b * tm2.re) * ir2, (a * t.im - b * tm2.im) * ir2};
                tm2 = t;
                t = tn;
            }
            if (j <= p) {                              // T_j^m M_j^m
                const double mre = M[ire(j, m)], mim = m ? M[iim(j, m)] : 0.0;
                s0 += w * (t.re * mre - t.im * mim);
            }
            if (j == 0) continue;
            const int n = j - 1;
            if (m <= n) {                              // T_{n+1}^m M_n^m
                const double mre = M[ire(n, m)], mim = m ? M[iim(n, m)] : 0.0;
                s1 += w * (t.re * mre - t.im * mim);
            }
            if (m + 1 <= n) {                          // T_{n+1}^m M_n^{m+1}
                const double mre = M[ire(n, m + 1)], mim = M[iim(n, m + 1)];
                Are += t.re * mre - t.im * mim;
                Aim += t.re * mim + t.im * mre;
            }
            if (m >= 1) {                              // -conj(T_{n+1}^m M_n^{m-1})
                const double mre = M[ire(n, m - 1)], mim = (m - 1) ? M[iim(n, m - 1)] : 0.0;
                Are -= t.re * mre - t.im * mim;
                Aim += t.re * mim + t.im * mre;
            }
        }
    }
    const double is2 = inv_s * inv_s;
    phi = s0 * inv_s;
    g[0] = -Are * is2;
    g[1] = Aim * is2;
    g[2] = -s1 * is2;
}

// Real-layout coefficient (n, m) as a complex number for any m in [-n, n]
// (0 outside), by the symmetry of a real potential C_n^{-m} = (-1)^m conj(C_n^m).
LSS_HD cd coef(const double *C, int n, int m) {
    if (n < 0 || m > n || m < -n) return cd{0.0, 0.0};
    const int a = m < 0 ? -m : m;
    cd v = {C[ire(n, a)], a ? C[iim(n, a)] : 0.0};
    if (m < 0) {
        v = cconj(v);
        if (a & 1) v = cscale(v, -1.0);
    }
    return v;
}

// Hessian H = (xx, xy, xz, yy, yz, zz) of a harmonic field from three
// complex second derivatives: Z = d2/dz2, W = dz (dx + i dy), P = (dx + i dy)^2
// (P = Hxx - Hyy + 2i Hxy, W = Hxz + i Hyz, Hxx + Hyy = -Hzz).
LSS_HD void hess_from(double Z, cd W, cd P, double H[6]) {
    H[5] = Z;
    H[2] = W.re;
    H[4] = W.im;
    H[1] = 0.5 * P.im;
    H[0] = 0.5 * (P.re - Z);
    H[3] = 0.5 * (-P.re - Z);
}

// L2P Hessian: second derivatives of the local expansion (scaled L~, box side
// s) at the scaled position r.  From dz U_n^m = U_{n-1}^m and (dx + i dy) U_n^m
// = U_{n-1}^{m+1}:
//   d2/dz2 Phi        = s^-2 sum_{j,s} L~_{j+2}^s     U_j^s(r)
//   dz (dx + i dy)Phi = s^-2 sum_{j,s} L~_{j+2}^{s-1} U_j^s(r)
//   (dx + i dy)^2 Phi = s^-2 sum_{j,s} L~_{j+2}^{s-2} U_j^s(r)
// with U_j^s generated column by column (s >= 0) and U_j^{-s} = (-1)^s conj(U_j^s).
LSS_HD void l2p_hess(const double *L, double rx, double ry, double rz, double inv_s, int p, double H[6]) {
    const double r2 = rx * rx + ry * ry + rz * rz;
    cd Z = {0.0, 0.0}, W = {0.0, 0.0}, P = {0.0, 0.0};
    cd diag = {1.0, 0.0};
    for (int m = 0; m + 2 <= p; ++m) {
        if (m > 0) diag = cscale(cmul(diag, cd{rx, ry}), -0.5 / (double)m);
        cd um2 = {0.0, 0.0}, u = diag;
        for (int j = m; j + 2 <= p; ++j) {
            if (j > m) {
                const double inv = 1.0 / ((double)(j + m) * (double)(j - m));
                cd un = {((2 * j - 1) * rz * u.re - r2 * um2.re) * inv, ((2 * j - 1) * rz * u.im - r2 * um2.im) * inv};
                um2 = u;
                u = un;
            }
            Z = cadd(Z, cmul(coef(L, j + 2, m), u));
            W = cadd(W, cmul(coef(L, j + 2, m - 1), u));
            P = cadd(P, cmul(coef(L, j + 2, m - 2), u));
            if (m > 0) {
                cd un = cconj(u);
                if (m & 1) un = cscale(un, -1.0);           // U_j^{-m}
                Z = cadd(Z, cmul(coef(L, j + 2, -m), un));
                W = cadd(W, cmul(coef(L, j + 2, -m - 1), un));
                P = cadd(P, cmul(coef(L, j + 2, -m - 2), un));
            }
        }
    }
    const double is2 = inv_s * inv_s;
    hess_from(Z.re * is2, cscale(W, is2), cscale(P, is2), H);
}

// M2P Hessian: second derivatives of a multipole expansion (scaled M~, box
// side s) at the scaled position r outside the box's sphere.  From
// dz T_n^m = -T_{n+1}^m and (dx - i dy) T_n^m = -T_{n+1}^{m-1} (unit side):
//   d2/dz2 Phi        = s^-3 sum_{n,m} T_{n+2}^m     M~_n^m
//   dz (dx - i dy)Phi = s^-3 sum_{n,m} T_{n+2}^{m-1} M~_n^m
//   (dx - i dy)^2 Phi = s^-3 sum_{n,m} T_{n+2}^{m-2} M~_n^m
// and, Phi being real, the (dx + i dy) forms are their conjugates.  T_j^mu is
// generated column by column (mu >= 0, j = mu..p+2) with T_j^{-mu} =
// (-1)^mu conj(T_j^mu); the term T_j^mu pairs with M~_{j-2}^{mu+q}, q = 0, 1, 2.
LSS_HD void m2p_hess(const double *M, double rx, double ry, double rz, double inv_s, int p, double H[6]) {
    const double r2 = rx * rx + ry * ry + rz * rz, ir2 = 1.0 / r2;
    cd Z = {0.0, 0.0}, W = {0.0, 0.0}, P = {0.0, 0.0};
    cd diag = {sqrt(ir2), 0.0};
    for (int mu = 0; mu <= p + 2; ++mu) {
        if (mu > 0) diag = cscale(cmul(diag, cd{rx, ry}), -(2.0 * mu - 1.0) * ir2);
        cd tm2 = {0.0, 0.0}, t = diag;
        for (int j = mu; j <= p + 2; ++j) {
            if (j > mu) {
                const double a = (2 * j - 1) * rz, b = (double)(j - 1 + mu) * (double)(j - 1 - mu);
                cd tn = {(a * t.re - b * tm2.re) * ir2, (a * t.im - b * tm2.im) * ir2};
                tm2 = t;
                t = tn;
            }
            if (j < 2) continue;
            const int n = j - 2;
            Z = cadd(Z, cmul(t, coef(M, n, mu)));
            W = cadd(W, cmul(t, coef(M, n, mu + 1)));
            P = cadd(P, cmul(t, coef(M, n, mu + 2)));
            if (mu > 0) {
                cd tn = cconj(t);
                if (mu & 1) tn = cscale(tn, -1.0);          // T_j^{-mu}
                Z = cadd(Z, cmul(tn, coef(M, n, -mu)));
                W = cadd(W, cmul(tn, coef(M, n, -mu + 1)));
                P = cadd(P, cmul(tn, coef(M, n, -mu + 2)));
            }
        }
    }
    const double is3 = inv_s * inv_s * inv_s;
    hess_from(Z.re * is3, cconj(cscale(W, is3)), cconj(cscale(P, is3)), H);
}

}  // namespace fmm
}  // namespace lss
