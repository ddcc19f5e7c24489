"""Host-side check of the M2P evaluation of the far-field code (the
header is host+device): the multipole series of point charges in a box,
evaluated at points outside it, against the direct sum."""

import os
import subprocess
import textwrap

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1909_13356_amd", "csrc")

PROG = textwrap.dedent(r"""
    #include <cmath>
    #include <cstdio>
    #include <cstdlib>
    #include <vector>
    #include "fmm_math.h"
    using namespace lss::fmm;
    // point charges q_k at y_k inside a box of side s (centre c): M~_n^m = sum q conj(U_n^m(y/s));
    // the M2P series at |x - c| >= rmin s against sum q / |x - y| and its gradient
    int main(int argc, char **argv) {
        const int p = atoi(argv[1]);
        const double rmin = atof(argv[2]);
        srand(7);
        auto rnd = [] { return rand() / (double)RAND_MAX - 0.5; };
        double worst = 0.0;
        for (int trial = 0; trial < 300; ++trial) {
            const double s = 0.37, c[3] = {0.1, -0.2, 0.3};
            std::vector<double> M(ncoef(p), 0.0);
            std::vector<cd> U(tri(p, p) + 1);
            double y[6][3], q[6], aq = 0.0;
            for (int k = 0; k < 6; ++k) {
                for (int d = 0; d < 3; ++d) y[k][d] = rnd() * s;
                q[k] = rnd();
                aq += fabs(q[k]);
                regular_table(y[k][0] / s, y[k][1] / s, y[k][2] / s, p, U.data());
                for (int n = 0; n <= p; ++n)
                    for (int m = 0; m <= n; ++m) {
                        M[ire(n, m)] += q[k] * U[tri(n, m)].re;
                        if (m) M[iim(n, m)] -= q[k] * U[tri(n, m)].im;
                    }
            }
            double dir[3] = {rnd(), rnd(), rnd()};
            const double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
            const double R = s * (rmin + 0.2 * (rnd() + 0.5));
            double x[3], ph, g[3], eph = 0.0, eg[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < 3; ++d) x[d] = c[d] + R * dir[d] / nd;
            m2p(M.data(), (x[0] - c[0]) / s, (x[1] - c[1]) / s, (x[2] - c[2]) / s, 1.0 / s, p, ph, g);
            for (int k = 0; k < 6; ++k) {
                const double d0 = x[0] - c[0] - y[k][0], d1 = x[1] - c[1] - y[k][1], d2 = x[2] - c[2] - y[k][2];
                const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2), r3 = r * r * r;
                eph += q[k] / r;
                eg[0] -= q[k] * d0 / r3; eg[1] -= q[k] * d1 / r3; eg[2] -= q[k] * d2 / r3;
            }
            worst = fmax(worst, fabs(ph - eph) / (aq / R));
            for (int d = 0; d < 3; ++d) worst = fmax(worst, fabs(g[d] - eg[d]) / (aq / (R * R)));
        }
        printf("%.6e\n", worst);
        return 0;
    }
""")


@pytest.fixture(scope="module")
def m2p_prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("m2p")
    src = d / "m2p.cpp"
    src.write_text(PROG)
    exe = d / "m2p"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)])
    return str(exe)


# (order, smallest distance in box sides, bound): the orders and separations of
# the two precisions' M2P lists (K = 4 mixed at p = 20, K = 7 FP64 at p = 26)
# and a low order that shows the series converging
@pytest.mark.parametrize("p,rmin,bound", [(20, 2.0, 1e-7), (26, 2.64, 1e-13), (8, 2.0, 1e-2)])
def test_m2p_series_matches_direct_sum(m2p_prog, p, rmin, bound):
    err = float(subprocess.check_output([m2p_prog, str(p), str(rmin)]).decode())
    assert err <= bound
    if p == 8:
        assert err > 1e-6                     # truncation visible: the high orders do matter


HESS_PROG = textwrap.dedent(r"""
    #include <cmath>
    #include <cstdio>
    #include <cstdlib>
    #include <vector>
    #include "fmm_math.h"
    using namespace lss::fmm;
    // Hessians of the M2P and L2P series of point charges against the direct
    // Hessian of sum q / |x - y|: d2/dxi dxj 1/|d| = (3 d_i d_j - delta_ij |d|^2) / |d|^5.
    static void direct(const double x[3], double y[][3], const double *q, int nq, double H[6]) {
        const int I[6] = {0, 0, 0, 1, 1, 2}, J[6] = {0, 1, 2, 1, 2, 2};
        for (int k = 0; k < 6; ++k) H[k] = 0.0;
        for (int e = 0; e < nq; ++e) {
            const double d[3] = {x[0] - y[e][0], x[1] - y[e][1], x[2] - y[e][2]};
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], r5 = r2 * r2 * sqrt(r2);
            for (int k = 0; k < 6; ++k) H[k] += q[e] * (3 * d[I[k]] * d[J[k]] - (I[k] == J[k] ? r2 : 0.0)) / r5;
        }
    }
    int main(int argc, char **argv) {
        const int p = atoi(argv[1]);
        const double rmin = atof(argv[2]);
        srand(11);
        auto rnd = [] { return rand() / (double)RAND_MAX - 0.5; };
        double worst_m = 0.0, worst_l = 0.0;
        for (int trial = 0; trial < 200; ++trial) {
            const double s = 0.37, c[3] = {0.1, -0.2, 0.3};
            double y[6][3], q[6], aq = 0.0;
            for (int k = 0; k < 6; ++k) q[k] = rnd(), aq += fabs(q[k]);
            double dir[3] = {rnd(), rnd(), rnd()};
            const double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
            const double R = s * (rmin + 0.2 * (rnd() + 0.5));
            // M2P: charges in the box, target at distance R
            {
                std::vector<double> M(ncoef(p), 0.0);
                std::vector<cd> U(tri(p, p) + 1);
                for (int k = 0; k < 6; ++k) {
                    for (int d = 0; d < 3; ++d) y[k][d] = c[d] + rnd() * s;
                    regular_table((y[k][0] - c[0]) / s, (y[k][1] - c[1]) / s, (y[k][2] - c[2]) / s, p, U.data());
                    for (int n = 0; n <= p; ++n)
                        for (int m = 0; m <= n; ++m) {
                            M[ire(n, m)] += q[k] * U[tri(n, m)].re;
                            if (m) M[iim(n, m)] -= q[k] * U[tri(n, m)].im;
                        }
                }
                double x[3], H[6], E[6];
                for (int d = 0; d < 3; ++d) x[d] = c[d] + R * dir[d] / nd;
                m2p_hess(M.data(), (x[0] - c[0]) / s, (x[1] - c[1]) / s, (x[2] - c[2]) / s, 1.0 / s, p, H);
                direct(x, y, q, 6, E);
                for (int k = 0; k < 6; ++k) worst_m = fmax(worst_m, fabs(H[k] - E[k]) / (aq / (R * R * R)));
            }
            // L2P: charges at distance R, target in the box; L~_n^m = s^n sum q conj(T_n^m(y - c))
            {
                std::vector<double> L(ncoef(p), 0.0);
                std::vector<cd> T(tri(p, p) + 1);
                for (int k = 0; k < 6; ++k) {
                    const double R2 = s * (rmin + 0.2 * (rnd() + 0.5));
                    double e[3] = {rnd(), rnd(), rnd()};
                    const double ne = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                    for (int d = 0; d < 3; ++d) y[k][d] = c[d] + R2 * e[d] / ne;
                    irregular_table(y[k][0] - c[0], y[k][1] - c[1], y[k][2] - c[2], p, T.data());
                    double sn = 1.0;
                    for (int n = 0; n <= p; ++n, sn *= s)
                        for (int m = 0; m <= n; ++m) {
                            L[ire(n, m)] += q[k] * sn * T[tri(n, m)].re;
                            if (m) L[iim(n, m)] -= q[k] * sn * T[tri(n, m)].im;
                        }
                }
                double x[3], H[6], E[6];
                for (int d = 0; d < 3; ++d) x[d] = c[d] + 0.5 * s * rnd();
                l2p_hess(L.data(), (x[0] - c[0]) / s, (x[1] - c[1]) / s, (x[2] - c[2]) / s, 1.0 / s, p, H);
                direct(x, y, q, 6, E);
                const double Rmin = s * rmin;
                for (int k = 0; k < 6; ++k) worst_l = fmax(worst_l, fabs(H[k] - E[k]) / (aq / (Rmin * Rmin * Rmin)));
            }
        }
        printf("%.6e %.6e\n", worst_m, worst_l);
        return 0;
    }
""")


@pytest.fixture(scope="module")
def hess_prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("hess")
    src = d / "hess.cpp"
    src.write_text(HESS_PROG)
    exe = d / "hess"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)])
    return str(exe)


# M2P and L2P Hessians against the direct Hessian of the charges (relative to
# sum |q| / R^3) at the separations of the two precisions' lists, and at a low
# order where the truncation shows
@pytest.mark.parametrize("p,rmin,bound", [(20, 2.0, 3e-6), (26, 2.83, 2e-12), (8, 2.0, 1.0)])
def test_m2p_l2p_hessian_match_direct_sum(hess_prog, p, rmin, bound):
    em, el = (float(v) for v in subprocess.check_output([hess_prog, str(p), str(rmin)]).decode().split())
    assert em <= bound and el <= bound
    if p == 8:
        assert max(em, el) > 1e-6
