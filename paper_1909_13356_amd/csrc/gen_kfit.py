"""Generate kfit_tables.h: rational approximations of the two radial functions
of the smoothed-indicator kernel, for the HIP pair kernels.

With u = rho / (sqrt(2) sigma) and x = u^2 the near-field kernel (section 4.1,
eq. kerpsi) and its exact gradient need

    S(x) = gamma(3/2, x) / x^(3/2)       (S(0) = 2/3)
    T(x) = gamma(5/2, x) / x^(5/2)       (T(0) = 2/5)

(lower incomplete gamma).  Both are entire in x, so on a bounded interval
[0, X] they are approximated well by rationals.  One common denominator is
fitted for the pair,

    S ~ P_S(t) / Q(t),   T ~ P_T(t) / Q(t),   t = x / X,

by linearised least squares (Sanathanan-Koerner iteration) followed by
Lawson re-weighting towards the minimax relative error, at 50 digits with
mpmath.  Beyond X the kernel is the Laplace dipole to the tail bound of the
cut (section 4.4, the 8 sigma bounds), so the kernels switch to
S = (sqrt(pi)/2) x^(-3/2), T = 1.5 S / x there.

Three fits are produced:
  * FP64: X = 32 (cut at 8 sigma), degree (13, 13) (fit error 7e-15; degree
    12 reaches only 1.7e-13, degree 15 7e-18);
  * FP32: X = 20 (cut at sqrt(40) sigma = 6.32 sigma), degree (7, 7);
  * FP64 for the Hessian: S, T and U(x) = gamma(7/2, x) / x^(7/2) (U(0) = 2/7)
    over one denominator, X = 32, degree (14, 14), not folded (fit error
    9e-16; degree 13 reaches 3.1e-14).

The pair kernels stage node records with the far-form constants folded in
(dipole vector times sqrt(pi)/2, 2 s2 times 1.5), so they need S / (sqrt(pi)/2)
and T / (1.5 sqrt(pi)/2); the numerators are emitted divided by those factors
(one rounding of the exact quotient).

Run:  python gen_kfit.py   (takes a few minutes; rewrites kfit_tables.h)
"""
import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 50
HESS_X, HESS_DEG = 32.0, 14
HERE = os.path.dirname(os.path.abspath(__file__))


def S(x):
    x = mp.mpf(x)
    return mp.mpf(2) / 3 if x == 0 else mp.gammainc(mp.mpf(1.5), 0, x) / x ** mp.mpf(1.5)


def T(x):
    x = mp.mpf(x)
    return mp.mpf(2) / 5 if x == 0 else mp.gammainc(mp.mpf(2.5), 0, x) / x ** mp.mpf(2.5)


def U(x):
    x = mp.mpf(x)
    return mp.mpf(2) / 7 if x == 0 else mp.gammainc(mp.mpf(3.5), 0, x) / x ** mp.mpf(3.5)


def fit_common(fs, X, n, m, K=300, iters=40):
    xs = [X * (1 - mp.cos(mp.pi * k / (K - 1))) / 2 for k in range(K)]
    ts = [x / X for x in xs]
    F = [[f(x) for x in xs] for f in fs]
    nf = len(fs)
    Q0 = [mp.mpf(1)] * K
    w = [mp.mpf(1)] * K
    best = None
    for it in range(iters):
        rows, rhs = [], []
        for fi in range(nf):
            for k in range(K):
                sc = mp.sqrt(w[k]) / (F[fi][k] * Q0[k])
                row = [mp.mpf(0)] * (nf * (n + 1) + m)
                for j in range(n + 1):
                    row[fi * (n + 1) + j] = ts[k] ** j * sc
                for j in range(1, m + 1):
                    row[nf * (n + 1) + j - 1] = -F[fi][k] * ts[k] ** j * sc
                rows.append(row)
                rhs.append(F[fi][k] * sc)
        A, b = mp.matrix(rows), mp.matrix(rhs)
        c = mp.lu_solve(A.T * A, A.T * b)
        P = [[c[fi * (n + 1) + j] for j in range(n + 1)] for fi in range(nf)]
        q = [mp.mpf(1)] + [c[nf * (n + 1) + j] for j in range(m)]
        Qv = [mp.polyval(q[::-1], t) for t in ts]
        errs = [max(abs(mp.polyval(P[fi][::-1], ts[k]) / Qv[k] / F[fi][k] - 1) for fi in range(nf))
                for k in range(K)]
        me = max(errs)
        if best is None or me < best[0]:
            best = (me, P, q)
        Q0 = Qv
        if it >= 8:
            s = sum(w[k] * errs[k] for k in range(K))
            w = [w[k] * errs[k] / s * K for k in range(K)]
    return best


FOLD = (mp.sqrt(mp.pi) / 2, mp.mpf(3) / 2 * mp.sqrt(mp.pi) / 2)   # S and T divisors


def fold(P, div=FOLD):
    return [[c / div[fi] for c in p] for fi, p in enumerate(P)]


def check(P, q, X, dt, fs=(S, T), div=FOLD):
    """Max relative error of the rounded (folded) coefficients evaluated in
    dtype dt against f / div for each fitted function f (FMA-free Horner, a
    pessimistic stand-in for the device evaluation)."""
    Pc = [np.array([float(c) for c in p], dtype=dt) for p in P]
    qc = np.array([float(c) for c in q], dtype=dt)
    xs = np.linspace(0.0, X, 4001)
    t = (xs.astype(dt) * dt(1.0 / X)).astype(dt)

    def horner(c):
        r = np.full_like(t, c[-1])
        for a in c[-2::-1]:
            r = (r * t + a).astype(dt)
        return r
    r = dt(1) / horner(qc)
    out = []
    for fi, f in enumerate(fs):
        v = horner(Pc[fi]) * r
        out.append(max(abs(float(v[i]) / float(f(xs[i]) / div[fi]) - 1) for i in range(len(xs))))
    return out


def emit(f, name, ctype, P, q, X, fit_err, eval_err, labels=("PS", "PT")):
    lit = (lambda v: "%.17e" % v) if ctype == "double" else (lambda v: "%.9ef" % v)
    f.write("// %s: x in [0, %g], degree (%d, %d); fit max rel err %.2e; "
            "rounded-coefficient Horner max rel err %s\n"
            % (name, X, len(P[0]) - 1, len(q) - 1, fit_err,
               ", ".join("%s %.2e" % (lb[1], e) for lb, e in zip(labels, eval_err))))
    f.write("#define %s_X %s\n" % (name.upper(), lit(X)))
    f.write("#define %s_INV_X %s\n" % (name.upper(), lit(1.0 / X)))
    for label, coef in list(zip(labels, P)) + [("Q", q)]:
        f.write("#define %s_%s_DEG %d\n" % (name.upper(), label, len(coef) - 1))
        f.write("__device__ __constant__ static const %s %s_%s[%d] = {\n" % (ctype, name, label.lower(), len(coef)))
        f.write(",\n".join("    " + lit(float(c)) for c in coef) + "};\n")
    f.write("\n")


def main():
    specs = [("kf64", 32.0, 13, 13, np.float64, "double"),
             ("kf32", 20.0, 7, 7, np.float32, "float")]
    out = os.path.join(HERE, "kfit_tables.h")
    with open(out + ".tmp", "w") as f:
        f.write("// Generated by gen_kfit.py -- do not edit.\n"
                "// Rational fits S' ~ P_S(t)/Q(t), T' ~ P_T(t)/Q(t), t = x/X, of\n"
                "// S' = S / (sqrt(pi)/2), T' = T / (1.5 sqrt(pi)/2) with\n"
                "// S(x) = gamma(3/2,x)/x^(3/2) and T(x) = gamma(5/2,x)/x^(5/2).\n"
                "#pragma once\n\n")
        for name, X, n, m, dt, ctype in specs:
            fe, P, q = fit_common([S, T], mp.mpf(X), n, m)
            P = fold(P)
            ee = check(P, q, X, dt)
            print(name, "fit", mp.nstr(fe, 3), "eval", ee, file=sys.stderr)
            emit(f, name, ctype, P, q, X, float(fe), ee)
        # the Hessian's three radial functions S, T, U (not folded): k1 = S,
        # k2 = -2 s2 T, k3 = 4 s2^2 U with U(x) = gamma(7/2,x)/x^(7/2)
        f.write("// kf64h: S, T and U(x) = gamma(7/2,x)/x^(7/2) over one denominator (not folded),\n"
                "// for the Hessian pairs inside the cut.\n")
        fe, P, q = fit_common([S, T, U], mp.mpf(HESS_X), HESS_DEG, HESS_DEG)
        ee = check(P, q, HESS_X, np.float64, fs=(S, T, U), div=(1, 1, 1))
        print("kf64h", "fit", mp.nstr(fe, 3), "eval", ee, file=sys.stderr)
        emit(f, "kf64h", "double", P, q, HESS_X, float(fe), ee, labels=("PS", "PT", "PU"))
    os.replace(out + ".tmp", out)


if __name__ == "__main__":
    main()
