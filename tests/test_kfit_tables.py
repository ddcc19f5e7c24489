"""The rational fits of the radial functions that the HIP pair kernels use
(kfit_tables.h), checked on the host against the regularised incomplete gamma
function of scipy:

    S(x) = gamma(3/2, x) / x^(3/2),  T(x) = gamma(5/2, x) / x^(5/2),
    U(x) = gamma(7/2, x) / x^(7/2)   (lower incomplete gamma; S(0) = 2/3,
    T(0) = 2/5, U(0) = 2/7),

the radial functions of the smoothed kernel and of its first and second
derivatives (section 4.1, eq. kerpsi and its derivatives).  The kf64 and
kf32 numerators are stored divided by sqrt(pi)/2 and 1.5 sqrt(pi)/2."""
import math
import os
import re

import numpy as np
import pytest
from scipy.special import gamma, gammainc

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1909_13356_amd", "csrc", "kfit_tables.h")


def tables():
    txt = open(HDR).read()
    out = {}
    for name, body in re.findall(r"static const (?:double|float) (\w+)\[\d+\] = \{([^}]*)\}", txt):
        out[name] = np.array([float(v.rstrip("f")) for v in body.replace("\n", " ").split(",")])
    for name, val in re.findall(r"#define (\w+_X) ([0-9.e+-]+)f?", txt):
        out[name] = float(val)
    return out


def radial(a, x):
    x = np.asarray(x, float)
    return gamma(a) * gammainc(a, x) / x ** a


def rational(num, q, t):
    # power basis in t = x / X, as the kernels evaluate it
    return np.polyval(num[::-1], t) / np.polyval(q[::-1], t)


XS = np.concatenate([np.geomspace(1e-3, 1.0, 200), np.linspace(1.0, 32.0, 2000)[1:]])


@pytest.mark.parametrize("name,X,fold,tol", [
    ("kf64", "KF64_X", True, 2e-14),
    ("kf64h", "KF64H_X", False, 2e-14),
    ("kf32", "KF32_X", True, 2e-6),
])
def test_fit_against_incomplete_gamma(name, X, fold, tol):
    tb = tables()
    Xv = tb[X]
    xs = XS[XS < Xv]
    t = xs / Xv
    q = tb[name + "_q"]
    fns = [("ps", 1.5, math.sqrt(math.pi) / 2), ("pt", 2.5, 1.5 * math.sqrt(math.pi) / 2)]
    if name == "kf64h":
        fns.append(("pu", 3.5, 1.0))
    for key, a, div in fns:
        exact = radial(a, xs) / (div if fold else 1.0)
        fit = rational(tb["%s_%s" % (name, key)], q, t)
        err = np.max(np.abs(fit / exact - 1.0))
        assert err < tol, (name, key, err)
        # the limit at x = 0: 1 / (a) (gamma(a, x) ~ x^a / a)
        v0 = tb["%s_%s" % (name, key)][0] / q[0]
        assert abs(v0 * (div if fold else 1.0) * a - 1.0) < 10 * tol, (name, key, v0)
