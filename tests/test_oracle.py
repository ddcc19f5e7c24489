"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with an
independent definition (incomplete gamma functions, closed-form Gaussian
convolutions of a box and a ball, Gauss's law / solid angles, finite
differences, brute force at 30 digits, symmetry) or with constants printed in
the paper (tests/golden/paper_constants.txt).
"""
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy.special import erf
from scipy.integrate import quad

import oracle
from workloads import (dunavant6, chart_nodes, cube_mesh, icosphere, star_surface, torus_mesh, quadratic_from_flat,
                       triangle_diameters, box_targets, shell_targets, configs)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")
RT2, PI = np.sqrt(2.0), np.pi


def golden():
    out = {}
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            out[k] = v
    return out


# ------------------------------------------------------------ closed forms
def box_closed(x, s, lo=0.0, hi=1.0):
    """Gaussian convolution of the box indicator and its gradient."""
    f = 0.5 * (erf((hi - x) / (RT2 * s)) + erf((x - lo) / (RT2 * s)))
    e = (np.exp(-(x - lo) ** 2 / (2 * s * s)) - np.exp(-(hi - x) ** 2 / (2 * s * s))) / (np.sqrt(2 * PI) * s)
    P = f.prod(1)
    G = np.stack([e[:, i] * np.prod(np.delete(f, i, 1), 1) for i in range(3)], 1)
    return P, G


def ball_closed(r, s):
    """Gaussian convolution of the unit-ball indicator, Phi(r) and dPhi/dr."""
    Em = np.exp(-(1 - r) ** 2 / (2 * s * s))
    Ep = np.exp(-(1 + r) ** 2 / (2 * s * s))
    phi = 0.5 * (erf((1 - r) / (RT2 * s)) + erf((1 + r) / (RT2 * s))) - s / (r * np.sqrt(2 * PI)) * (Em - Ep)
    dphi = ((s / r ** 2 - 1 / (r * s)) * Em - (s / r ** 2 + 1 / (r * s)) * Ep) / np.sqrt(2 * PI)
    return phi, dphi


def test_ball_closed_form_is_the_convolution():
    # the ball formula itself against direct radial quadrature of the convolution
    s = 0.2
    for r in (0.3, 0.9, 1.1, 1.7):
        f = lambda q: (q / r) * (np.exp(-(r - q) ** 2 / (2 * s * s)) - np.exp(-(r + q) ** 2 / (2 * s * s)))
        val = quad(f, 0, 1, epsabs=1e-14, epsrel=1e-14)[0] / (np.sqrt(2 * PI) * s)
        assert abs(val - ball_closed(np.array([r]), s)[0][0]) < 1e-12
        h = 1e-5
        fd = (ball_closed(np.array([r + h]), s)[0] - ball_closed(np.array([r - h]), s)[0]) / (2 * h)
        assert abs(fd[0] - ball_closed(np.array([r]), s)[1][0]) < 1e-8


# -------------------------------------------------------- radial functions
def test_radial_vs_incomplete_gamma():
    mp.mp.dps = 40
    for sigma in (0.05, 1.0):
        c = 1 / (4 * mp.sqrt(2) * mp.pi ** 1.5 * mp.mpf(sigma) ** 3)
        us = np.concatenate([np.linspace(1e-4, 3, 61), [0.999999, 1.0, 1.000001, 4, 5.66, 8, 12]])
        rho = us * RT2 * sigma
        K, F = oracle.radial(rho, sigma)
        for i, u in enumerate(us):
            u = mp.mpf(u)
            Kx = c * mp.gammainc(1.5, 0, u * u) / u ** 3
            Fx = -c * mp.gammainc(2.5, 0, u * u) / (u ** 5 * mp.mpf(sigma) ** 2)
            assert abs(K[i] - float(Kx)) <= 2e-15 * abs(float(Kx)), (sigma, float(u))
            assert abs(F[i] - float(Fx)) <= 1e-14 * abs(float(Fx)), (sigma, float(u))
    # rho = 0: finite limits 2/3 c and -2/5 c / sigma^2
    K, F = oracle.radial(np.array([0.0]), 1.0)
    c0 = 1 / (4 * RT2 * PI ** 1.5)
    assert abs(K[0] - 2 / 3 * c0) < 1e-16 and abs(F[0] + 2 / 5 * c0) < 1e-16


def test_radial_matches_printed_series():
    g = golden()
    coef = [float(Fraction(c)) for c in g["series_K"]]
    ucut, err = map(float, g["series_err_below_u"])
    sigma = 0.3
    c0 = 1 / (4 * np.sqrt(2 * PI ** 3) * sigma ** 3)
    us = np.linspace(0, ucut, 41)
    K, _ = oracle.radial(us * RT2 * sigma, sigma)
    printed = sum(cf * us ** (2 * k) for k, cf in enumerate(coef))
    # "about 1e-13": the first omitted term, -u^10/780, is 1.28e-13 in size at u = 0.1
    assert np.max(np.abs(K / c0 - printed)) < 1.5 * err
    assert np.max(np.abs(K / c0 - printed + us ** 10 / 780)) < 1e-15


def test_far_kernel_is_dipole_beyond_8sigma():
    # at rho >= 8 sigma K is the Laplace dipole factor 1/(4 pi rho^3) to the
    # paper's tail bounds (section 4.4): erf deficit + exp term
    g = golden()
    b = float(g["tail_8sigma_erf"][0]) + float(g["tail_8sigma_exp"][0])
    sigma = 0.01
    rho = np.array([8.0, 9.0, 12.0]) * sigma
    K, F = oracle.radial(rho, sigma)
    dip = 1 / (4 * PI * rho ** 3)
    rel = np.abs(K - dip) / dip
    assert 1e-15 < rel[0] < 10 * b and np.all(rel[1:] < 1e-15)
    # F = K'/rho -> -3/(4 pi rho^5); its exp term is larger by (rho/sigma)^3 / 3
    relF = np.abs(F + 3 * dip / rho ** 2) / (3 * dip / rho ** 2)
    bF = b * (1 + np.sqrt(2 / PI) * (rho / sigma) ** 3 / 3)
    assert np.all(relF < 2 * bF) and relF[0] > 1e-13


# ----------------------------------------------------------- quadrature nodes
def test_nodes_closed_surface_identities():
    v, t = cube_mesh(4)
    y, a = oracle.nodes(v, t, dunavant6())
    assert np.abs(a.sum(0)).max() < 1e-14                     # sum of w J over a closed surface
    assert abs(np.sum(y * a) / 3 - 1.0) < 1e-13               # divergence theorem: volume
    v, t = icosphere(3)
    y, a = oracle.nodes(v, t, dunavant6())
    # nodes lie on the triangles, normals outward
    assert np.all(np.einsum("ij,ij->i", a, y) > 0)


# ------------------------------------------------------- box (config 1 geometry)
@pytest.mark.slow
def test_box_closed_form_config1():
    c = configs.config1()
    phi, g = oracle.evaluate(c["verts"], c["tris"], c["sigma"], c["rule"], c["targets"])
    P, G = box_closed(c["targets"], 0.1)
    assert np.abs(phi - P).max() < 5e-11
    assert np.abs(g - G).max() < 1e-9


def test_box_closed_form_fine_mesh():
    v, t = cube_mesh(32)
    x = box_targets(64, seed=11)
    phi, g = oracle.evaluate(v, t, [0.1], dunavant6(), x)
    P, G = box_closed(x, 0.1)
    assert np.abs(phi - P).max() < 2e-13
    assert np.abs(g - G).max() < 5e-12


def test_box_shifted_and_per_triangle_sigma_equal():
    v, t = cube_mesh(16)
    v2 = v * 2.0 - 0.5                       # box [-0.5, 1.5]^3, sigma scaled with it
    x = box_targets(48, -1.0, 2.0, seed=3)
    phi, g = oracle.evaluate(v2, t, np.full(len(t), 0.2), dunavant6(), x)
    P, G = box_closed(x, 0.2, -0.5, 1.5)
    assert np.abs(phi - P).max() < 5e-11 and np.abs(g - G).max() < 1e-9
    phi1, g1 = oracle.evaluate(v2, t, [0.2], dunavant6(), x)
    assert np.array_equal(phi, phi1) and np.array_equal(g, g1)


# -------------------------------------------------------------- ball (config 2)
def test_ball_far_and_near():
    v, t = icosphere(5)
    x = shell_targets(400, 0.5, 1.5, seed=2)
    r = np.linalg.norm(x, axis=1)
    far = np.abs(r - 1) >= 0.4
    xs = np.concatenate([x[far][:60], x[~far][:40]])
    rs = np.linalg.norm(xs, axis=1)
    phi, g = oracle.evaluate(v, t, [0.05], dunavant6(), xs)
    P, dP = ball_closed(rs, 0.05)
    G = dP[:, None] * xs / rs[:, None]
    assert np.abs(phi[:60] - P[:60]).max() < 1e-13
    assert np.abs(g[:60] - G[:60]).max() < 1e-12
    # near the surface the flat polyhedron differs from the ball by O(h^2)
    assert np.abs(phi[60:] - P[60:]).max() < 5e-3


def test_ball_near_error_is_second_order():
    x = shell_targets(60, 0.9, 1.1, seed=7)
    rs = np.linalg.norm(x, axis=1)
    errs = []
    for lev in (2, 3):
        v, t = icosphere(lev)
        phi, _ = oracle.evaluate(v, t, [0.2], dunavant6(), x)
        errs.append(np.abs(phi - ball_closed(rs, 0.2)[0]).max())
    assert 3.0 < errs[0] / errs[1] < 5.0


# -------------------------------------------------- derivatives and symmetry
def test_gradient_matches_finite_differences():
    v, t = star_surface(6, seed=5)
    sig = 0.5 * triangle_diameters(v, t)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1.2, 1.2, size=(6, 3))
    _, g = oracle.evaluate(v, t, sig, dunavant6(), x)
    hs = 1e-3
    fd = np.zeros_like(g)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1

        def D(h):
            p = oracle.evaluate(v, t, sig, dunavant6(), np.concatenate([x + h * e, x - h * e]))[0]
            return (p[:6] - p[6:]) / (2 * h)
        fd[:, i] = (4 * D(hs / 2) - D(hs)) / 3
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_invariances():
    v, t = star_surface(5, seed=2)
    sig = 0.5 * triangle_diameters(v, t)
    rule = dunavant6()
    x = box_targets(20, -1.2, 1.2, seed=4)
    phi, g = oracle.evaluate(v, t, sig, rule, x)
    # translation
    s = np.array([0.3, -1.1, 2.0])
    p2, g2 = oracle.evaluate(v + s, t, sig, rule, x + s)
    assert np.abs(p2 - phi).max() < 1e-13 and np.abs(g2 - g).max() < 1e-12
    # rotation
    Q, _ = np.linalg.qr(np.random.default_rng(0).normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    p3, g3 = oracle.evaluate(v @ Q.T, t, sig, rule, x @ Q.T)
    assert np.abs(p3 - phi).max() < 1e-13 and np.abs(g3 - g @ Q.T).max() < 1e-12
    # scaling geometry and sigma together
    p4, g4 = oracle.evaluate(v * 3.0, t, sig * 3.0, rule, x * 3.0)
    assert np.abs(p4 - phi).max() < 1e-13 and np.abs(g4 * 3.0 - g).max() < 1e-12
    # permutation of the triangles
    perm = np.random.default_rng(1).permutation(len(t))
    p5, g5 = oracle.evaluate(v, t[perm], sig[perm], rule, x)
    assert np.abs(p5 - phi).max() < 1e-14 and np.abs(g5 - g).max() < 1e-13
    # orientation flip: Phi -> -Phi
    p6, g6 = oracle.evaluate(v, t[:, ::-1].copy(), sig, rule, x)
    assert np.abs(p6 + phi).max() < 1e-14 and np.abs(g6 + g).max() < 1e-13


def test_additivity_and_batch_offsets():
    v1, t1 = cube_mesh(4)
    v2, t2 = icosphere(2)
    v2 = v2 * 0.5 + 3.0
    rule = dunavant6()
    x = box_targets(10, -0.5, 3.5, seed=6)
    pa, ga = oracle.evaluate(v1, t1, [0.1], rule, x)
    pb, gb = oracle.evaluate(v2, t2, [0.1], rule, x)
    V = np.concatenate([v1, v2])
    T = np.concatenate([t1, t2 + len(v1)])
    pc, gc = oracle.evaluate(V, T, [0.1], rule, x)
    assert np.abs(pc - pa - pb).max() < 1e-14 and np.abs(gc - ga - gb).max() < 1e-12
    # CSR offsets + per-target mesh ids select one mesh per target
    off = np.array([0, len(t1), len(t1) + len(t2)])
    xm = np.arange(10, dtype=np.int32) % 2
    pd, gd = oracle.evaluate(V, T, [0.1], rule, x, tri_offsets=off, x_mesh=xm)
    want = np.where(xm == 0, pa, pb)
    assert np.array_equal(pd, want)


# ------------------------------------------------------------ Gauss / solid angle
def test_gauss_law_far_from_surface():
    # far from a closed surface the kernel is the Laplace double layer, whose
    # integral is 1 inside and 0 outside; the discrete sum approaches it as the
    # quadrature resolves the surface
    inside = np.array([[0.0, 0.0, 0.0], [0.05, -0.02, 0.03]])
    outside = np.array([[4.0, 0.0, 0.0], [0.0, -5.0, 3.0]])
    for nu, tol in ((16, 5e-12), (32, 1e-13)):
        v, t = star_surface(nu, seed=8)
        sig = 0.5 * triangle_diameters(v, t)
        pin, _ = oracle.evaluate(v, t, sig, dunavant6(), inside)
        pout, _ = oracle.evaluate(v, t, sig, dunavant6(), outside)
        assert np.abs(pin - 1).max() < tol and np.abs(pout).max() < tol


def test_single_triangle_far_field_solid_angle():
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.2, 0.9, 0]])
    t = np.array([[0, 1, 2]], np.int32)
    x = np.array([[0.4, 0.3, -20.0], [15.0, 7.0, -9.0], [0.1, 0.2, 25.0]])
    phi, _ = oracle.evaluate(P, t, [0.01], dunavant6(), x)
    for k in range(3):
        R = P - x[k]
        r = np.linalg.norm(R, axis=1)
        num = np.dot(R[0], np.cross(R[1], R[2]))
        den = r.prod() + np.dot(R[0], R[1]) * r[2] + np.dot(R[0], R[2]) * r[1] + np.dot(R[1], R[2]) * r[0]
        omega = 2 * np.arctan2(num, den)
        assert abs(phi[k] - omega / (4 * PI)) < 1e-8 * abs(omega / (4 * PI))


def test_bruteforce_30_digits():
    mp.mp.dps = 30
    P = np.array([[0.0, 0, 0], [1.0, 0.1, 0], [0.3, 0.8, 0.2], [0.5, 0.4, -0.7]])
    t = np.array([[0, 1, 2], [0, 2, 3], [1, 3, 2]], np.int32)
    sig = np.array([0.3, 0.15, 0.6])
    rule = dunavant6()
    y, a = oracle.nodes(P, t, rule)
    # targets: generic points, one exactly on a node, one very close to a node
    x = np.array([[0.4, 0.3, 0.1], [1.5, -0.4, 0.9], y[5], y[17] + 1e-9])
    phi, g = oracle.evaluate(P, t, sig, rule, x)
    for i in range(len(x)):
        S = mp.mpf(0)
        Gs = [mp.mpf(0)] * 3
        for k in range(len(y)):
            s = mp.mpf(sig[k // 12])
            d = [mp.mpf(x[i, c]) - mp.mpf(y[k, c]) for c in range(3)]
            rho = mp.sqrt(sum(q * q for q in d))
            ak = [mp.mpf(a[k, c]) for c in range(3)]
            ad = sum(ak[c] * d[c] for c in range(3))
            u = rho / (mp.sqrt(2) * s)
            if rho == 0:
                Kv = 2 / (3 * 4 * mp.sqrt(2 * mp.pi ** 3) * s ** 3)
                Fv = -2 / (5 * 4 * mp.sqrt(2 * mp.pi ** 3) * s ** 5)
            else:
                Kv = mp.erf(u) / (4 * mp.pi * rho ** 3) - mp.sqrt(2 / mp.pi) * mp.exp(-u * u) / (4 * mp.pi * s * rho ** 2)
                Kp = mp.diff(lambda r: mp.erf(r / (mp.sqrt(2) * s)) / (4 * mp.pi * r ** 3)
                             - mp.sqrt(2 / mp.pi) * mp.exp(-r * r / (2 * s * s)) / (4 * mp.pi * s * r ** 2), rho)
                Fv = Kp / rho
            S += -ad * Kv
            for c in range(3):
                Gs[c] += -ak[c] * Kv - ad * Fv * d[c]
        scale = max(1.0, abs(float(S)))
        assert abs(phi[i] - float(S)) < 1e-14 * scale, i
        gs = max(1.0, max(abs(float(q)) for q in Gs))
        for c in range(3):
            assert abs(g[i, c] - float(Gs[c])) < 1e-13 * gs, (i, c)


# --------------------------------------------------------------- pseudonormals
def test_pseudonormals():
    v, t = cube_mesh(3)
    H = oracle.pseudonormals(v, t)
    corner = np.all((v == 0) | (v == 1), axis=1)
    exp = np.where(v[corner] > 0.5, 1.0, -1.0) / 3.0      # (n1 + n2 + n3) / 3 at a corner
    assert np.abs(H[corner] - exp).max() < 1e-15
    face = (np.sum((v == 0) | (v == 1), axis=1) == 1)
    n = np.where(v[face] == 1, 1.0, np.where(v[face] == 0, -1.0, 0.0))
    assert np.abs(H[face] - n).max() < 1e-15
    v, t = icosphere(4)
    H = oracle.pseudonormals(v, t)
    cosang = np.einsum("ij,ij->i", H, v) / np.linalg.norm(H, axis=1)
    assert cosang.min() > 1 - 1e-4


# ---------------------------------------------------------------------- Newton
def test_newton_flat_face_h_zero():
    # cube 32x32 per face, sigma = 0.02: chart nodes of triangles whose nodes
    # are all >= 8.5 sigma from every edge stay on the face (section 2: flat
    # regions wider than the kernel are preserved on the 1/2 level set)
    v, t = cube_mesh(32)
    sigma = 0.02
    cen = v[t].mean(1)
    # distance of the centroid to the nearest cube edge within its face
    inner = np.sort(np.minimum(cen, 1 - cen), axis=1)[:, 1]
    sel = np.nonzero(inner > 8.5 * sigma + 1.0 / 32)[0][::97][:12]
    uv = chart_nodes(4)
    h, x, st, it = oracle.project(v, t, [sigma], dunavant6(), uv, tau=1e-12, sel=sel)
    assert np.all(st == 0)
    assert np.abs(h).max() < 1e-12 * sigma * 10
    phi, _ = oracle.evaluate(v, t, [sigma], dunavant6(), x)
    assert np.abs(phi - 0.5).max() < 1e-12


def test_newton_sphere_level_set_and_status():
    v, t = icosphere(3)
    sigma = 0.1
    uv = chart_nodes(2)
    sel = np.arange(0, len(t), 97)
    h, x, st, it = oracle.project(v, t, [sigma], dunavant6(), uv, sel=sel)
    assert np.all(st == 0) and it.max() <= 8
    phi, _ = oracle.evaluate(v, t, [sigma], dunavant6(), x)
    assert np.abs(phi - 0.5).max() < 1e-12
    # the 1/2 level set of the ball convolution (smoke check, O(h^2) polyhedron gap)
    from scipy.optimize import brentq
    rstar = brentq(lambda r: ball_closed(np.array([r]), sigma)[0][0] - 0.5, 0.5, 1.5)
    assert np.abs(np.linalg.norm(x, axis=1) - rstar).max() < 0.02
    # forced statuses: one iteration only -> MAXITER
    _, _, st1, it1 = oracle.project(v, t, [sigma], dunavant6(), uv, sel=sel[:3], max_iter=1)
    assert np.all(st1 == 1) and np.all(it1 == 1)


def test_newton_nobracket_and_degenerate():
    # tiny cube with sigma much larger than the cube: Phi < 1/2 everywhere
    v, t = cube_mesh(1)
    _, _, st, _ = oracle.project(v, t, [5.0], dunavant6(), chart_nodes(1), sel=[0, 5])
    assert np.all(st == 2)
    # two coincident triangles of opposite orientation: vertex pseudonormals vanish
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    t2 = np.array([[0, 1, 2], [0, 2, 1]], np.int32)
    h, x, st, it = oracle.project(P, t2, [0.1], dunavant6(), chart_nodes(1))
    assert np.all(st == 3) and np.all(h == 0) and np.all(it == 0)


def test_newton_no_root_is_never_converged():
    """Where Phi - 1/2 keeps one sign on the whole search segment there is no
    root: whatever the tolerance, the node ends NOBRACKET within a few
    bisection steps instead of creeping to the end of the range."""
    v, t = cube_mesh(1)
    sigma = 5.0
    uv = chart_nodes(1)
    H = oracle.pseudonormals(v, t)
    j = 0
    T = v[t[j, 0]] + uv[0, 0] * (v[t[j, 1]] - v[t[j, 0]]) + uv[0, 1] * (v[t[j, 2]] - v[t[j, 0]])
    Hj = H[t[j, 0]] + uv[0, 0] * (H[t[j, 1]] - H[t[j, 0]]) + uv[0, 1] * (H[t[j, 2]] - H[t[j, 0]])
    hmax = 16 * sigma / np.linalg.norm(Hj)
    hs = np.linspace(-hmax, hmax, 41)
    phi, _ = oracle.evaluate(v, t, [sigma], dunavant6(), T[None, :] + hs[:, None] * Hj[None, :])
    assert np.all(phi < 0.5)
    for tau in (1e-6, 1e-12):
        h, x, st, it = oracle.project(v, t, [sigma], dunavant6(), uv[:1], sel=[j], tau=tau)
        assert st[0] == 2 and it[0] <= 6 and abs(h[0]) > 0.75 * hmax


# ------------------------------------------------------------- chart geometry
def test_chart_geometry_tangents_match_finite_differences():
    """x_u and x_v of eq. u_vector / v_vector against central differences of
    the oracle's own Newton solution x(u +- d, v), x(u, v +- d): a dropped
    term (h H_u), a sign or the dh/du quotient of eq. U_vector_2 would show."""
    v, t = star_surface(6, lmax=6, var0=0.1, seed=3)
    sig = 0.5 * triangle_diameters(v, t)
    uv = np.array([[0.2, 0.3], [0.55, 0.15], [0.1, 0.7]])
    sel = np.array([3, 40, 111])
    h, x, st, _ = oracle.project(v, t, sig, dunavant6(), uv, tau=1e-14, sel=sel)
    assert np.all(st == 0)
    xu, xv, da, nrm = oracle.chart_geometry(v, t, sig, dunavant6(), uv, h, sel=sel)
    d = 1e-4
    for k, (du, dv) in enumerate(((d, 0.0), (0.0, d))):
        up = oracle.project(v, t, sig, dunavant6(), uv + [du, dv], tau=1e-14, sel=sel)[1]
        dn = oracle.project(v, t, sig, dunavant6(), uv - [du, dv], tau=1e-14, sel=sel)[1]
        fd = (up - dn) / (2 * d)
        an = xu if k == 0 else xv
        err = np.linalg.norm(fd - an, axis=1) / np.linalg.norm(an, axis=1)
        assert err.max() < 1e-6, err
    # tangency, the normal's orientation and the area element's definition
    assert np.abs(np.sum(xu * nrm, axis=1)).max() < 1e-10 * np.linalg.norm(xu, axis=1).max()
    assert np.abs(np.sum(xv * nrm, axis=1)).max() < 1e-10 * np.linalg.norm(xv, axis=1).max()
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
    c = v.mean(axis=0)
    assert np.all(np.sum((x - c) * nrm, axis=1) > 0)             # outward on a star-shaped surface
    assert np.allclose(da, np.linalg.norm(np.cross(xu, xv), axis=1))


def test_chart_geometry_sphere_normals_and_area():
    """On a fine icosphere the 1/2 level set is nearly a sphere: the normals
    are nearly radial and the charts' areas (interpolatory weights of the
    chart nodes times da) add up to nearly 4 pi r^2."""
    v, t = icosphere(3)
    sigma = 0.1
    uv = chart_nodes(4)
    h, x, st, _ = oracle.project(v, t, [sigma], dunavant6(), uv)
    assert np.all(st == 0)
    xu, xv, da, nrm = oracle.chart_geometry(v, t, [sigma], dunavant6(), uv, h)
    r = np.linalg.norm(x, axis=1)
    cosang = np.sum(x * nrm, axis=1) / r
    assert cosang.min() > 0.999
    w = simplex_weights(uv, 4)
    area = np.sum(da.reshape(len(t), -1) * w[None, :])
    rm = r.mean()
    assert abs(area / (4 * np.pi * rm ** 2) - 1) < 5e-3


def simplex_weights(uv, deg):
    """Interpolatory quadrature weights of the nodes uv on the standard
    simplex: exact for every monomial u^a v^b with a + b <= deg (moments
    a! b! / (a + b + 2)!)."""
    from math import factorial
    rows, mom = [], []
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            rows.append(uv[:, 0] ** a * uv[:, 1] ** b)
            mom.append(factorial(a) * factorial(b) / factorial(a + b + 2))
    return np.linalg.solve(np.array(rows), np.array(mom))


# --------------------------------------------------- Koornwinder interpolation
def test_koornwinder_basis_is_orthogonal_on_the_simplex():
    """Gram matrix of the basis by a collapsed Gauss-Legendre rule exact to
    degree 2p: diagonal only (a wrong Jacobi parameter or homogenisation
    would couple the columns)."""
    p = 6
    g, w = np.polynomial.legendre.leggauss(p + 2)
    a, b = (g + 1) / 2, (g + 1) / 2
    A, B = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(w / 2, w / 2, indexing="ij")
    v = B.ravel()
    u = A.ravel() * (1 - v)
    wt = (WA * WB).ravel() * (1 - v)                          # du dv = (1 - v) da db
    K = oracle.koornwinder(np.stack([u, v], 1), p)
    G = K.T @ (wt[:, None] * K)
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-13 * np.abs(np.diag(G)).max()
    assert np.isclose(G[0, 0], 0.5)                           # K_00 = 1: the simplex area


@pytest.mark.parametrize("p", [2, 4, 8])
def test_chart_interp_reproduces_polynomials(p):
    rng = np.random.default_rng(p)
    uv = chart_nodes(p)
    ev = rng.dirichlet([1, 1, 1], 50)[:, :2]
    mons = [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]
    ntris = 3
    co = rng.standard_normal((ntris, len(mons), 2))
    q = lambda pts, j, c: sum(co[j, k, c] * pts[:, 0] ** a * pts[:, 1] ** b for k, (a, b) in enumerate(mons))
    f = np.stack([np.stack([q(uv, j, c) for c in range(2)], 1) for j in range(ntris)]).reshape(-1, 2)
    want = np.stack([np.stack([q(ev, j, c) for c in range(2)], 1) for j in range(ntris)]).reshape(-1, 2)
    got = oracle.chart_interp(uv, f, ev)
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()


def test_chart_interp_converges_on_a_smooth_function():
    rng = np.random.default_rng(1)
    ev = rng.dirichlet([1, 1, 1], 200)[:, :2]
    exact = np.exp(ev[:, 0] + 2 * ev[:, 1])
    errs = []
    for p in (2, 4, 8):
        uv = chart_nodes(p)
        errs.append(np.abs(oracle.chart_interp(uv, np.exp(uv[:, 0] + 2 * uv[:, 1]), ev) - exact).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-5


# ------------------------------------------------ quadratic skeleton triangles
def _unit_sphere(p):
    return p / np.linalg.norm(p, axis=1, keepdims=True)


def test_quadratic_nodes_sit_on_their_six_points():
    """The rule points (0,0), (1,0), (0,1), (1/2,0), (1/2,1/2), (0,1/2) of T0
    land on P1..P6 (node order: corners, then the edges P1P2, P2P3, P3P1)."""
    rng = np.random.default_rng(3)
    verts = rng.normal(size=(6, 3))
    uvw = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1], [.5, 0, 1], [.5, .5, 1], [0, .5, 1]], float)
    y, _ = oracle.nodes(verts, np.arange(6, dtype=np.int32)[None], uvw)
    assert np.array_equal(y, verts)


def test_quadratic_with_midpoint_edges_is_the_flat_triangle():
    v, t = icosphere(1)
    v6, t6 = quadratic_from_flat(v, t)
    rule = dunavant6()
    y3, a3 = oracle.nodes(v, t, rule)
    y6, a6 = oracle.nodes(v6, t6, rule)
    assert np.max(np.abs(y6 - y3)) < 1e-15
    assert np.max(np.abs(a6 - a3)) < 1e-15


def test_quadratic_patch_vector_area_is_the_boundary_integral():
    """Stokes: the vector area of a surface patch, int n dA, equals half the
    boundary integral of y x dy.  The boundary of a quadratic triangle is
    three parabolic arcs through a corner, the edge point and the next corner,
    and c x c' is a cubic in the arc parameter, so 3-point Gauss-Legendre
    integrates it exactly; the 12-point rule is exact for the degree-2
    integrand y_u x y_v."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        P = rng.normal(size=(6, 3))
        _, a = oracle.nodes(P, np.arange(6, dtype=np.int32)[None], dunavant6())
        g, gw = np.polynomial.legendre.leggauss(3)
        t, gw = 0.5 * (g + 1.0), 0.5 * gw
        ref = np.zeros(3)
        for A, M, B in ((P[0], P[3], P[1]), (P[1], P[4], P[2]), (P[2], P[5], P[0])):
            c = (np.outer((1 - t) * (1 - 2 * t), A) + np.outer(4 * t * (1 - t), M)
                 + np.outer(t * (2 * t - 1), B))
            dc = np.outer(4 * t - 3, A) + np.outer(4 - 8 * t, M) + np.outer(4 * t - 1, B)
            ref += 0.5 * np.sum(gw[:, None] * np.cross(c, dc), axis=0)
        assert np.max(np.abs(a.sum(0) - ref)) < 1e-13 * (1 + np.abs(ref).max())


def test_quadratic_paraboloid_patch_fluxes():
    """A quadratic triangle whose six points lie on z = f(x, y) = x^2 +
    0.5 x y - 0.3 y^2 over the unit right triangle (edge points above the
    edge midpoints) is exactly that graph, with y_u x y_v = (-f_x, -f_y, 1).
    Closed forms over the triangle: int x^2 = int y^2 = 1/12, int xy = 1/24,
    int x = int y = 1/6."""
    xy = np.array([[0, 0], [1, 0], [0, 1], [.5, 0], [.5, .5], [0, .5]], float)
    f = xy[:, 0] ** 2 + 0.5 * xy[:, 0] * xy[:, 1] - 0.3 * xy[:, 1] ** 2
    P = np.column_stack([xy, f])
    y, a = oracle.nodes(P, np.arange(6, dtype=np.int32)[None], dunavant6())
    assert abs(a[:, 2].sum() - 0.5) < 1e-15
    assert abs(a[:, 0].sum() + (2 / 6 + 0.5 / 6)) < 1e-15
    assert abs(a[:, 1].sum() + (0.5 / 6 - 0.6 / 6)) < 1e-15
    assert abs(np.sum(y[:, 2] * a[:, 2]) - (1 / 12 + 0.5 / 24 - 0.3 / 12)) < 1e-15
    fx = 2 * y[:, 0] + 0.5 * y[:, 1]
    assert np.max(np.abs(y[:, 2] - (y[:, 0] ** 2 + 0.5 * y[:, 0] * y[:, 1] - 0.3 * y[:, 1] ** 2))) < 1e-15
    w = dunavant6()[:, 2]
    assert np.max(np.abs(a[:, 0] + w * fx)) < 1e-15


def test_quadratic_sphere_closed_and_volume_converges_at_fourth_order():
    """Edge points lifted onto the unit sphere: sum a = 0 (closed surface),
    and the divergence-theorem volume (1/3) sum y . a tends to 4 pi / 3 with
    error O(h^4) (the flat skeleton's is O(h^2))."""
    rule = dunavant6()
    eq, ef = [], []
    for lev in (1, 2, 3):
        v, t = icosphere(lev)
        v6, t6 = quadratic_from_flat(v, t, lift=_unit_sphere)
        y6, a6 = oracle.nodes(v6, t6, rule)
        y3, a3 = oracle.nodes(v, t, rule)
        assert np.max(np.abs(a6.sum(0))) < 1e-13
        eq.append(abs(np.sum(y6 * a6) / 3 - 4 * PI / 3))
        ef.append(abs(np.sum(y3 * a3) / 3 - 4 * PI / 3))
    for k in (0, 1):
        assert 12.0 < eq[k] / eq[k + 1] < 20.0, eq
        assert 3.0 < ef[k] / ef[k + 1] < 5.0, ef
    assert eq[-1] < 1e-2 * ef[-1]


def test_quadratic_torus_level_set_closer_to_the_surface():
    """With every skeleton point on a torus, Phi at points of the torus is
    closer to 1/2 for the quadratic skeleton than for the flat one with the
    same corners; deep inside Phi is 1 and far outside 0 in both."""
    rule = dunavant6()
    v3, t3 = torus_mesh(24, 12)
    v6, t6 = torus_mesh(24, 12, quadratic=True)
    s = 0.05
    rng = np.random.default_rng(2)
    th, ph = rng.uniform(0, 2 * PI, 40), rng.uniform(0, 2 * PI, 40)
    xs = np.column_stack([(1 + 0.4 * np.cos(ph)) * np.cos(th), (1 + 0.4 * np.cos(ph)) * np.sin(th),
                          0.4 * np.sin(ph)])
    p3, _ = oracle.evaluate(v3, t3, s, rule, xs)
    p6, _ = oracle.evaluate(v6, t6, s, rule, xs)
    e3, e6 = np.abs(p3 - 0.5).max(), np.abs(p6 - 0.5).max()
    assert e6 < 0.2 * e3 and e6 < 0.05, (e3, e6)
    core = np.array([[1.0, 0, 0], [0, -1.0, 0]])
    far = np.array([[0, 0, 0.0], [3.0, 0, 0]])
    for v, t in ((v3, t3), (v6, t6)):
        pc, _ = oracle.evaluate(v, t, s, rule, core)
        pf, _ = oracle.evaluate(v, t, s, rule, far)
        assert np.max(np.abs(pc - 1)) < 1e-3 and np.max(np.abs(pf)) < 1e-3


# ------------------------------------------------ Hessian and chart curvature
def box_hessian(x, s, lo=0.0, hi=1.0):
    """Hessian of the Gaussian convolution of the box indicator (n, 3, 3):
    products of the 1-D factor f and its first two derivatives."""
    el, eh = np.exp(-(x - lo) ** 2 / (2 * s * s)), np.exp(-(hi - x) ** 2 / (2 * s * s))
    f = 0.5 * (erf((hi - x) / (RT2 * s)) + erf((x - lo) / (RT2 * s)))
    f1 = (el - eh) / (np.sqrt(2 * PI) * s)
    f2 = (-(x - lo) * el - (hi - x) * eh) / (np.sqrt(2 * PI) * s ** 3)
    out = np.empty((len(x), 3, 3))
    for i in range(3):
        for j in range(3):
            d = [f[:, k] for k in range(3)]
            if i == j:
                d[i] = f2[:, i]
            else:
                d[i], d[j] = f1[:, i], f1[:, j]
            out[:, i, j] = d[0] * d[1] * d[2]
    return out


def test_radial_G_vs_incomplete_gamma_and_derivative():
    """G = F'/rho = 15 P(7/2, u^2) / (4 pi rho^7) against mpmath at 40 digits
    across the u = 1.5 switch, and against central differences of F."""
    mp.mp.dps = 40
    for sigma in (0.05, 1.0):
        us = np.concatenate([np.linspace(1e-4, 4, 81), [1.4999999, 1.5, 1.5000001, 5.66, 8, 12]])
        rho = us * RT2 * sigma
        G = oracle.radial_G(rho, sigma)
        for i, u in enumerate(us):
            r = mp.mpf(rho[i])
            Gx = 15 * mp.gammainc(3.5, 0, mp.mpf(u) ** 2, regularized=True) / (4 * mp.pi * r ** 7)
            assert abs(G[i] - float(Gx)) <= 1e-14 * abs(float(Gx)), (sigma, u)
        r = np.linspace(0.3, 6.0, 40) * sigma
        d = 1e-5 * sigma
        fd = (oracle.radial(r + d, sigma)[1] - oracle.radial(r - d, sigma)[1]) / (2 * d) / r
        assert np.max(np.abs(fd - oracle.radial_G(r, sigma)) / np.abs(oracle.radial_G(r, sigma))) < 1e-6


def test_hessian_box_closed_form():
    v, t = cube_mesh(32)
    x = box_targets(48, seed=12)
    B = oracle.sym3(oracle.hessian(v, t, [0.1], dunavant6(), x))
    ref = box_hessian(x, 0.1)
    assert np.abs(B - ref).max() < 1e-10 * np.abs(ref).max()


def test_hessian_is_the_derivative_of_the_gradient_and_harmonic_far_away():
    v, t = star_surface(6, lmax=6, var0=0.1, seed=3)
    sig = 0.5 * triangle_diameters(v, t)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(12, 3)) * 0.6
    B = oracle.sym3(oracle.hessian(v, t, sig, dunavant6(), x))
    d = 1e-4
    for c in range(3):
        e = np.zeros(3)
        e[c] = d
        gp = oracle.evaluate(v, t, sig, dunavant6(), x + e)[1]
        gm = oracle.evaluate(v, t, sig, dunavant6(), x - e)[1]
        gp2 = oracle.evaluate(v, t, sig, dunavant6(), x + 2 * e)[1]
        gm2 = oracle.evaluate(v, t, sig, dunavant6(), x - 2 * e)[1]
        fd = (8 * (gp - gm) - (gp2 - gm2)) / (12 * d)              # fourth-order central difference
        assert np.abs(fd - B[:, :, c]).max() < 1e-7 * np.abs(B).max()
    # an open patch (on a closed surface the far field cancels to rounding):
    # beyond 8 sigma its field is the Laplace double layer, so trace B = 0
    far = np.array([[4.0, 0.5, -1.0], [0.2, -5.0, 0.3]])           # > 8 sigma_max from every node
    Bf = oracle.sym3(oracle.hessian(v, t[:60], sig[:60], dunavant6(), far))
    tr = np.trace(Bf, axis1=1, axis2=2)
    assert np.all(np.abs(tr) < 1e-11 * np.abs(Bf).reshape(2, -1).max(axis=1))


def test_chart_curvature_matches_implicit_surface_and_finite_differences():
    """x_uu, x_uv, x_vv against central differences of the oracle's x_u, x_v
    at shifted chart nodes; the Gaussian and mean curvature from the charts
    equal those of the level set computed from grad Phi and the Hessian alone
    (Goldman's formulas: K = -det [[B, g], [g^T, 0]] / |g|^4, mean =
    (g^T B g - |g|^2 tr B) / (2 |g|^3) for the outward normal -g/|g|)."""
    v, t = star_surface(6, lmax=6, var0=0.1, seed=3)
    sig = 0.5 * triangle_diameters(v, t)
    uv = np.array([[0.2, 0.3], [0.55, 0.15], [0.1, 0.7]])
    sel = np.array([3, 40, 111])
    rule = dunavant6()
    h, x, st, _ = oracle.project(v, t, sig, rule, uv, tau=1e-14, sel=sel)
    assert np.all(st == 0)
    xuu, xuv, xvv, K, Hm = oracle.chart_curvature(v, t, sig, rule, uv, h, sel=sel)
    d = 1e-4
    for k, (du, dv) in enumerate(((d, 0.0), (0.0, d))):
        hp = oracle.project(v, t, sig, rule, uv + [du, dv], tau=1e-14, sel=sel)[0]
        hm = oracle.project(v, t, sig, rule, uv - [du, dv], tau=1e-14, sel=sel)[0]
        up = oracle.chart_geometry(v, t, sig, rule, uv + [du, dv], hp, sel=sel)
        dn = oracle.chart_geometry(v, t, sig, rule, uv - [du, dv], hm, sel=sel)
        fdu, fdv = (up[0] - dn[0]) / (2 * d), (up[1] - dn[1]) / (2 * d)
        an_u, an_v = (xuu, xuv) if k == 0 else (xuv, xvv)
        scale = max(np.abs(xuu).max(), np.abs(xvv).max())
        assert np.abs(fdu - an_u).max() < 1e-5 * scale
        assert np.abs(fdv - an_v).max() < 1e-5 * scale
    _, g = oracle.evaluate(v, t, sig, rule, x)
    B = oracle.sym3(oracle.hessian(v, t, sig, rule, x))
    gn = np.linalg.norm(g, axis=1)
    bord = np.zeros((len(x), 4, 4))
    bord[:, :3, :3], bord[:, :3, 3], bord[:, 3, :3] = B, g, g
    Ki = -np.linalg.det(bord) / gn ** 4
    Hi = (np.einsum("ni,nij,nj->n", g, B, g) - gn ** 2 * np.trace(B, axis1=1, axis2=2)) / (2 * gn ** 3)
    assert np.abs(K - Ki).max() < 1e-9 * np.abs(Ki).max()
    assert np.abs(Hm - Hi).max() < 1e-9 * np.abs(Hi).max()


def test_chart_curvature_sphere():
    """On a fine sphere skeleton with a narrow sigma the level set is a
    sphere of radius |x|: Gaussian curvature 1/|x|^2, mean curvature 1/|x|."""
    v, t = icosphere(4)
    uv = chart_nodes(2)
    sel = np.arange(0, len(t), 97)
    rule = dunavant6()
    h, x, st, _ = oracle.project(v, t, [0.05], rule, uv, sel=sel)
    assert np.all(st == 0)
    _, _, _, K, Hm = oracle.chart_curvature(v, t, [0.05], rule, uv, h, sel=sel)
    R = np.linalg.norm(x, axis=1)
    assert np.abs(K * R ** 2 - 1).max() < 5e-2
    assert np.abs(Hm * R - 1).max() < 2.5e-2


# ------------------------------------------------ multiscale sigma(x) (eq. sigma2)
def graded_cube(n, power=1.6):
    """Unit cube with each coordinate warped by s -> s^power: the faces stay
    planar, the grid is graded (triangle diameters vary about 4x)."""
    v, t = cube_mesh(n)
    return v ** power, t


def test_triangle_diameter_is_the_smallest_enclosing_ball():
    from scipy.optimize import minimize
    rng = np.random.default_rng(8)
    P = rng.normal(size=(12, 3, 3))
    P[::3, 2] = 0.5 * (P[::3, 0] + P[::3, 1]) + 0.05 * rng.normal(size=(4, 3))   # obtuse ones
    v = P.reshape(-1, 3)
    t = np.arange(len(v), dtype=np.int32).reshape(-1, 3)
    _, _, sj, _ = oracle.sigma_field(v, t, np.zeros((1, 3)), lam=1.0)
    for k in range(len(t)):
        A, B, C = P[k]
        f = lambda c: max(np.linalg.norm(c - A), np.linalg.norm(c - B), np.linalg.norm(c - C))
        best = min(minimize(f, x0, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-13, maxiter=20000)).fun
                   for x0 in (P[k].mean(0), A, 0.5 * (A + B)))
        assert abs(sj[k] - 2 * best) < 1e-8 * sj[k]


def test_sigma_field_constant_and_bounds_and_gradient():
    v, t = cube_mesh(6)                        # congruent triangles: sigma(x) = D/lambda
    x = box_targets(50, seed=3)
    s, g, sj, s0 = oracle.sigma_field(v, t, x, lam=2.5)
    D = np.sqrt(2) / 6
    assert np.allclose(sj, D / 2.5, rtol=1e-14) and np.allclose(s, D / 2.5, rtol=1e-13)
    assert np.abs(g).max() < 1e-12 and abs(s0[0] - np.sqrt(5) * D) < 1e-14
    p1, g1, _ = oracle.evaluate_multiscale(v, t, dunavant6(), x, lam=2.5)
    p0, g0 = oracle.evaluate(v, t, [D / 2.5], dunavant6(), x)
    assert np.abs(p1 - p0).max() < 1e-14 and np.abs(g1 - g0).max() < 1e-12
    vg, tg = graded_cube(8)
    xg = np.concatenate([box_targets(40, seed=4), box_targets(10, -3.0, 4.0, seed=5) * 30])   # some far away
    s, g, sj, s0 = oracle.sigma_field(vg, tg, xg, lam=2.5, sigma0=0.1)
    assert np.all(s >= sj.min() * (1 - 1e-14)) and np.all(s <= sj.max() * (1 + 1e-14))
    d = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = d
        fd = (oracle.sigma_field(vg, tg, xg + e, 2.5, 0.1)[0] - oracle.sigma_field(vg, tg, xg - e, 2.5, 0.1)[0]) / (2 * d)
        assert np.abs(fd - g[:, c]).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_multiscale_phi_is_the_box_convolution_at_sigma_x():
    """For each x, Phi(x) is the Gaussian convolution of the indicator with
    width sigma(x), evaluated at x: the box closed form at sigma(x)."""
    v, t = graded_cube(24)
    x = box_targets(48, seed=13)
    phi, g, s = oracle.evaluate_multiscale(v, t, dunavant6(), x, lam=0.5, sigma0=0.2)
    P, _ = box_closed(x, s[:, None])
    assert np.abs(phi - P).max() < 1e-9


def test_multiscale_gradient_includes_the_sigma_term():
    """grad Phi against differences of Phi with sigma(x) re-evaluated at the
    shifted points; without the (dPhi/dsigma) grad sigma term (or with its
    sign flipped) the difference is far above the bar."""
    v, t = graded_cube(8)
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.2, 1.2, size=(20, 3))
    rule = dunavant6()
    p, g, s = oracle.evaluate_multiscale(v, t, rule, x, lam=2.5, sigma0=0.15)
    d = 1e-5
    fd = np.empty_like(g)
    for c in range(3):
        e = np.zeros(3)
        e[c] = d
        fd[:, c] = (oracle.evaluate_multiscale(v, t, rule, x + e, 2.5, 0.15)[0]
                    - oracle.evaluate_multiscale(v, t, rule, x - e, 2.5, 0.15)[0]) / (2 * d)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err < 1e-7, err
    # the same sums at the fixed width sigma(x_i): the gradient without the term
    g_fixed = np.concatenate([oracle.evaluate(v, t, [s[i]], rule, x[i:i + 1])[1] for i in range(len(x))])
    assert np.abs(fd - g_fixed).max() / np.abs(g).max() > 1e-4


def test_quadratic_refinement_keeps_the_surface():
    """refine_1to4_quadratic: the refined skeleton is closed, shares its edge
    points, and encloses exactly the parent's volume with the same (zero)
    vector area: its patches are pieces of the parent patches."""
    from workloads import refine_1to4_quadratic, mesh_check
    v, t = torus_mesh(12, 6, quadratic=True)
    rule = dunavant6()
    y, a = oracle.nodes(v, t, rule)
    vol0 = np.sum(y * a) / 3
    for _ in range(2):
        v, t = refine_1to4_quadratic(v, t)
        closed, _ = mesh_check(v, np.ascontiguousarray(t[:, :3]))
        assert closed and len(np.unique(t)) == len(v)
        y, a = oracle.nodes(v, t, rule)
        assert abs(np.sum(y * a) / 3 - vol0) < 1e-13 and np.abs(a.sum(0)).max() < 1e-13


def _two_obtuse_triangles():
    """Two obtuse triangles with exact centroids and diameters: for an obtuse
    triangle the smallest enclosing ball has the longest edge as diameter.
    T1: base 0.4 along x, apex 0.03 above its midpoint -> c1 = (0, 0.01, 0),
    D1 = 0.4; T2: base 0.8, apex 0.06 above -> c2 = (0.9, 0.32, 0.2), D2 = 0.8."""
    v = np.array([[-0.2, 0.0, 0.0], [0.2, 0.0, 0.0], [0.0, 0.03, 0.0],
                  [0.5, 0.3, 0.2], [1.3, 0.3, 0.2], [0.9, 0.36, 0.2]])
    t = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    c = np.array([[0.0, 0.01, 0.0], [0.9, 0.32, 0.2]])
    return v, t, c, np.array([0.4, 0.8])


def test_sigma_blend_exact_weights_three_to_one():
    """eq. sigma2 with two centroids: the weights are exp(-|x - c_j|^2 /
    (2 sigma0^2)), so where |x - c2|^2 - |x - c1|^2 = 2 sigma0^2 ln 3 they are
    exactly 3 : 1 and sigma(x) = (3 sigma_1 + sigma_2) / 4, whatever the offset
    of x across the line c1 c2.  A width sigma0^2 in place of 2 sigma0^2 gives
    9 : 1 (sigma = 0.22 here instead of 0.25), and a weight centred on the
    midpoint of the longest edge (the enclosing-ball centre) or on the
    circumcentre instead of the centroid moves the ratio away from 3."""
    v, t, c, D = _two_obtuse_triangles()
    lam, s0 = 2.0, 0.5
    s1, s2 = D / lam
    e = c[1] - c[0]
    L2 = e @ e
    s = 0.5 * (1.0 - 2.0 * s0 * s0 * np.log(3.0) / L2)      # x = c1 + s e on the line
    perp = np.cross(e, [0.0, 0.0, 1.0])
    perp2 = np.cross(e, perp)
    x = np.array([c[0] + s * e + a * perp + b * perp2 for a, b in ((0, 0), (0.3, 0), (-0.2, 0.5), (1.1, -0.7))])
    sig, _, sj, s0_used = oracle.sigma_field(v, t, x, lam=lam, sigma0=s0)
    assert np.allclose(sj, [s1, s2], rtol=1e-15, atol=0) and s0_used[0] == s0
    assert np.abs(sig - (3 * s1 + s2) / 4).max() < 1e-14
    # the pin separates the readings: 9 : 1 with the narrower width, and another
    # ratio with the enclosing-ball centres (midpoints of the longest edges)
    assert abs((9 * s1 + s2) / 10 - (3 * s1 + s2) / 4) > 1e-2
    m = np.array([[0.0, 0.0, 0.0], [0.9, 0.3, 0.2]])
    r = np.exp(-(((x - m[0]) ** 2).sum(1) - ((x - m[1]) ** 2).sum(1)) / (2 * s0 * s0))
    assert np.abs((r * s1 + s2) / (r + 1) - (3 * s1 + s2) / 4).min() > 1e-4


def test_sigma_blend_midpoint_value_and_gradient():
    """At any point equidistant from the two centroids the weights are equal:
    sigma = (sigma_1 + sigma_2) / 2, and differentiating eq. sigma2 there gives
    grad sigma = (sigma_2 - sigma_1) (c2 - c1) / (4 sigma0^2) (the components
    across c1 c2 cancel).  With the width sigma0^2 the gradient doubles."""
    v, t, c, D = _two_obtuse_triangles()
    lam, s0 = 2.0, 0.45
    s1, s2 = D / lam
    e = c[1] - c[0]
    perp = np.cross(e, [0.0, 1.0, 0.0])
    perp2 = np.cross(e, perp)
    mid = 0.5 * (c[0] + c[1])
    x = np.array([mid + a * perp + b * perp2 for a, b in ((0, 0), (0.4, 0), (0, -0.3), (-0.5, 0.25))])
    sig, g, _, _ = oracle.sigma_field(v, t, x, lam=lam, sigma0=s0)
    assert np.abs(sig - 0.5 * (s1 + s2)).max() < 1e-15
    want = (s2 - s1) * e / (4 * s0 * s0)
    assert np.abs(g - want).max() < 1e-14 * np.abs(want).max()


def test_sigma_blend_nearest_centroid_dominates_far_away():
    """Far from both centroids along c1 -> c2 the weight ratio exp(-(|x-c1|^2 -
    |x-c2|^2) / (2 sigma0^2)) underflows in FP64: sigma(x) must then be the
    nearest triangle's sigma_j (the weights are taken relative to the largest,
    so there is no 0/0), with zero gradient."""
    v, t, c, D = _two_obtuse_triangles()
    e = (c[1] - c[0]) / np.linalg.norm(c[1] - c[0])
    x = np.array([c[1] + 40.0 * e, c[0] - 40.0 * e])
    sig, g, sj, _ = oracle.sigma_field(v, t, x, lam=2.0, sigma0=0.2)
    assert sig[0] == sj[1] and sig[1] == sj[0]
    assert np.abs(g).max() == 0.0


# ------------------------------------- curved chart bases (quadratic skeletons)
def test_quadratic_shape_functions_interpolate_and_differentiate():
    """The six shape functions are 1 at their own point and 0 at the other
    five (corners (0,0), (1,0), (0,1), edge midpoints), sum to 1, and their
    first and second derivatives equal central differences of them."""
    pts = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]], float)
    N, Nu, Nv, Nuu, Nuv, Nvv = oracle.quad_shape(pts[:, 0], pts[:, 1])
    assert np.allclose(N, np.eye(6), atol=1e-15)
    rng = np.random.default_rng(2)
    u, v = rng.uniform(0.05, 0.4, 20), rng.uniform(0.05, 0.4, 20)
    assert np.allclose(oracle.quad_shape(u, v)[0].sum(1), 1.0, atol=1e-15)
    d = 1e-5
    f = lambda a, b: oracle.quad_shape(a, b)[0]
    _, Nu, Nv, Nuu, Nuv, Nvv = oracle.quad_shape(u, v)
    assert np.abs((f(u + d, v) - f(u - d, v)) / (2 * d) - Nu).max() < 1e-9
    assert np.abs((f(u, v + d) - f(u, v - d)) / (2 * d) - Nv).max() < 1e-9
    g = lambda a, b: oracle.quad_shape(a, b)[1]
    assert np.abs((g(u + d, v) - g(u - d, v)) / (2 * d) - Nuu).max() < 1e-8
    assert np.abs((g(u, v + d) - g(u, v - d)) / (2 * d) - Nuv).max() < 1e-8
    h = lambda a, b: oracle.quad_shape(a, b)[2]
    assert np.abs((h(u, v + d) - h(u, v - d)) / (2 * d) - Nvv).max() < 1e-8


def test_curved_pseudonormals():
    """Curved-vertex pseudonormals (eq. mkvertexpn on the quadratic patches):
    with straight edges (edge points at the midpoints) each patch is its
    flat triangle, so they equal the flat pseudonormals; on a sphere whose
    edge points are lifted onto it they point radially to a fraction of the
    flat ones' deviation (the corner normals are those of the curved patch)."""
    v, t = icosphere(2)
    vq, tq = quadratic_from_flat(v, t)
    assert np.abs(oracle.pseudonormals(vq, tq, curved=True)[:len(v)] - oracle.pseudonormals(v, t)).max() < 1e-14
    vs, ts = quadratic_from_flat(v, t, lift=lambda p: p / np.linalg.norm(p, axis=1, keepdims=True))
    Hc = oracle.pseudonormals(vs, ts, curved=True)[:len(v)]
    Hf = oracle.pseudonormals(vs, ts, curved=False)[:len(v)]
    ang = lambda H: np.degrees(np.arccos(np.clip(np.sum(H * v, 1) / np.linalg.norm(H, axis=1)
                                                 / np.linalg.norm(v, axis=1), -1, 1)))
    assert ang(Hc).max() < 0.2 * ang(Hf).max() and ang(Hf).max() > 0.1


def test_curved_charts_projection():
    """Chart bases on the curved patches: the projected points lie on Phi = 1/2
    (re-evaluated by the direct sum); with straight-edged quadratic triangles
    they are the flat-based charts; on a torus whose six points per triangle
    lie on it the chart base T = x - h H lies on the torus up to the patch's
    interpolation error, far closer than the corner triangles' chords."""
    v, t = torus_mesh(12, 6, quadratic=True)
    D = triangle_diameters(v, np.ascontiguousarray(t[:, :3]))
    sig = D / 4.0
    uv = chart_nodes(2)
    sel = np.arange(0, len(t), 11)
    rule = dunavant6()
    hc, xc, stc, _ = oracle.project(v, t, sig, rule, uv, tau=1e-13, sel=sel, curved=True)
    hf, xf, stf, _ = oracle.project(v, t, sig, rule, uv, tau=1e-13, sel=sel, curved=False)
    assert np.all(stc == 0) and np.all(stf == 0)
    p, _ = oracle.evaluate(v, t, sig, rule, xc)
    assert np.abs(p - 0.5).max() < 1e-12
    def base(x, h, curved):
        Hv = oracle.pseudonormals(v, t, curved)
        c = t[sel][:, :3]
        u_, w_ = uv[None, :, 0:1], uv[None, :, 1:2]
        H = Hv[c[:, 0]][:, None] + u_ * (Hv[c[:, 1]] - Hv[c[:, 0]])[:, None] + w_ * (Hv[c[:, 2]] - Hv[c[:, 0]])[:, None]
        return x - h[:, None] * H.reshape(-1, 3)
    torus_dist = lambda p: np.abs(np.hypot(np.hypot(p[:, 0], p[:, 1]) - 1.0, p[:, 2]) - 0.4)
    dc, df = torus_dist(base(xc, hc, True)), torus_dist(base(xf, hf, False))
    assert dc.max() < 0.05 * df.max()
    vf, tf = torus_mesh(12, 6)
    vq, tq = quadratic_from_flat(vf, tf)                         # straight edges
    sf = triangle_diameters(vf, tf) / 4.0
    a = oracle.project(vq, tq, sf, rule, uv, tau=1e-13, sel=sel, curved=True)
    b = oracle.project(vq, tq, sf, rule, uv, tau=1e-13, sel=sel, curved=False)
    assert np.abs(a[0] - b[0]).max() < 1e-12 * sf.max() and np.array_equal(a[2], b[2])


def test_curved_chart_tangents_and_second_derivatives():
    """x_u, x_v of the curved charts against central differences of the
    oracle's own curved Newton charts x(u +- d, v), x(u, v +- d), and x_uu,
    x_uv, x_vv against differences of x_u, x_v: a missing T_u, T_uu term of
    the patch (or the flat T_u in its place) fails it."""
    v, t = torus_mesh(12, 6, quadratic=True)
    sig = triangle_diameters(v, np.ascontiguousarray(t[:, :3])) / 4.0
    uv = np.array([[0.2, 0.3], [0.55, 0.15], [0.1, 0.7]])
    sel = np.array([3, 40, 111])
    rule = dunavant6()
    h, x, st, _ = oracle.project(v, t, sig, rule, uv, tau=1e-14, sel=sel, curved=True)
    assert np.all(st == 0)
    xu, xv, da, nrm = oracle.chart_geometry(v, t, sig, rule, uv, h, sel=sel, curved=True)
    xuu, xuv, xvv, K, Hm = oracle.chart_curvature(v, t, sig, rule, uv, h, sel=sel, curved=True)
    d = 1e-4
    for k, (du, dv) in enumerate(((d, 0.0), (0.0, d))):
        hp, up_x = oracle.project(v, t, sig, rule, uv + [du, dv], tau=1e-14, sel=sel, curved=True)[:2]
        hm, dn_x = oracle.project(v, t, sig, rule, uv - [du, dv], tau=1e-14, sel=sel, curved=True)[:2]
        fd = (up_x - dn_x) / (2 * d)
        an = xu if k == 0 else xv
        assert (np.linalg.norm(fd - an, axis=1) / np.linalg.norm(an, axis=1)).max() < 1e-6
        up = oracle.chart_geometry(v, t, sig, rule, uv + [du, dv], hp, sel=sel, curved=True)
        dn = oracle.chart_geometry(v, t, sig, rule, uv - [du, dv], hm, sel=sel, curved=True)
        fdu, fdv = (up[0] - dn[0]) / (2 * d), (up[1] - dn[1]) / (2 * d)
        an_u, an_v = (xuu, xuv) if k == 0 else (xuv, xvv)
        scale = max(np.abs(xuu).max(), np.abs(xvv).max())
        assert np.abs(fdu - an_u).max() < 1e-5 * scale
        assert np.abs(fdv - an_v).max() < 1e-5 * scale
    assert np.abs(np.sum(xu * nrm, axis=1)).max() < 1e-10 * np.linalg.norm(xu, axis=1).max()
