"""CPU oracle (test infrastructure only).

A plain FP64 OpenMP C implementation of the direct discrete sum for Phi and
grad Phi, the vertex pseudonormals and the Newton chart projection, written
from the paper (see ``oracle.c`` for the equations it follows).  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
import this package; the product library never touches it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_radial.argtypes = [P, i64, f64, P, P]
        L.oracle_nodes.argtypes = [P, P, i32, i64, P, i32, P, P]
        L.oracle_eval.argtypes = [P, P, i32, i64, P, P, i64, P, i32, P, P, i64, P, P, P, P, ctypes.c_int]
        L.oracle_pseudonormals.argtypes = [P, i64, P, i64, P]
        L.oracle_radial_G.argtypes = [P, i64, f64, P]
        L.oracle_hessian.argtypes = [P, P, i32, i64, P, P, i64, P, i32, P, P, i64, P, ctypes.c_int]
        L.oracle_sigma_field.argtypes = [P, P, i32, i64, P, i32, f64, f64, P, P, i64, P, P, P, P]
        L.oracle_eval_multiscale.argtypes = [P, P, i32, i64, P, P, i32, P, P, i64, P, P, P, P, ctypes.c_int]
        L.oracle_project.argtypes = [P, i64, P, i32, i64, P, i32, P, i64, P, i32, P, i32, P, i64,
                                     f64, i32, i32, P, P, P, P, ctypes.c_int]
        L.oracle_pseudonormals_curved.argtypes = [P, i64, P, i64, P]
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads():
    return _load().oracle_threads()


def radial(rho, sigma):
    """K(rho) and F(rho) = K'(rho)/rho for one sigma (see oracle.c)."""
    rho = _f64(rho).ravel()
    K, F = np.empty_like(rho), np.empty_like(rho)
    _load().oracle_radial(_p(rho), rho.size, float(sigma), _p(K), _p(F))
    return K, F


def _tris(tris):
    """Triangle index array and its width: (ntris, 3) flat, (ntris, 6)
    quadratic (corners P1 P2 P3, then the edge points of P1P2, P2P3, P3P1)."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    if tris.ndim != 2 or tris.shape[1] not in (3, 6):
        raise ValueError("tris must be (ntris, 3) or (ntris, 6)")
    return tris, tris.shape[1]


def radial_G(rho, sigma):
    """G(rho) = F'(rho)/rho, the Hessian's third radial function (see oracle.c)."""
    rho = _f64(rho).ravel()
    G = np.empty_like(rho)
    _load().oracle_radial_G(_p(rho), rho.size, float(sigma), _p(G))
    return G


def nodes(verts, tris, rule):
    """Quadrature nodes y (N, 3) and weighted area normals a = w J (N, 3)."""
    verts, rule = _f64(verts), _f64(rule)
    tris, nvt = _tris(tris)
    n = len(tris) * len(rule)
    y, a = np.empty((n, 3)), np.empty((n, 3))
    _load().oracle_nodes(_p(verts), _p(tris), nvt, len(tris), _p(rule), len(rule), _p(y), _p(a))
    return y, a


def evaluate(verts, tris, sigma, rule, x, tri_offsets=None, x_mesh=None,
             with_abs=False, nthreads=0):
    """Phi (n,) and grad Phi (n, 3) by the direct FP64 sum over all nodes."""
    verts, rule, x = _f64(verts), _f64(rule), _f64(x).reshape(-1, 3)
    sigma = _f64(np.atleast_1d(sigma))
    tris, nvt = _tris(tris)
    off = None if tri_offsets is None else np.ascontiguousarray(tri_offsets, dtype=np.int64)
    xm = None if x_mesh is None else np.ascontiguousarray(x_mesh, dtype=np.int32)
    n = len(x)
    phi, grad = np.empty(n), np.empty((n, 3))
    aphi = np.empty(n) if with_abs else None
    agrad = np.empty(n) if with_abs else None
    _load().oracle_eval(_p(verts), _p(tris), nvt, len(tris), _p(off), _p(sigma), sigma.size,
                        _p(rule), len(rule), _p(x), _p(xm), n, _p(phi), _p(grad),
                        _p(aphi), _p(agrad), int(nthreads))
    if with_abs:
        return phi, grad, aphi, agrad
    return phi, grad


def hessian(verts, tris, sigma, rule, x, tri_offsets=None, x_mesh=None, nthreads=0):
    """Hessian of Phi at x (n, 3) by the direct FP64 sum: (n, 6) as xx, xy,
    xz, yy, yz, zz."""
    verts, rule, x = _f64(verts), _f64(rule), _f64(x).reshape(-1, 3)
    sigma = _f64(np.atleast_1d(sigma))
    tris, nvt = _tris(tris)
    off = None if tri_offsets is None else np.ascontiguousarray(tri_offsets, dtype=np.int64)
    xm = None if x_mesh is None else np.ascontiguousarray(x_mesh, dtype=np.int32)
    out = np.empty((len(x), 6))
    _load().oracle_hessian(_p(verts), _p(tris), nvt, len(tris), _p(off), _p(sigma), sigma.size,
                           _p(rule), len(rule), _p(x), _p(xm), len(x), _p(out), int(nthreads))
    return out


def sigma_field(verts, tris, x, lam=2.5, sigma0=0.0, tri_offsets=None, x_mesh=None):
    """Multiscale width of eq. sigma2 at x (n, 3): returns sigma(x) (n,),
    grad sigma (n, 3), sigma_j = D_j / lambda (ntris,) and sigma0 per mesh
    (sqrt(5) max_j D_j of the mesh when sigma0 <= 0)."""
    verts, x = _f64(verts), _f64(x).reshape(-1, 3)
    tris, nvt = _tris(tris)
    off = None if tri_offsets is None else np.ascontiguousarray(tri_offsets, dtype=np.int64)
    nmesh = 1 if off is None else len(off) - 1
    xm = None if x_mesh is None else np.ascontiguousarray(x_mesh, dtype=np.int32)
    s, g = np.empty(len(x)), np.empty((len(x), 3))
    sj, s0 = np.empty(len(tris)), np.empty(nmesh)
    _load().oracle_sigma_field(_p(verts), _p(tris), nvt, len(tris), _p(off), nmesh, float(lam),
                               float(sigma0), _p(x), _p(xm), len(x), _p(s), _p(g), _p(sj), _p(s0))
    return s, g, sj, s0


def evaluate_multiscale(verts, tris, rule, x, lam=2.5, sigma0=0.0, tri_offsets=None, x_mesh=None,
                        nthreads=0):
    """Phi (n,), grad Phi (n, 3) and sigma(x) (n,) with the target-attached
    width of eq. basemodelk / sigma2, by the direct FP64 sum."""
    verts, rule, x = _f64(verts), _f64(rule), _f64(x).reshape(-1, 3)
    tris, nvt = _tris(tris)
    off = None if tri_offsets is None else np.ascontiguousarray(tri_offsets, dtype=np.int64)
    xm = None if x_mesh is None else np.ascontiguousarray(x_mesh, dtype=np.int32)
    s, g, _, _ = sigma_field(verts, tris, x, lam, sigma0, tri_offsets, x_mesh)
    phi, grad = np.empty(len(x)), np.empty((len(x), 3))
    _load().oracle_eval_multiscale(_p(verts), _p(tris), nvt, len(tris), _p(off), _p(rule), len(rule),
                                   _p(x), _p(xm), len(x), _p(s), _p(g), _p(phi), _p(grad), int(nthreads))
    return phi, grad, s


def sym3(h6):
    """(n, 6) xx, xy, xz, yy, yz, zz -> (n, 3, 3)."""
    h6 = np.asarray(h6)
    i = np.array([[0, 1, 2], [1, 3, 4], [2, 4, 5]])
    return h6[:, i]


def pseudonormals(verts, tris, curved=False):
    """Vertex pseudonormals (eq. mkvertexpn): of the flat triangles (the
    corners of a quadratic skeleton), or with ``curved`` of the quadratic
    patches (tris (n, 6)): corner normals y_u x y_v and corner angles of the
    curved triangles."""
    verts = _f64(verts)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    H = np.empty((len(verts), 3))
    if curved and tris.shape[1] == 6:
        _load().oracle_pseudonormals_curved(_p(verts), len(verts), _p(tris), len(tris), _p(H))
    else:
        tris = np.ascontiguousarray(tris[:, :3])
        _load().oracle_pseudonormals(_p(verts), len(verts), _p(tris), len(tris), _p(H))
    return H


def quad_shape(u, v):
    """Quadratic Lagrange shape functions of the six-point triangle (corners,
    then the edge points of P1P2, P2P3, P3P1) at (u, v) and their first and
    second derivatives: N, Nu, Nv (..., 6) and the constants Nuu, Nuv, Nvv (6,)."""
    u, v = np.asarray(u, float), np.asarray(v, float)
    w = 1.0 - u - v
    N = np.stack([w * (2 * w - 1), u * (2 * u - 1), v * (2 * v - 1), 4 * u * w, 4 * u * v, 4 * v * w], -1)
    z = np.zeros_like(u)
    Nu = np.stack([1 - 4 * w, 4 * u - 1, z, 4 * (w - u), 4 * v, -4 * v], -1)
    Nv = np.stack([1 - 4 * w, z, 4 * v - 1, -4 * u, 4 * u, 4 * (w - v)], -1)
    Nuu = np.array([4.0, 4.0, 0.0, -8.0, 0.0, 0.0])
    Nuv = np.array([4.0, 0.0, 0.0, -4.0, 4.0, -4.0])
    Nvv = np.array([4.0, 0.0, 4.0, 0.0, 0.0, -8.0])
    return N, Nu, Nv, Nuu, Nuv, Nvv


def chart_frame(verts, tris, sel, chart_uv, curved=False):
    """Chart base T(u, v) of eq. tparam and its derivatives at the chart nodes
    of the triangles ``sel``: T, Tu, Tv, Tuu, Tuv, Tvv of shape (nsel, np, 3).
    Flat (the corner triangle): T linear, second derivatives zero; with
    ``curved`` and six-point triangles: the quadratic patch."""
    verts = _f64(verts)
    tris = np.asarray(tris)
    uv = _f64(chart_uv).reshape(-1, 2)
    t = tris[np.asarray(sel, dtype=np.int64)]
    if curved and tris.shape[1] == 6:
        P = verts[t]                                            # (nsel, 6, 3)
        N, Nu, Nv, Nuu, Nuv, Nvv = quad_shape(uv[:, 0], uv[:, 1])
        T = np.einsum("ik,skc->sic", N, P)
        Tu = np.einsum("ik,skc->sic", Nu, P)
        Tv = np.einsum("ik,skc->sic", Nv, P)
        Tuu = np.broadcast_to(np.einsum("k,skc->sc", Nuu, P)[:, None], T.shape)
        Tuv = np.broadcast_to(np.einsum("k,skc->sc", Nuv, P)[:, None], T.shape)
        Tvv = np.broadcast_to(np.einsum("k,skc->sc", Nvv, P)[:, None], T.shape)
        return T, Tu, Tv, Tuu, Tuv, Tvv
    P1, P2, P3 = verts[t[:, 0]][:, None], verts[t[:, 1]][:, None], verts[t[:, 2]][:, None]
    u, v = uv[None, :, 0:1], uv[None, :, 1:2]
    T = P1 + u * (P2 - P1) + v * (P3 - P1)
    Tu, Tv = np.broadcast_to(P2 - P1, T.shape), np.broadcast_to(P3 - P1, T.shape)
    z = np.zeros_like(T)
    return T, Tu, Tv, z, z, z


def project(verts, tris, sigma, rule, chart_uv, tau=1e-12, max_iter=40, sel=None,
            tri_offsets=None, nthreads=0, curved=False):
    """Newton chart projection onto Phi = 1/2 for the chart nodes of the
    triangles ``sel`` (all if None).  Returns h, x, status, iters with
    index k * np + i.  ``curved``: on a quadratic skeleton, chart bases on the
    curved patches (see oracle_project)."""
    verts, rule, uv = _f64(verts), _f64(rule), _f64(chart_uv).reshape(-1, 2)
    sigma = _f64(np.atleast_1d(sigma))
    tris, nvt = _tris(tris)
    off = None if tri_offsets is None else np.ascontiguousarray(tri_offsets, dtype=np.int64)
    nmesh = 0 if off is None else len(off) - 1
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    nsel = len(tris) if s is None else len(s)
    npn = len(uv)
    tot = nsel * npn
    h, xo = np.empty(tot), np.empty((tot, 3))
    st, it = np.empty(tot, np.int8), np.empty(tot, np.int8)
    _load().oracle_project(_p(verts), len(verts), _p(tris), nvt, len(tris), _p(off), nmesh,
                           _p(sigma), sigma.size, _p(rule), len(rule), _p(uv), npn,
                           _p(s), nsel, float(tau), int(max_iter), int(bool(curved)), _p(h), _p(xo),
                           _p(st), _p(it), int(nthreads))
    return h, xo, st, it


def chart_geometry(verts, tris, sigma, rule, chart_uv, h, sel=None, tri_offsets=None, nthreads=0, curved=False):
    """Tangents x_u, x_v, area element |x_u x x_v| and outward unit normal of
    the charts x = T + h H (section 3.1, eq. chart, u_vector, U_vector_2,
    v_vector, v_vector_2, eq. da) at the chart nodes of the triangles ``sel``
    (all if None), for the given h (index k * np + i over sel).  T and H are
    the linear maps of eq. tparam and mkpseudovec (vertex pseudonormals of eq.
    mkvertexpn), on the corner triangles when ``tris`` is quadratic, or with
    ``curved`` T is the quadratic patch and H interpolates its curved-vertex
    pseudonormals; grad Phi comes from ``evaluate``; the normal is
    -grad Phi / |grad Phi|, outward because Phi grows inward."""
    verts = _f64(verts)
    tris, _ = _tris(tris)
    corner = np.ascontiguousarray(tris[:, :3])
    uv = _f64(chart_uv).reshape(-1, 2)
    s = np.arange(len(tris)) if sel is None else np.asarray(sel, dtype=np.int64)
    npn = len(uv)
    Hv = pseudonormals(verts, tris, curved)
    t = corner[s]
    H1, H2, H3 = Hv[t[:, 0]][:, None], Hv[t[:, 1]][:, None], Hv[t[:, 2]][:, None]
    u, v = uv[None, :, 0:1], uv[None, :, 1:2]
    T, Tu, Tv, _, _, _ = chart_frame(verts, tris, s, uv, curved)
    H = H1 + u * (H2 - H1) + v * (H3 - H1)
    hh = _f64(h).reshape(len(s), npn, 1)
    x = T + hh * H
    xm = None
    if tri_offsets is not None:
        mesh = np.searchsorted(np.asarray(tri_offsets), s, side="right") - 1
        xm = np.repeat(mesh, npn).astype(np.int32)
    _, g = evaluate(verts, tris, sigma, rule, x.reshape(-1, 3), tri_offsets=tri_offsets, x_mesh=xm,
                    nthreads=nthreads)
    g = g.reshape(len(s), npn, 3)
    Hu, Hvv = H2 - H1, H3 - H1
    den = np.sum(H * g, axis=-1, keepdims=True)
    au, av = Tu + hh * Hu, Tv + hh * Hvv
    hu = -np.sum(au * g, axis=-1, keepdims=True) / den
    hv = -np.sum(av * g, axis=-1, keepdims=True) / den
    xu, xv = au + hu * H, av + hv * H
    da = np.linalg.norm(np.cross(xu, xv), axis=-1)
    nrm = -g / np.linalg.norm(g, axis=-1, keepdims=True)
    return xu.reshape(-1, 3), xv.reshape(-1, 3), da.reshape(-1), nrm.reshape(-1, 3)


def chart_curvature(verts, tris, sigma, rule, chart_uv, h, sel=None, tri_offsets=None, nthreads=0, curved=False):
    """Second derivatives of the charts x = T + h H and the curvatures of the
    surface at the chart nodes (section 3.1, eq. uu_vector, uu_vector_aux1,
    uu_vector_aux2 and the analogous uv, vv expressions).  H is linear on the
    triangle (H_uu = 0) and so is T on a flat base (T_uu = 0); with ``curved``
    T is the quadratic patch, whose second derivatives are constant.  With
    w_u = x_u, w_v = x_v, g = grad Phi, B = grad grad Phi, D = g . H:
        h_uu = -(w_u B w_u + 2 h_u g.H_u + g.T_uu) / D,
                                                 x_uu = T_uu + 2 h_u H_u + h_uu H,
        h_uv = -(w_u B w_v + g.(h_u H_v + h_v H_u) + g.T_uv) / D,
                                                 x_uv = T_uv + h_u H_v + h_v H_u + h_uv H,
        h_vv = -(w_v B w_v + 2 h_v g.H_v + g.T_vv) / D,
                                                 x_vv = T_vv + 2 h_v H_v + h_vv H.
    (The printed eq. uu_vector groups its last terms as 2 h_u + h_uu H_u; the
    derivative of eq. u_vector, and eq. uu_vector_aux1 itself, give
    2 h_u H_u + h_uu H.)  With the outward normal n = -g/|g| and the first and
    second fundamental forms E, F, G and L = x_uu.n, M = x_uv.n, N = x_vv.n:
    Gaussian curvature (LN - M^2)/(EG - F^2), mean curvature
    -(EN - 2FM + GL)/(2(EG - F^2)) (1/R on a sphere of radius R).
    Returns xuu, xuv, xvv (N, 3), gauss (N), mean (N)."""
    verts = _f64(verts)
    tris, _ = _tris(tris)
    corner = np.ascontiguousarray(tris[:, :3])
    uv = _f64(chart_uv).reshape(-1, 2)
    s = np.arange(len(tris)) if sel is None else np.asarray(sel, dtype=np.int64)
    npn = len(uv)
    Hv = pseudonormals(verts, tris, curved)
    t = corner[s]
    H1, H2, H3 = Hv[t[:, 0]][:, None], Hv[t[:, 1]][:, None], Hv[t[:, 2]][:, None]
    u, v = uv[None, :, 0:1], uv[None, :, 1:2]
    T, Tu, Tv, Tuu, Tuv, Tvv = chart_frame(verts, tris, s, uv, curved)
    H = H1 + u * (H2 - H1) + v * (H3 - H1)
    hh = _f64(h).reshape(len(s), npn, 1)
    x = (T + hh * H).reshape(-1, 3)
    xm = None
    if tri_offsets is not None:
        mesh = np.searchsorted(np.asarray(tri_offsets), s, side="right") - 1
        xm = np.repeat(mesh, npn).astype(np.int32)
    _, g = evaluate(verts, tris, sigma, rule, x, tri_offsets=tri_offsets, x_mesh=xm, nthreads=nthreads)
    B = sym3(hessian(verts, tris, sigma, rule, x, tri_offsets=tri_offsets, x_mesh=xm, nthreads=nthreads))
    g = g.reshape(len(s), npn, 3)
    B = B.reshape(len(s), npn, 3, 3)
    Hu, Hw = H2 - H1, H3 - H1
    Hu, Hw = np.broadcast_to(Hu, g.shape), np.broadcast_to(Hw, g.shape)
    dot = lambda a, b: np.sum(a * b, axis=-1, keepdims=True)
    D = dot(H, g)
    hu = -dot(Tu + hh * Hu, g) / D
    hv = -dot(Tv + hh * Hw, g) / D
    xu = Tu + hu * H + hh * Hu
    xv = Tv + hv * H + hh * Hw
    quad = lambda a, b: np.einsum("...i,...ij,...j->...", a, B, b)[..., None]
    huu = -(quad(xu, xu) + 2 * hu * dot(g, Hu) + dot(g, Tuu)) / D
    huv = -(quad(xu, xv) + dot(g, hu * Hw + hv * Hu) + dot(g, Tuv)) / D
    hvv = -(quad(xv, xv) + 2 * hv * dot(g, Hw) + dot(g, Tvv)) / D
    xuu = Tuu + 2 * hu * Hu + huu * H
    xuv = Tuv + hu * Hw + hv * Hu + huv * H
    xvv = Tvv + 2 * hv * Hw + hvv * H
    n = -g / np.linalg.norm(g, axis=-1, keepdims=True)
    E, F, G = dot(xu, xu), dot(xu, xv), dot(xv, xv)
    L, M, N = dot(xuu, n), dot(xuv, n), dot(xvv, n)
    det = E * G - F * F
    gauss = (L * N - M * M) / det
    mean = -(E * N - 2 * F * M + G * L) / (2 * det)
    return (xuu.reshape(-1, 3), xuv.reshape(-1, 3), xvv.reshape(-1, 3), gauss.reshape(-1),
            mean.reshape(-1))


def koornwinder(uv, p):
    """Koornwinder (Dubiner) orthogonal basis of the polynomials of total
    degree <= p on the standard simplex (section 3.3), at points uv (n, 2):
    (n, (p+1)(p+2)/2), columns ordered by (m, n), m + n <= p, with
    K_mn(u, v) = P_m((2u + v - 1)/(1 - v)) (1 - v)^m P_n^(2m+1, 0)(2v - 1)
    (Legendre P_m, Jacobi P_n^(a, b); points with v < 1)."""
    from scipy.special import eval_jacobi, eval_legendre
    uv = _f64(uv).reshape(-1, 2)
    u, v = uv[:, 0], uv[:, 1]
    t = 1.0 - v
    cols = []
    for m in range(p + 1):
        lm = eval_legendre(m, (2 * u + v - 1) / t) * t ** m
        for n in range(p + 1 - m):
            cols.append(lm * eval_jacobi(n, 2 * m + 1, 0, 2 * v - 1))
    return np.stack(cols, axis=1)


def chart_interp(chart_uv, f, eval_uv):
    """Values at eval_uv of every triangle's degree-p polynomial interpolant
    of the node data f ((ntris * np,) or (ntris * np, ncomp), index j * np + i)
    given at chart_uv, np = (p+1)(p+2)/2 (section 3.3): Koornwinder
    coefficients c = V^-1 f per triangle, values E c."""
    uv = _f64(chart_uv).reshape(-1, 2)
    npn = len(uv)
    p = 0
    while (p + 1) * (p + 2) // 2 < npn:
        p += 1
    assert (p + 1) * (p + 2) // 2 == npn
    f = _f64(f)
    flat = f.ndim == 1
    F = f.reshape(-1, npn, 1 if flat else f.shape[1])
    ntris, ncomp = F.shape[0], F.shape[2]
    coef = np.linalg.solve(koornwinder(uv, p), F.transpose(1, 0, 2).reshape(npn, -1))
    out = (koornwinder(eval_uv, p) @ coef).reshape(-1, ntris, ncomp).transpose(1, 0, 2)
    return out.reshape(-1) if flat else out.reshape(-1, ncomp)
