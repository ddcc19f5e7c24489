"""Water-tight, outward-oriented flat skeleton triangulations (section 3: the
skeleton is a conforming, positively oriented triangle mesh).

All generators return ``(verts, tris)`` with ``verts`` (nv, 3) float64 and
``tris`` (nt, 3) int32, vertex order counter-clockwise seen from outside.
Quadratic (second-order curvilinear) skeletons have ``tris`` (nt, 6): the
corners P1 P2 P3 as above, then the edge points of P1P2, P2P3 and P3P1, each
shared by the two triangles of its edge.
"""
import numpy as np


# ----------------------------------------------------------------- cube
def cube_mesh(n, lo=0.0, hi=1.0):
    """Surface of the cube [lo, hi]^3, each face an n x n grid of squares,
    each square cut into two triangles (12 n^2 triangles)."""
    g = np.linspace(lo, hi, n + 1)
    keys = {}
    verts = []

    def vid(p):
        k = tuple(int(round((c - lo) / (hi - lo) * n)) for c in p)
        i = keys.get(k)
        if i is None:
            i = len(verts)
            keys[k] = i
            verts.append(p)
        return i

    tris = []
    # each face: fixed axis a at value s, outward normal sign sg, (b, c) in-plane axes
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s, sg in ((lo, -1.0), (hi, 1.0)):
            for i in range(n):
                for j in range(n):
                    quad = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0.0, 0.0, 0.0]
                        p[a] = s
                        p[b] = g[i + di]
                        p[c] = g[j + dj]
                        quad.append(vid(tuple(p)))
                    # (b, c, a) is a right-handed frame, so quad order is CCW seen
                    # from +a; reverse it on the -a face
                    q0, q1, q2, q3 = quad if sg > 0 else quad[::-1]
                    tris.append((q0, q1, q2))
                    tris.append((q0, q2, q3))
    return np.array(verts, dtype=np.float64), np.array(tris, dtype=np.int32)


# ----------------------------------------------------------- icosahedral
def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces = triples of mutually adjacent vertices (edge length is the minimum distance)
    d = np.linalg.norm(v[:, None] - v[None], axis=2)
    e = d.min(where=d > 1e-9, initial=10.0)
    adj = np.abs(d - e) < 1e-6
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    f = [i, j, k]
                    nrm = np.cross(v[j] - v[i], v[k] - v[i])
                    if np.dot(nrm, v[i] + v[j] + v[k]) < 0:
                        f = [i, k, j]
                    faces.append(f)
    return v, np.array(faces, dtype=np.int64)


def geodesic_sphere(nu, project=True):
    """Class-I geodesic sphere: every icosahedron face cut into nu^2 triangles
    by a uniform barycentric grid, then (optionally) projected to |x| = 1.
    20 nu^2 triangles, 10 nu^2 + 2 vertices."""
    V, F = _icosahedron()
    edges = {}
    for f in F:
        for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            key = (min(a, b), max(a, b))
            if key not in edges:
                edges[key] = len(edges)
    ne = len(edges)
    n_edge_pts = max(nu - 1, 0)
    n_int = max((nu - 1) * (nu - 2) // 2, 0)
    nv = 12 + ne * n_edge_pts + len(F) * n_int
    verts = np.zeros((nv, 3))
    verts[:12] = V

    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    m = (ii + jj) <= nu
    ii, jj = ii[m], jj[m]
    kk = nu - ii - jj
    lid = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    tris = []
    int_base = 12 + ne * n_edge_pts
    for fi, (A, B, C) in enumerate(F):
        gid = np.empty(ii.shape, dtype=np.int64)
        pos = V[A] + np.outer(ii / nu, V[B] - V[A]) + np.outer(jj / nu, V[C] - V[A])

        def edge_ids(p, q, t):
            # point at fraction t/nu from p towards q on edge (p, q)
            e = edges[(min(p, q), max(p, q))]
            tt = np.where(p < q, t, nu - t)
            return 12 + e * n_edge_pts + (tt - 1)

        corner_a = (ii == 0) & (jj == 0)
        corner_b = ii == nu
        corner_c = jj == nu
        on_ab = (jj == 0) & (ii > 0) & (ii < nu)
        on_ac = (ii == 0) & (jj > 0) & (jj < nu)
        on_bc = (kk == 0) & (ii > 0) & (jj > 0)
        inner = (ii > 0) & (jj > 0) & (kk > 0)
        gid[corner_a] = A
        gid[corner_b] = B
        gid[corner_c] = C
        gid[on_ab] = edge_ids(A, B, ii[on_ab])
        gid[on_ac] = edge_ids(A, C, jj[on_ac])
        gid[on_bc] = edge_ids(B, C, jj[on_bc])
        n_in = int(inner.sum())
        gid[inner] = int_base + fi * n_int + np.arange(n_in)
        verts[gid] = pos
        lid[ii, jj] = gid
        # up triangles (i,j),(i+1,j),(i,j+1); down (i+1,j),(i+1,j+1),(i,j+1)
        ui, uj = np.nonzero(np.add.outer(np.arange(nu + 1), np.arange(nu + 1)) <= nu - 1)
        up = np.stack([lid[ui, uj], lid[ui + 1, uj], lid[ui, uj + 1]], 1)
        di, dj = np.nonzero(np.add.outer(np.arange(nu + 1), np.arange(nu + 1)) <= nu - 2)
        dn = np.stack([lid[di + 1, dj], lid[di + 1, dj + 1], lid[di, dj + 1]], 1)
        tris.append(up)
        tris.append(dn)
    tris = np.concatenate(tris).astype(np.int32)
    if project:
        verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    return verts, tris


def icosphere(level):
    """Icosahedron subdivided ``level`` times (each face into 4^level flat
    triangles) and projected to the unit sphere: 20 * 4^level triangles."""
    return geodesic_sphere(2 ** level)


# ------------------------------------------------------ spherical harmonics
def _real_sph_harm_sum(theta, phi, coef, lmax):
    """sum_{l<=lmax, |m|<=l} coef[l][m] Y_lm(theta, phi), real orthonormal Y_lm.
    ``coef`` is a dict l -> array of length 2l+1 (m = -l..l)."""
    ct, st = np.cos(theta), np.sin(theta)
    out = np.zeros_like(theta)
    pmm = np.full_like(theta, 0.5 / np.sqrt(np.pi))        # \bar P_0^0
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * pmm
        cm, sm = (np.cos(m * phi), np.sin(m * phi)) if m > 0 else (None, None)
        p_lm2, p_lm1 = None, pmm
        for l in range(m, lmax + 1):
            if l == m:
                p = pmm
            elif l == m + 1:
                p = np.sqrt(2.0 * m + 3.0) * ct * pmm
            else:
                a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                p = a * (ct * p_lm1 - b * p_lm2)
            if l >= 1 and l in coef:
                c = coef[l]
                if m == 0:
                    out += c[l] * p
                else:
                    out += np.sqrt(2.0) * p * (c[l + m] * cm + c[l - m] * sm)
            if l > m:
                p_lm2, p_lm1 = p_lm1, p
            else:
                p_lm1 = p
    return out


def _sph(p):
    r = np.linalg.norm(p, axis=1)
    theta = np.arccos(np.clip(p[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(p[:, 1], p[:, 0])
    return theta, phi


def _normals(verts, tris):
    p0, p1, p2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    return np.cross(p1 - p0, p2 - p0)


def star_surface(nu, lmax=12, var0=0.1, seed=0, max_tries=50):
    """Star-shaped genus-0 surface r = 1 + sum_{1<=l<=lmax} a_lm Y_lm on a
    geodesic sphere of 20 nu^2 triangles, a_lm ~ N(0, var0 / l^2) (variance).
    Redrawn (same generator stream) until min r >= 0.3 and every triangle
    normal makes n . r_hat > 0.1 with its centroid direction."""
    rng = np.random.default_rng(seed)
    base, tris = geodesic_sphere(nu)
    theta, phi = _sph(base)
    for _ in range(max_tries):
        coef = {l: rng.normal(0.0, np.sqrt(var0) / l, size=2 * l + 1) for l in range(1, lmax + 1)}
        r = 1.0 + _real_sph_harm_sum(theta, phi, coef, lmax)
        if r.min() < 0.3:
            continue
        v = base * r[:, None]
        n = _normals(v, tris)
        c = v[tris].mean(axis=1)
        cosang = np.einsum("ij,ij->i", n, c) / (np.linalg.norm(n, axis=1) * np.linalg.norm(c, axis=1))
        if cosang.min() > 0.1:
            return v, tris
    raise RuntimeError("star_surface: no admissible draw")


def _mobius(p, lam):
    """Conformal self-map of the unit sphere: stereographic projection from
    the north pole, scaling by lam in the plane, inverse projection.  Local
    length scale grows by lam at the south pole and shrinks by 1/lam at the
    north pole (a lam^2 range), angles are preserved."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    den = np.maximum(1.0 - z, 1e-300)
    wx, wy = lam * x / den, lam * y / den
    w2 = wx * wx + wy * wy
    out = np.stack([2 * wx, 2 * wy, w2 - 1.0], 1) / (w2 + 1.0)[:, None]
    north = z > 1.0 - 1e-15
    out[north] = (0.0, 0.0, 1.0)
    return out


def bumpy_sphere(nu, grade=10.0, lmax=64, amp=0.05, nbumps=2000, seed=5,
                 height=(1e-3, 3e-2), width=(2e-3, 0.2), slope=0.3):
    """Large multiscale star-shaped surface.

    Geodesic sphere (20 nu^2 triangles) graded by the conformal map
    ``_mobius(., grade)`` (edge length varies by grade^2 over the surface),
    then displaced radially by r = 1 + sum_{1<=l<=lmax} a_lm Y_lm + bumps with
    a_lm ~ N(0, (amp / l^2)^2), and ``nbumps`` Gaussian bumps with centres
    uniform on the sphere, widths log-uniform in ``width`` and heights
    log-uniform in ``height`` capped at ``slope`` * width (keeps the surface
    star-shaped and the triangles outward-facing)."""
    rng = np.random.default_rng(seed)
    base, tris = geodesic_sphere(nu)
    base = _mobius(base, grade)
    theta, phi = _sph(base)
    coef = {l: rng.normal(0.0, amp / l ** 2, size=2 * l + 1) for l in range(1, lmax + 1)}
    r = 1.0 + _real_sph_harm_sum(theta, phi, coef, lmax)
    if nbumps:
        from scipy.spatial import cKDTree
        c = rng.normal(size=(nbumps, 3))
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        w = np.exp(rng.uniform(np.log(width[0]), np.log(width[1]), nbumps))
        h = np.exp(rng.uniform(np.log(height[0]), np.log(height[1]), nbumps))
        h = np.minimum(h, slope * w)
        sgn = rng.choice([-1.0, 1.0], nbumps)
        tree = cKDTree(base)
        for b in range(nbumps):
            idx = np.asarray(tree.query_ball_point(c[b], 6.0 * w[b]), dtype=np.int64)
            if idx.size:
                d2 = np.sum((base[idx] - c[b]) ** 2, axis=1)
                r[idx] += sgn[b] * h[b] * np.exp(-d2 / (2.0 * w[b] ** 2))
    return base * r[:, None], tris


# ----------------------------------------------------------------- torus
def torus_mesh(nu, nv, R=1.0, r=0.4, quadratic=False):
    """Torus ((R + r cos p) cos t, (R + r cos p) sin t, r sin p) on an nu x nv
    grid of (t, p), each cell split along its diagonal into two triangles
    (counter-clockwise in (t, p), which is outward).  With ``quadratic`` the
    edge points are the surface points at the parameter midpoints, so every
    one of the six points lies on the torus."""
    k = 2 if quadratic else 1
    gi, gj = np.meshgrid(np.arange(k * nu), np.arange(k * nv), indexing="ij")
    t = 2.0 * np.pi * gi.ravel() / (k * nu)
    p = 2.0 * np.pi * gj.ravel() / (k * nv)
    verts = np.stack([(R + r * np.cos(p)) * np.cos(t), (R + r * np.cos(p)) * np.sin(t),
                      r * np.sin(p)], axis=1)

    def vid(i, j):  # vertex at half-step grid point (i, j) of the k-refined grid
        return (i % (k * nu)) * (k * nv) + (j % (k * nv))

    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = k * i.ravel(), k * j.ravel()
    a, b, c, d = vid(i, j), vid(i + k, j), vid(i + k, j + k), vid(i, j + k)
    if not quadratic:
        tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
        return verts, tris.astype(np.int32)
    ab, bc, ac = vid(i + 1, j), vid(i + 2, j + 1), vid(i + 1, j + 1)
    cd, da = vid(i + 1, j + 2), vid(i, j + 1)
    tris = np.concatenate([np.stack([a, b, c, ab, bc, ac], 1), np.stack([a, c, d, ac, cd, da], 1)])
    used = np.unique(tris)
    remap = np.full(len(verts), -1, np.int64)
    remap[used] = np.arange(len(used))
    return verts[used], remap[tris].astype(np.int32)


def quadratic_from_flat(verts, tris, lift=None):
    """Quadratic skeleton from a flat one: one edge point per edge at the
    edge midpoint, mapped through ``lift`` (points (n, 3) -> (n, 3)) when
    given, e.g. onto the surface the flat mesh approximates.  Returns
    (verts, tris6); the corner vertices keep their indices."""
    nv, nt = len(verts), len(tris)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    uk, inv = np.unique(np.sort(e, axis=1), axis=0, return_inverse=True)
    mid = 0.5 * (verts[uk[:, 0]] + verts[uk[:, 1]])
    if lift is not None:
        mid = lift(mid)
    inv = inv.reshape(-1)
    t6 = np.concatenate([tris, np.stack([nv + inv[:nt], nv + inv[nt:2 * nt], nv + inv[2 * nt:]], 1)], 1)
    return np.concatenate([verts, mid]), t6.astype(np.int32)


# ----------------------------------------------------------- utilities
def refine_1to4(verts, tris):
    """Split every triangle into four by its edge midpoints (section 4.5)."""
    nv = len(verts)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    key = np.sort(e, axis=1)
    uk, inv = np.unique(key, axis=0, return_inverse=True)
    mid = 0.5 * (verts[uk[:, 0]] + verts[uk[:, 1]])
    nt = len(tris)
    m01, m12, m20 = (nv + inv[:nt], nv + inv[nt:2 * nt], nv + inv[2 * nt:])
    a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
    new = np.concatenate([np.stack([a, m01, m20], 1), np.stack([m01, b, m12], 1),
                          np.stack([m20, m12, c], 1), np.stack([m01, m12, m20], 1)])
    return np.concatenate([verts, mid]), new.astype(np.int32)


def refine_1to4_quadratic(verts, tris6):
    """Split every quadratic triangle into four (section 4.5 applied to the
    curved skeleton): the new corners are the old corners and edge points,
    the new edge points are points of the old patch, so the refined skeleton
    describes the same surface.  On a patch with parameters (u, v) on T0 the
    sub-triangles are (0,0)(1/2,0)(0,1/2), (1/2,0)(1,0)(1/2,1/2),
    (0,1/2)(1/2,1/2)(0,1), (1/2,0)(1/2,1/2)(0,1/2); edge points on an old edge
    are its quadratic curve at t = 1/4 and 3/4 (computed once per edge, so
    neighbours share them), interior ones the patch at (1/4,1/4), (1/2,1/4),
    (1/4,1/2)."""
    verts = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris6, dtype=np.int64)
    nt = len(t)
    P = verts[t]                                        # (nt, 6, 3)

    def patch(u, v):                                    # quadratic Lagrange patch at (u, v)
        l1, l2, l3 = 1.0 - u - v, u, v
        N = np.array([l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), l3 * (2 * l3 - 1), 4 * l1 * l2, 4 * l2 * l3, 4 * l3 * l1])
        return np.einsum("k,nkc->nc", N, P)

    # old edges (corner a, edge point m, corner b) as P1P2, P2P3, P3P1
    ea = np.concatenate([t[:, 0], t[:, 1], t[:, 2]])
    eb = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])
    em = np.concatenate([t[:, 3], t[:, 4], t[:, 5]])
    lo, hi = np.minimum(ea, eb), np.maximum(ea, eb)
    key = lo * (len(verts) + 1) + hi
    uk, first, inv = np.unique(key, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    A, B, M = verts[lo[first]], verts[hi[first]], verts[em[first]]

    def curve(s):                                       # the edge's quadratic, s = 0 at the lower-index corner
        return (1 - s) * (1 - 2 * s) * A + 4 * s * (1 - s) * M + s * (2 * s - 1) * B

    nv = len(verts)
    q_lo = curve(0.25)                                  # quarter point next to the lower-index corner
    q_hi = curve(0.75)
    ne = len(uk)
    new = [verts, q_lo, q_hi]
    base_lo, base_hi = nv, nv + ne
    ins = [patch(0.25, 0.25), patch(0.5, 0.25), patch(0.25, 0.5)]
    base_in = nv + 2 * ne
    new += ins

    def quarter(e_slot, near):
        """index of the quarter point of old edge slot e_slot (0: P1P2, 1: P2P3,
        2: P3P1 of every triangle) next to corner array `near`"""
        e = inv[e_slot * nt:(e_slot + 1) * nt]
        lo_e = lo[e_slot * nt:(e_slot + 1) * nt]
        return np.where(near == lo_e, base_lo + e, base_hi + e)
    c1, c2, c3, m12, m23, m31 = (t[:, k] for k in range(6))
    q12a, q12b = quarter(0, c1), quarter(0, c2)         # (1/4,0) and (3/4,0)
    q23a, q23b = quarter(1, c2), quarter(1, c3)         # (3/4,1/4) and (1/4,3/4)
    q31a, q31b = quarter(2, c3), quarter(2, c1)         # (0,3/4) and (0,1/4)
    i11 = base_in + np.arange(nt)                       # (1/4,1/4)
    i21 = base_in + nt + np.arange(nt)                  # (1/2,1/4)
    i12 = base_in + 2 * nt + np.arange(nt)              # (1/4,1/2)
    out = np.concatenate([
        np.stack([c1, m12, m31, q12a, i11, q31b], 1),
        np.stack([m12, c2, m23, q12b, q23a, i21], 1),
        np.stack([m31, m23, c3, i12, q23b, q31a], 1),
        np.stack([m12, m23, m31, i21, i12, i11], 1)])
    return np.concatenate(new), out.astype(np.int32)


def mesh_check(verts, tris):
    """Return (closed, signed_volume): closed is True when every directed edge
    appears exactly once and its reverse exactly once (water-tight, consistently
    oriented, manifold)."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    n = int(verts.shape[0])
    fwd = e[:, 0] * n + e[:, 1]
    rev = e[:, 1] * n + e[:, 0]
    u, cnt = np.unique(fwd, return_counts=True)
    closed = bool(np.all(cnt == 1)) and bool(np.all(np.isin(rev, u)))
    p0, p1, p2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    vol = float(np.sum(np.einsum("ij,ij->i", p0, np.cross(p1, p2))) / 6.0)
    return closed, vol


def triangle_diameters(verts, tris):
    """D_j: diameter of the smallest ball enclosing triangle j (section 2, the
    multiscale mollifier): the longest edge for a right or obtuse triangle,
    twice the circumradius otherwise."""
    p0, p1, p2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    a2 = np.sum((p1 - p2) ** 2, 1)
    b2 = np.sum((p2 - p0) ** 2, 1)
    c2 = np.sum((p0 - p1) ** 2, 1)
    l2 = np.stack([a2, b2, c2], 1)
    lmax2 = l2.max(1)
    obtuse = 2.0 * lmax2 >= a2 + b2 + c2      # lmax^2 >= sum of the other two
    area2 = np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)   # 2 * area
    circ_d = np.sqrt(a2 * b2 * c2) / np.maximum(area2, 1e-300)   # 2R = abc / (2 area)
    return np.where(obtuse, np.sqrt(lmax2), circ_d)


# ------------------------------------------------------- graded torus (C3)
def _torus_p_of_v(v, R, r):
    """Inverse of the conformal tube coordinate v(p) = int_0^p r / (R + r cos q) dq
    of a torus: p in [0, 2 pi) for v in [0, V), V = 2 pi r / sqrt(R^2 - r^2)."""
    k = np.sqrt(R * R - r * r) / (2.0 * r)
    phi = v * k
    return np.mod(2.0 * np.arctan2(np.sqrt((R + r) / (R - r)) * np.sin(phi), np.cos(phi)), 2.0 * np.pi)


def _torus_point(t, p, R, r):
    rho = R + r * np.cos(p)
    return np.stack([rho * np.cos(t), rho * np.sin(t), r * np.sin(p)], axis=-1)


def graded_torus(n_tris=200_000, R=1.0, r=0.3, nbumps=200, seed=3, height=(2e-3, 5e-2), width=(1e-2, 0.1),
                 h_range=100.0, grade_rate=1.0, size_power=2.0, slope=0.3, tries=4):
    """Multiscale torus: a torus (R, r) carrying ``nbumps`` Gaussian bumps,
    triangulated with edge lengths graded over a ``h_range`` ratio.

    Bumps: centres uniform by area on the torus, widths and heights
    log-uniform in ``width`` / ``height`` (heights capped at ``slope`` x width),
    random sign, displacement along the torus normal with a Gaussian of the
    3D chord distance.  Size field: h(x) = c w_b (w_b / w_max)^(size_power - 1)
    inside 3 w_b of bump b (finer, relative to its width, for a narrower bump:
    with size_power 2 the tenfold width range spans a hundredfold size
    range), growing by ``grade_rate`` per unit distance beyond, the smallest
    over the bumps, clamped to [h_min, h_range h_min] (h_min the size at the
    narrowest bump), with c chosen so that the mesh has about ``n_tris``
    triangles.

    Triangulation: conformal coordinates (u, v) = (t, int r dp / (R + r cos p))
    make the torus a flat 2 pi x V rectangle with metric
    (R + r cos p)^2 (du^2 + dv^2); a 2:1-balanced periodic quadtree is refined
    until every cell's diagonal (in 3D) is at most h at its centre, and the
    jittered cell corners are triangulated by a periodic Delaunay
    triangulation in (u, v), which is angle-preserving up to the bumps.
    Returns verts (n, 3), tris (m, 3) int32, outward (counter-clockwise in
    (t, p))."""
    from scipy.spatial import Delaunay, cKDTree
    rng = np.random.default_rng(seed)
    # bumps: t uniform, p with density (R + r cos p) / (2 pi R) by rejection
    tb = rng.uniform(0.0, 2.0 * np.pi, nbumps)
    pb = np.empty(nbumps)
    k = 0
    while k < nbumps:
        p = rng.uniform(0.0, 2.0 * np.pi, 4 * nbumps)
        acc = p[rng.uniform(0.0, R + r, p.size) < R + r * np.cos(p)]
        take = min(acc.size, nbumps - k)
        pb[k:k + take] = acc[:take]
        k += take
    wb = np.exp(rng.uniform(np.log(width[0]), np.log(width[1]), nbumps))
    hb = np.minimum(np.exp(rng.uniform(np.log(height[0]), np.log(height[1]), nbumps)), slope * wb)
    sb = rng.choice([-1.0, 1.0], nbumps)
    cb = _torus_point(tb, pb, R, r)
    tree_b = cKDTree(cb)
    kb = min(32, nbumps)
    U, V = 2.0 * np.pi, 2.0 * np.pi * r / np.sqrt(R * R - r * r)
    nv0 = 6
    nu0 = int(round(U / V * nv0))
    du0, dv0 = U / nu0, V / nv0
    wfine = wb * (wb / wb.max()) ** (size_power - 1.0)     # bump size in units of c
    wmin = wfine.min()

    def size_at(uv, c):
        t, p = uv[:, 0], _torus_p_of_v(uv[:, 1], R, r)
        x = _torus_point(t, p, R, r)
        d, nb = tree_b.query(x, k=kb)                 # the nearest bumps decide the minimum
        hb_i = c * wfine[nb] + grade_rate * np.maximum(0.0, d - 3.0 * wb[nb])
        h = np.minimum(h_range * c * wmin, hb_i.min(axis=1))
        return np.maximum(h, c * wmin), (R + r * np.cos(p))

    def quadtree(c):
        # leaves per level: lv[l] = {(i, j)}, level-l cells du0 / 2^l x dv0 / 2^l
        lv = [{(i, j) for i in range(nu0) for j in range(nv0)}]
        level = 0
        while level < len(lv) and lv[level]:
            arr = np.array(sorted(lv[level]), dtype=np.int64)
            sc = 0.5 ** level
            uv = np.stack([(arr[:, 0] + 0.5) * du0 * sc, (arr[:, 1] + 0.5) * dv0 * sc], 1)
            h, lam = size_at(uv, c)
            split = arr[lam * np.hypot(du0, dv0) * sc > h]
            if len(split):
                if len(lv) == level + 1:
                    lv.append(set())
                lv[level].difference_update(map(tuple, split.tolist()))
                ch = (2 * split[:, None, :] + np.array([[0, 0], [0, 1], [1, 0], [1, 1]])[None]).reshape(-1, 2)
                lv[level + 1].update(map(tuple, ch.tolist()))
            level += 1
        # 2:1 balance across edges and corners (periodic): every leaf of level
        # m >= 2 sees leaves of level >= m - 1 around its parent
        for m in range(len(lv) - 1, 1, -1):
            par = {(i >> 1, j >> 1) for (i, j) in lv[m]}
            l = m - 1
            nl_u, nl_v = nu0 << l, nv0 << l
            nbr = {((pi + a) % nl_u, (pj + b) % nl_v) for (pi, pj) in par for a in (-1, 0, 1) for b in (-1, 0, 1)}
            for (i, j) in nbr - par:
                _ensure_level(lv, l, i, j)
        return lv

    c = 2.6 * np.sqrt(200_000 / n_tris)        # about right for the defaults; refined below
    for _ in range(tries):
        lv = quadtree(c)
        est = 2.0 * sum(len(q) for q in lv)
        if abs(est / n_tris - 1.0) < 0.1:
            break
        c *= np.sqrt(est / n_tris)
    leaves = {(l, i, j) for l, q in enumerate(lv) for (i, j) in q}
    maxl = max(q[0] for q in leaves)
    NU, NV = nu0 << maxl, nv0 << maxl
    pts = set()
    for (l, i, j) in leaves:
        f = 1 << (maxl - l)
        for a in (0, 1):
            for b in (0, 1):
                pts.add((((i + a) * f) % NU, ((j + b) * f) % NV))
    pts = np.array(sorted(pts), dtype=np.int64)
    uv = np.stack([pts[:, 0] * (U / NU), pts[:, 1] * (V / NV)], 1)
    uv += rng.normal(0.0, 1e-4 * min(U / NU, V / NV), uv.shape)     # no cocircular quadruples
    n = len(uv)
    # periodic Delaunay: the points plus their images within a margin
    m = 3.0 * max(du0, dv0)
    ext, ids = [uv], [np.arange(n)]
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            if a == 0 and b == 0:
                continue
            q = uv + np.array([a * U, b * V])
            sel = (q[:, 0] > -m) & (q[:, 0] < U + m) & (q[:, 1] > -m) & (q[:, 1] < V + m)
            ext.append(q[sel])
            ids.append(np.nonzero(sel)[0])
    ext, ids = np.concatenate(ext), np.concatenate(ids)
    tri = Delaunay(ext).simplices
    cen = ext[tri].mean(axis=1)
    eps = 1e-9
    keep = (cen[:, 0] >= eps) & (cen[:, 0] < U + eps) & (cen[:, 1] >= eps) & (cen[:, 1] < V + eps)
    tri = tri[keep]
    p0, p1, p2 = ext[tri[:, 0]], ext[tri[:, 1]], ext[tri[:, 2]]
    cr = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    tris = ids[tri]
    flip = cr < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    t = uv[:, 0]
    p = _torus_p_of_v(uv[:, 1], R, r)
    x = _torus_point(t, p, R, r)
    nrm = np.stack([np.cos(p) * np.cos(t), np.cos(p) * np.sin(t), np.sin(p)], axis=1)
    disp = np.zeros(n)
    for b, cand in enumerate(cKDTree(x).query_ball_point(cb, 6.0 * wb)):
        cand = np.asarray(cand, dtype=np.int64)
        if cand.size:
            d2 = np.sum((x[cand] - cb[b]) ** 2, axis=1)
            disp[cand] += sb[b] * hb[b] * np.exp(-d2 / (2.0 * wb[b] ** 2))
    return x + disp[:, None] * nrm, tris.astype(np.int32)


def _ensure_level(lv, l, i, j):
    """Split quadtree leaves (lv[L] = {(i, j)} per level L) so that cell
    (l, i, j) is a leaf or lies inside finer leaves (no coarser leaf covers it)."""
    L = l
    while L >= 0 and (i >> (l - L), j >> (l - L)) not in lv[L]:
        L -= 1
    if L < 0 or L == l:
        return                       # already subdivided at least to level l
    while L < l:
        I, J = i >> (l - L), j >> (l - L)
        lv[L].discard((I, J))
        lv[L + 1].update({(2 * I + a, 2 * J + b) for a in (0, 1) for b in (0, 1)})
        L += 1
