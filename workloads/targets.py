"""Seeded target point sets."""
import numpy as np


def box_targets(n, lo=-0.5, hi=1.5, seed=0):
    """n points uniform in [lo, hi]^3 (rng.uniform, one (n, 3) draw)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 3))


def shell_targets(n, rmin=0.5, rmax=1.5, seed=2):
    """n points with radius uniform in [rmin, rmax] and direction the
    normalised standard normal vector."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(rmin, rmax, size=n)
    return d * r[:, None]


def bbox_targets(verts, n, pad=0.25, seed=4):
    """n points uniform in the bounding box of ``verts`` enlarged by ``pad``
    times its extent on every side."""
    rng = np.random.default_rng(seed)
    lo, hi = verts.min(0), verts.max(0)
    ext = hi - lo
    return rng.uniform(lo - pad * ext, hi + pad * ext, size=(n, 3))


def surface_offset_targets(verts, tris, sigma, n, tmax=3.0, seed=5, chunk=1 << 22, meta=False):
    """n points near the skeleton surface: a triangle drawn with probability
    proportional to its area, a uniform point on it, then an offset t * sigma_j
    along its unit normal with t ~ U[-tmax, tmax] (the spread of Newton
    iterates around the level set).  Generated in chunks to bound memory.
    With ``meta`` also returns each point's triangle j (int32) and t."""
    rng = np.random.default_rng(seed)
    p0, p1, p2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    area2 = np.linalg.norm(nrm, axis=1)
    cdf = np.cumsum(area2)
    cdf /= cdf[-1]
    out = np.empty((n, 3))
    if meta:
        mj, mt = np.empty(n, np.int32), np.empty(n)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        j = np.minimum(np.searchsorted(cdf, rng.uniform(size=m)), len(tris) - 1)
        a, b = rng.uniform(size=m), rng.uniform(size=m)
        flip = a + b > 1.0
        a[flip], b[flip] = 1.0 - a[flip], 1.0 - b[flip]
        t = rng.uniform(-tmax, tmax, size=m)
        q = p0[j] + a[:, None] * (p1[j] - p0[j]) + b[:, None] * (p2[j] - p0[j])
        out[s:s + m] = q + (t * sigma[j] / area2[j])[:, None] * nrm[j]
        if meta:
            mj[s:s + m], mt[s:s + m] = j, t
    if meta:
        return out, mj, mt
    return out
