"""The five benchmark workloads, as seeded recipes.

Each ``configN(scale=...)`` returns a dict with ``verts``, ``tris``,
``sigma`` (per triangle, or a length-1 array for a constant width),
``rule`` (Dunavant-6), ``targets`` and, where the workload has a chart
projection, ``chart_uv``.  ``scale`` < 1 shrinks the target count (and for the
graded meshes the triangle count) for parity tests; scale = 1 is the full
workload.

* C1  unit cube, 16 x 16 squares per face (3072 triangles), sigma = 0.1,
      4096 targets uniform in [-0.5, 1.5]^3, seed 0.
* C2  icosphere level 5 (20,480 triangles), sigma = 0.05, 1e6 targets with
      radius U[0.5, 1.5] and isotropic direction, seed 2.
* C3  multiscale torus (R = 1, r = 0.3) with 200 Gaussian bumps (heights
      log-uniform in [0.002, 0.05], widths in [0.01, 0.1]), triangulated
      with triangle diameters graded about 110x (see ``graded_torus``),
      ~2.3e5 triangles, sigma_j = 0.5 D_j, 45 order-8 chart nodes per
      triangle (~1e7 Newton targets), seed 3.
* C4  64 star-shaped surfaces, triangle counts log-uniform in [500, 50000]
      (geodesic 20 nu^2), sigma_j = 0.5 D_j, 1e4 targets per surface in the
      25 %-padded bounding box, seed 4.
* C5  large multiscale bumpy sphere, ~2e6 triangles (nu = 316), edge length
      graded 100x, l <= 64 harmonics + 2000 bumps, sigma_j = 0.5 D_j,
      5e7 near-surface targets (offsets t sigma_j n, t ~ U[-3, 3]), seed 5.
"""
import numpy as np

from .rules import dunavant6, chart_nodes_45
from .meshes import (cube_mesh, icosphere, star_surface, bumpy_sphere, graded_torus,
                     triangle_diameters)
from .targets import (box_targets, shell_targets, bbox_targets,
                      surface_offset_targets)


def config1(n_targets=4096):
    v, t = cube_mesh(16)
    return dict(name="cube-3072tri-sigma0.1", verts=v, tris=t,
                sigma=np.array([0.1]), rule=dunavant6(),
                targets=box_targets(4096, -0.5, 1.5, seed=0)[:n_targets])


def config2(n_targets=1_000_000, level=5):
    v, t = icosphere(level)
    return dict(name="icosphere%d-%dtri-sigma0.05" % (level, len(t)), verts=v, tris=t,
                sigma=np.array([0.05]), rule=dunavant6(),
                targets=shell_targets(n_targets, 0.5, 1.5, seed=2))


def config3(n_tris=200_000, seed=3):
    v, t = graded_torus(n_tris=n_tris, R=1.0, r=0.3, nbumps=200, seed=seed, height=(2e-3, 5e-2),
                        width=(1e-2, 0.1))
    sig = 0.5 * triangle_diameters(v, t)
    return dict(name="graded-torus-%dtri" % len(t), verts=v, tris=t, sigma=sig,
                rule=dunavant6(), chart_uv=chart_nodes_45(), targets=None)


def config4(n_surf=64, mmin=500, mmax=50_000, n_targets=10_000, seed=4):
    rng = np.random.default_rng(seed)
    meshes = []
    for s in range(n_surf):
        m = np.exp(rng.uniform(np.log(mmin), np.log(mmax)))
        nu = int(np.clip(round(np.sqrt(m / 20.0)), 5, 50))
        v, t = star_surface(nu, lmax=12, var0=0.1, seed=int(rng.integers(1 << 31)))
        sig = 0.5 * triangle_diameters(v, t)
        x = bbox_targets(v, n_targets, pad=0.25, seed=int(rng.integers(1 << 31)))
        meshes.append(dict(verts=v, tris=t, sigma=sig, targets=x))
    return dict(name="batch-%d-star" % n_surf, meshes=meshes, rule=dunavant6(),
                chart_uv=chart_nodes_45())


def concat_batch(meshes):
    """Concatenate a list of meshes into one ragged batch: vertex arrays are
    stacked, triangle indices offset, and CSR triangle / target offsets per mesh."""
    vs, ts, ss, xs, xm = [], [], [], [], []
    toff, voff = [0], 0
    for i, m in enumerate(meshes):
        vs.append(m["verts"])
        ts.append(m["tris"] + voff)
        voff += len(m["verts"])
        toff.append(toff[-1] + len(m["tris"]))
        ss.append(np.broadcast_to(m["sigma"], (len(m["tris"]),)) if len(m["sigma"]) == 1 else m["sigma"])
        if m.get("targets") is not None:
            xs.append(m["targets"])
            xm.append(np.full(len(m["targets"]), i, dtype=np.int32))
    return dict(verts=np.concatenate(vs), tris=np.concatenate(ts).astype(np.int32),
                sigma=np.concatenate(ss), tri_offsets=np.array(toff, dtype=np.int64),
                targets=np.concatenate(xs) if xs else None,
                target_mesh=np.concatenate(xm) if xm else None)


def config5(nu=316, n_targets=50_000_000, seed=5, lmax=64, nbumps=2000, meta=False):
    """meta: also return, per target, the triangle it was drawn on
    (``target_tri``) and its normal offset in units of that triangle's sigma
    (``target_t``), for stratified samples; the targets are the same."""
    v, t = bumpy_sphere(nu, grade=10.0, lmax=lmax, amp=0.05, nbumps=nbumps, seed=seed)
    sig = 0.5 * triangle_diameters(v, t)
    out = surface_offset_targets(v, t, sig, n_targets, tmax=3.0, seed=seed + 1000, meta=meta)
    cfg = dict(name="graded-bumpy-sphere-%dtri" % len(t), verts=v, tris=t, sigma=sig, rule=dunavant6())
    if meta:
        cfg["targets"], cfg["target_tri"], cfg["target_t"] = out
    else:
        cfg["targets"] = out
    return cfg
