"""GPU parity of the direct-sum path (every pair with the full kernel) against
the CPU oracle, through the C ABI.

Error metric (relative to the largest oracle value over the compared set):
  e_phi  = max |dPhi| / max |Phi_oracle|
  e_grad = max ||d grad|| / max ||grad_oracle||
Bars: FP64 <= 1e-12, mixed <= 1e-6.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1909_13356_amd as lss
from workloads import (dunavant6, chart_nodes, cube_mesh, icosphere, star_surface,
                       triangle_diameters, box_targets, shell_targets, configs)

pytestmark = pytest.mark.gpu

TOL = {lss.FP64: 1e-12, lss.MIXED: 1e-6}


def errs(phi, g, phi_o, g_o):
    ep = np.max(np.abs(phi - phi_o)) / np.max(np.abs(phi_o))
    eg = np.max(np.linalg.norm(g - g_o, axis=1)) / np.max(np.linalg.norm(g_o, axis=1))
    return ep, eg


def ctx_for(verts, tris, sigma, prec=lss.FP64, offsets=None, **opt):
    c = lss.Context()
    c.set_sources(verts, tris, dunavant6(), tri_offsets=offsets)
    c.set_sigma(np.atleast_1d(np.asarray(sigma, float)))
    c.set_options(precision=prec, **opt)
    return c


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    cfg = configs.config1()
    po, go = oracle.evaluate(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], cfg["targets"])
    return cfg, po, go


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_config1_cube_all_targets(c1, prec):
    cfg, po, go = c1
    say("case: cube 3072 tri, 4096 targets, precision", prec)
    c = ctx_for(cfg["verts"], cfg["tris"], cfg["sigma"], prec)
    phi, g = c.eval(cfg["targets"])
    ep, eg = errs(phi, g, po, go)
    say("  e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]
    st = c.stats()
    assert st["last_pairs"] == 4096 * 36864


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_tiles_and_ragged_tail(c1, tile):
    cfg, po, go = c1
    n = 1000 + tile // 2 + 7            # not a multiple of any tile
    say("case: cube, tile", tile, "n", n)
    c = ctx_for(cfg["verts"], cfg["tris"], cfg["sigma"], lss.FP64, tile=tile)
    phi, g = c.eval(cfg["targets"][:n])
    ep, eg = errs(phi, g, po[:n], go[:n])
    assert ep <= 1e-12 and eg <= 1e-12


def test_config2_sphere_full_size_sampled():
    cfg = configs.config2()
    x = cfg["targets"]
    rng = np.random.default_rng(12)
    sample = np.sort(rng.choice(len(x), 2048, replace=False))
    po, go = oracle.evaluate(cfg["verts"], cfg["tris"], cfg["sigma"], cfg["rule"], x[sample])
    for prec in (lss.FP64, lss.MIXED):
        say("case: icosphere-5, 1e6 targets, precision", prec)
        c = ctx_for(cfg["verts"], cfg["tris"], cfg["sigma"], prec)
        phi, g = c.eval(x)
        ep, eg = errs(phi[sample], g[sample], po, go)
        say("  e_phi %.3e e_grad %.3e" % (ep, eg))
        assert ep <= TOL[prec] and eg <= TOL[prec]
        assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g))


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_per_triangle_sigma(prec):
    v, t = star_surface(12, seed=3)
    sig = 0.5 * triangle_diameters(v, t)
    x = box_targets(3000, -1.5, 1.5, seed=9)
    say("case: star surface per-triangle sigma, precision", prec)
    po, go = oracle.evaluate(v, t, sig, dunavant6(), x)
    c = ctx_for(v, t, sig, prec)
    phi, g = c.eval(x)
    ep, eg = errs(phi, g, po, go)
    say("  e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]


def test_edge_cases():
    v, t = cube_mesh(2)
    say("case: edge cases on a 48-triangle cube")
    c = ctx_for(v, t, [0.3])
    y, _ = oracle.nodes(v, t, dunavant6())
    # target exactly on a node, one very close, one far away, one single target
    x = np.array([y[7], y[7] + 1e-12, [40.0, -3.0, 2.0], [0.5, 0.5, 0.5]])
    phi, g = c.eval(x)
    po, go = oracle.evaluate(v, t, [0.3], dunavant6(), x)
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g))
    assert np.max(np.abs(phi - po)) <= 1e-12 * np.abs(po).max()
    assert np.max(np.abs(g - go)) <= 1e-12 * np.abs(go).max()
    p1, g1 = c.eval(x[3:4])
    assert abs(p1[0] - po[3]) <= 1e-12
    # empty input is a no-op
    p0, g0 = c.eval(np.zeros((0, 3)))
    assert p0.shape == (0,)
    # non-finite target -> NaN outputs, the others unaffected
    xn = np.array([[np.nan, 0.0, 0.0], [0.5, 0.5, 0.5]])
    pn, gn = c.eval(xn)
    assert np.isnan(pn[0]) and abs(pn[1] - po[3]) <= 1e-12


def test_ragged_batch_of_meshes():
    meshes = []
    for i, (nu, s) in enumerate([(3, 0.2), (7, 0.1), (5, 0.15)]):
        v, tt = star_surface(nu, seed=20 + i)
        meshes.append(dict(verts=v + 3.0 * i, tris=tt, sigma=np.array([s]),
                           targets=box_targets(50 + 37 * i, -1.2 + 3 * i, 1.2 + 3 * i, seed=i)))
    b = configs.concat_batch(meshes)
    say("case: ragged batch of 3 meshes", len(b["tris"]), "triangles")
    c = ctx_for(b["verts"], b["tris"], b["sigma"], lss.FP64, offsets=b["tri_offsets"])
    phi, g = c.eval(b["targets"], x_mesh=b["target_mesh"])
    po, go = oracle.evaluate(b["verts"], b["tris"], b["sigma"], dunavant6(), b["targets"],
                             tri_offsets=b["tri_offsets"], x_mesh=b["target_mesh"])
    ep, eg = errs(phi, g, po, go)
    assert ep <= 1e-12 and eg <= 1e-12
    cm = ctx_for(b["verts"], b["tris"], b["sigma"], lss.MIXED, offsets=b["tri_offsets"])
    phi, g = cm.eval(b["targets"], x_mesh=b["target_mesh"])
    ep, eg = errs(phi, g, po, go)
    assert ep <= 1e-6 and eg <= 1e-6


def test_device_pointers_and_determinism(c1):
    import torch
    cfg, po, go = c1
    say("case: device tensors, run twice")
    c = ctx_for(cfg["verts"], cfg["tris"], cfg["sigma"], lss.FP64)
    xd = torch.as_tensor(cfg["targets"], device="cuda")
    p1, g1 = c.eval(xd)
    p2, g2 = c.eval(xd)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(g1, g2)
    ph, gh = c.eval(cfg["targets"])
    assert np.array_equal(p1.cpu().numpy(), ph) and np.array_equal(g1.cpu().numpy(), gh)


def test_error_codes():
    v, t = cube_mesh(1)
    c = lss.Context()
    with pytest.raises(lss.LssError) as e:
        c.eval(np.zeros((1, 3)))
    assert e.value.code == 4                                   # ESTATE: no sources
    bad = t.copy()
    bad[0, 0] = 99
    with pytest.raises(lss.LssError) as e:
        c.set_sources(v, bad, dunavant6())
    assert e.value.code == 1                                   # EINVAL: index
    with pytest.raises(lss.LssError) as e:
        c.set_sources(v, t[:, ::-1].copy(), dunavant6())
    assert e.value.code == 5                                   # EORIENT
    c.set_sources(v, t, dunavant6())
    with pytest.raises(lss.LssError) as e:
        c.eval(np.zeros((1, 3)))
    assert e.value.code == 4                                   # ESTATE: no sigma
    for s in ([0.0], [-1.0], [np.nan], np.ones(5)):
        with pytest.raises(lss.LssError) as e:
            c.set_sigma(np.asarray(s, float))
        assert e.value.code == 1
    with pytest.raises(lss.LssError) as e:
        c.set_options(tile=100)
    assert e.value.code == 1
    c.set_sigma([0.1])
    phi, _ = c.eval(np.array([[0.5, 0.5, 0.5]]))
    assert phi[0] > 0.5


def test_default_rule_when_rule_is_null(c1):
    """rule_uvw == NULL selects the library's Dunavant-6 rule: the sums are
    bitwise those with the same rule passed explicitly (direct and FMM), and
    a NULL rule with nq other than 0 or 12 is rejected."""
    import ctypes
    cfg, po, go = c1
    say("case: NULL rule vs explicit Dunavant-6, cube 3072 tri")
    for far in (lss.FAR_DIRECT, lss.FAR_FMM):
        ca = lss.Context()
        ca.set_sources(cfg["verts"], cfg["tris"], None)
        cb = ctx_for(cfg["verts"], cfg["tris"], cfg["sigma"])
        for c in (ca, cb):
            c.set_sigma(cfg["sigma"])
            c.set_options(precision=lss.FP64, far_field=far)
        pa, ga = ca.eval(cfg["targets"])
        pb, gb = cb.eval(cfg["targets"])
        assert np.array_equal(pa, pb) and np.array_equal(ga, gb), far
        assert ca.stats()["n_nodes"] == 12 * len(cfg["tris"])
    v = np.ascontiguousarray(cfg["verts"])
    t = np.ascontiguousarray(cfg["tris"], dtype=np.int32)
    rc = ca._lib.lss_set_sources(ca._h, v.ctypes.data_as(ctypes.c_void_p), len(v), t.ctypes.data_as(ctypes.c_void_p),
                                 len(t), None, 0, None, 7, 0)
    assert rc == 1                                             # EINVAL: NULL rule with nq = 7


# ------------------------------------------------------------------ Newton
@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_project_sphere_vs_oracle(prec):
    v, t = icosphere(3)
    sigma = 0.1
    uv = chart_nodes(2)
    say("case: project icosphere-3, np=6, precision", prec)
    c = ctx_for(v, t, [sigma], prec)
    h, x, st, it = c.project(uv)
    sel = np.arange(0, len(t), 37)
    tau = 1e-12 if prec == lss.FP64 else 1e-6
    ho, xo, sto, ito = oracle.project(v, t, [sigma], dunavant6(), uv, tau=tau, sel=sel)
    idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
    assert np.all(st == 0) and np.all(sto == 0)
    eh = np.max(np.abs(h[idx] - ho)) / sigma
    ex = np.max(np.linalg.norm(x[idx] - xo, axis=1)) / sigma
    say("  e_h %.3e e_x %.3e iters max %d" % (eh, ex, it.max()))
    bar = 1e-11 if prec == lss.FP64 else 2e-6
    assert eh <= bar and ex <= bar
    phi, _ = oracle.evaluate(v, t, [sigma], dunavant6(), x[idx])
    assert np.max(np.abs(phi - 0.5)) <= (1e-12 if prec == lss.FP64 else 1e-6)


def test_project_statuses():
    say("case: project statuses")
    v, t = cube_mesh(1)
    c = ctx_for(v, t, [5.0])
    h, x, st, it = c.project(chart_nodes(1))
    assert np.all(st == lss.NODE_NOBRACKET)
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0.3, 0.3, 1.0]])
    tt = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], np.int32)   # tetrahedron
    c = ctx_for(P, tt, [0.05], newton_max_iter=1)
    h, x, st, it = c.project(chart_nodes(1))
    assert np.all((st == lss.NODE_MAXITER) | (st == lss.NODE_CONVERGED)) and np.all(it == 1)
    ho, xo, sto, ito = oracle.project(P, tt, [0.05], dunavant6(), chart_nodes(1), max_iter=1)
    assert np.array_equal(st, sto)
    assert np.max(np.abs(h - ho)) <= 1e-12


@pytest.mark.parametrize("max_iter", [3, 20, 0])
def test_project_repeated_graph_launches(max_iter):
    """Newton iterations run as captured graphs launched in chunks; repeated
    projections with other work in between, a smaller second call and an
    iteration cap that is not a multiple of the chunk must all agree with the
    oracle, and the statistics must match the per-node iteration counts."""
    v, t = icosphere(3)
    sigma = 0.1
    say("case: repeated projections, max_iter", max_iter)
    c = ctx_for(v, t, [sigma], lss.FP64, newton_max_iter=max_iter)
    sel = np.arange(0, len(t), 41)
    kw = dict(max_iter=max_iter) if max_iter else {}
    for uv in (chart_nodes(2), chart_nodes(1), chart_nodes(2)):
        h, x, st, it = c.project(uv)
        stt = c.stats()
        assert stt["newton_iters"] == it.max()
        assert stt["last_targets"] == int(it.astype(np.int64).sum())
        ho, xo, sto, ito = oracle.project(v, t, [sigma], dunavant6(), uv, sel=sel, **kw)
        idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
        assert np.array_equal(st[idx], sto)
        assert np.max(np.abs(h[idx] - ho)) / sigma <= 1e-11
        c.eval(np.array([[0.1, 0.2, 0.3]]))     # eager work between graph launches
