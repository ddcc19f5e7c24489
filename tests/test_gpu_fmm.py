"""GPU parity of the octree + Laplace-dipole FMM path (far_field = FMM)
against the CPU oracle (sampled) and against the GPU direct sum (all
targets).  Same error metric and bars as the direct path: FP64 <= 1e-12,
mixed <= 1e-6 (max error over the compared set, relative to the largest
oracle value)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1909_13356_amd as lss
from workloads import (dunavant6, chart_nodes, icosphere, bumpy_sphere, triangle_diameters,
                       shell_targets, surface_offset_targets, box_targets)

pytestmark = pytest.mark.gpu
TOL = {lss.FP64: 1e-12, lss.MIXED: 1e-6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def errs(phi, g, phi_o, g_o):
    ep = np.max(np.abs(phi - phi_o)) / np.max(np.abs(phi_o))
    eg = np.max(np.linalg.norm(g - g_o, axis=1)) / np.max(np.linalg.norm(g_o, axis=1))
    return ep, eg


def ctx(v, t, sigma, prec, far, **kw):
    c = lss.Context()
    c.set_sources(v, t, dunavant6())
    c.set_sigma(np.atleast_1d(np.asarray(sigma, float)))
    c.set_options(precision=prec, far_field=far, **kw)
    return c


@pytest.fixture(scope="module")
def graded():
    v, t = bumpy_sphere(40, grade=4.0, lmax=12, nbumps=60, seed=7)
    sig = 0.5 * triangle_diameters(v, t)
    x = surface_offset_targets(v, t, sig, 60000, tmax=3.0, seed=8)
    return v, t, sig, x


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_vs_direct_all_targets(graded, prec):
    v, t, sig, x = graded
    say("case: graded bumpy sphere %d tri, %d targets, FMM vs direct, precision %d" % (len(t), len(x), prec))
    cd = ctx(v, t, sig, lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(x)
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    pf, gf = cf.eval(x)
    st = cf.stats()
    say("  tree depth %d boxes %d leaves %d m2l %d p %d pairs/target %.0f" % (
        st["tree_depth"], st["n_boxes"], st["n_leaves"], st["n_m2l"], st["fmm_order"], st["last_pairs"] / len(x)))
    ep, eg = errs(pf, gf, pd, gd)
    say("  e_phi %.3e e_grad %.3e" % (ep, eg))
    assert st["n_m2l"] > 0 and st["tree_depth"] >= 3
    assert ep <= TOL[prec] and eg <= TOL[prec]


def test_fmm_fp64_tile_widths_agree(graded):
    """FP64 through the octree at 64-target tiles (the kernel that sends every
    node beyond its cut radius of the whole tile to the dipole-only loop) and at
    128 and 256 (one loop for every node): the same sums up to rounding order,
    all within the FP64 bar of the direct sum; only the narrow tiles use the
    dipole-only loop."""
    v, t, sig, x = graded
    say("case: FP64 FMM at tiles 64, 128, 256, %d targets" % len(x))
    cd = ctx(v, t, sig, lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(x)
    out = {}
    for tile in (64, 128, 256):
        cf = ctx(v, t, sig, lss.FP64, lss.FAR_FMM, tile=tile, count_useful=1)
        out[tile] = cf.eval(x)
        st = cf.stats()
        ep, eg = errs(*out[tile], pd, gd)
        say("  tile %d: e_phi %.3e e_grad %.3e, dipole-only pairs %.0f of %.0f" % (
            tile, ep, eg, st["dipole_pairs"], st["last_pairs"]))
        assert ep <= TOL[lss.FP64] and eg <= TOL[lss.FP64]
        assert (st["dipole_pairs"] > 0) == (tile == 64)
        assert st["useful_pairs"] <= st["last_pairs"] - st["dipole_pairs"]
    for tile in (128, 256):
        ep, eg = errs(*out[tile], *out[64])
        assert ep <= 1e-13 and eg <= 1e-13


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_vs_oracle_sampled(graded, prec):
    v, t, sig, x = graded
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(len(x), 1500, replace=False))
    po, go = oracle.evaluate(v, t, sig, dunavant6(), x[sel])
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    pf, gf = cf.eval(x)
    ep, eg = errs(pf[sel], gf[sel], po, go)
    say("case: FMM vs oracle, precision %d: e_phi %.3e e_grad %.3e" % (prec, ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]


def test_fmm_constant_sigma_sphere_deep_tree():
    v, t = icosphere(5)
    x = shell_targets(40000, 0.8, 1.2, seed=3)
    x = np.concatenate([x, box_targets(500, -3.0, 3.0, seed=4)])     # some outside the root cube
    say("case: icosphere-5 sigma 0.01, FMM vs direct, %d targets" % len(x))
    cd = ctx(v, t, [0.01], lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(x)
    for prec in (lss.FP64, lss.MIXED):
        cf = ctx(v, t, [0.01], prec, lss.FAR_FMM)
        pf, gf = cf.eval(x)
        ep, eg = errs(pf, gf, pd, gd)
        st = cf.stats()
        say("  prec %d depth %d m2l %d e_phi %.3e e_grad %.3e" % (prec, st["tree_depth"], st["n_m2l"], ep, eg))
        assert ep <= TOL[prec] and eg <= TOL[prec]


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_project_vs_oracle(prec):
    v, t = bumpy_sphere(16, grade=3.0, lmax=8, nbumps=10, seed=2)
    sig = 0.5 * triangle_diameters(v, t)
    uv = chart_nodes(2)
    say("case: FMM projection, %d tri, precision %d" % (len(t), prec))
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    h, xs, st, it = cf.project(uv)
    sel = np.arange(0, len(t), 53)
    tau = 1e-12 if prec == lss.FP64 else 1e-6
    ho, xo, sto, ito = oracle.project(v, t, sig, dunavant6(), uv, tau=tau, sel=sel)
    idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
    assert np.all(st[idx] == sto)
    eh = np.max(np.abs(h[idx] - ho) / sig[sel].repeat(len(uv)))
    say("  e_h %.3e iters max %d" % (eh, it.max()))
    assert eh <= (1e-11 if prec == lss.FP64 else 2e-6)


def test_fmm_determinism_and_device_pointers(graded):
    import torch
    v, t, sig, x = graded
    cf = ctx(v, t, sig, lss.FP64, lss.FAR_FMM)
    xd = torch.as_tensor(x, device="cuda")
    p1, g1 = cf.eval(xd)
    p2, g2 = cf.eval(xd)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(g1, g2)
    ph, gh = cf.eval(x)
    assert np.array_equal(p1.cpu().numpy(), ph)


def test_autotune_and_cache(graded, tmp_path):
    """lss_autotune searches leaf shrink, capacity, admissibility K and order
    p, accepting only candidates within a quarter of the bar against the
    exact sum; the choice meets the parity bar and is cached."""
    v, t, sig, x = graded
    cache = tmp_path / "tune.jsonl"
    for prec in (lss.MIXED, lss.FP64):
        cf = ctx(v, t, sig, prec, lss.FAR_FMM)
        o1 = cf.autotune(x[:20000], eval_weight=3.0, cache_path=cache)
        say("case: autotune precision %d -> %s" % (prec, o1))
        assert o1["tile"] in (64, 128, 256) and o1["leaf_capacity"] > 0 and 1.0 <= o1["leaf_shrink"] <= 3.0
        assert 4 <= o1["admissibility"] <= 18 and o1["fmm_order"] > 0   # K and p are searched too
        # the tuned options still meet the parity bar
        pf, gf = cf.eval(x[:3000])
        cd = ctx(v, t, sig, lss.FP64, lss.FAR_DIRECT)
        pd, gd = cd.eval(x[:3000])
        ep, eg = errs(pf, gf, pd, gd)
        assert ep <= TOL[prec] and eg <= TOL[prec]
        # a second context reads the cached choice without timing
        c2 = ctx(v, t, sig, prec, lss.FAR_FMM)
        o2 = c2.autotune(x[:20000], eval_weight=3.0, cache_path=cache)
        assert o2 == o1
    assert len(cache.read_text().strip().splitlines()) == 2


def test_fmm_project_repeated(graded):
    """FMM projection twice in a row (second call smaller) with an evaluation in
    between: identical answers to a fresh context, and to the oracle."""
    v, t, sig, _ = graded
    sel = np.arange(0, len(t), 97)
    for prec in (lss.MIXED, lss.FP64):
        say("case: repeated FMM projections, precision %d" % prec)
        cf = ctx(v, t, sig, prec, lss.FAR_FMM, newton_max_iter=12)
        tau = 1e-12 if prec == lss.FP64 else 1e-6
        for uv in (chart_nodes(2), chart_nodes(1)):
            h, xs, st, it = cf.project(uv)
            cf.eval(xs[:100])
            fresh = ctx(v, t, sig, prec, lss.FAR_FMM, newton_max_iter=12)
            h2, _, st2, it2 = fresh.project(uv)
            assert np.array_equal(h, h2) and np.array_equal(st, st2) and np.array_equal(it, it2)
            ho, xo, sto, ito = oracle.project(v, t, sig, dunavant6(), uv, tau=tau, sel=sel, max_iter=12)
            idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
            assert np.all(st[idx] == sto)
            eh = np.max(np.abs(h[idx] - ho) / sig[sel].repeat(len(uv)))
            say("  np %d e_h %.3e iters max %d" % (len(uv), eh, it.max()))
            assert eh <= (1e-11 if prec == lss.FP64 else 2e-6)


@pytest.fixture(scope="module")
def batch():
    """Five star-shaped surfaces of uneven size that overlap in space (any
    leak between meshes would show), per-triangle sigma, near-surface,
    box and far targets per mesh."""
    from workloads import configs, star_surface, bbox_targets
    meshes = []
    for i, (nu, shift) in enumerate([(12, 0.0), (4, 0.3), (20, 0.1), (2, 5.0), (9, -0.2)]):
        v, tt = star_surface(nu, lmax=8, var0=0.1, seed=40 + i)
        v = v + shift
        sig = 0.5 * triangle_diameters(v, tt)
        x = np.concatenate([surface_offset_targets(v, tt, sig, 1500, tmax=3.0, seed=60 + i),
                            bbox_targets(v, 300, pad=0.25, seed=80 + i),
                            shift + np.array([[12.0, 0.0, 0.0], [0.0, -9.0, 3.0]])])
        meshes.append(dict(verts=v, tris=tt, sigma=sig, targets=x))
    return configs.concat_batch(meshes)


def bctx(b, prec, far, **kw):
    c = lss.Context()
    c.set_sources(b["verts"], b["tris"], dunavant6(), tri_offsets=b["tri_offsets"])
    c.set_sigma(b["sigma"])
    c.set_options(precision=prec, far_field=far, **kw)
    return c


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_batch_vs_direct_and_oracle(batch, prec):
    b = batch
    say("case: FMM forest, batch of %d meshes, %d tri, %d targets, precision %d" % (
        len(b["tri_offsets"]) - 1, len(b["tris"]), len(b["targets"]), prec))
    cf = bctx(b, prec, lss.FAR_FMM)
    pf, gf = cf.eval(b["targets"], x_mesh=b["target_mesh"])
    cd = bctx(b, lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(b["targets"], x_mesh=b["target_mesh"])
    ep, eg = errs(pf, gf, pd, gd)
    say("  vs direct: e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]
    sel = np.arange(0, len(b["targets"]), 23)
    po, go = oracle.evaluate(b["verts"], b["tris"], b["sigma"], dunavant6(), b["targets"][sel],
                             tri_offsets=b["tri_offsets"], x_mesh=b["target_mesh"][sel])
    ep, eg = errs(pf[sel], gf[sel], po, go)
    say("  vs oracle: e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]
    st = cf.stats()
    assert st["n_mesh"] == 5 and st["n_boxes"] >= 5


def test_fmm_batch_project_vs_oracle(batch):
    b = batch
    uv = chart_nodes(2)
    ntri = len(b["tris"])
    sel = np.arange(0, ntri, 31)
    idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
    for prec in (lss.FP64, lss.MIXED):
        say("case: FMM forest projection, precision %d" % prec)
        cf = bctx(b, prec, lss.FAR_FMM)
        h, xs, st, it = cf.project(uv)
        tau = 1e-12 if prec == lss.FP64 else 1e-6
        ho, xo, sto, ito = oracle.project(b["verts"], b["tris"], b["sigma"], dunavant6(), uv, tau=tau, sel=sel,
                                          tri_offsets=b["tri_offsets"])
        assert np.all(st[idx] == sto)
        eh = np.max(np.abs(h[idx] - ho) / b["sigma"][sel].repeat(len(uv)))
        say("  e_h %.3e iters max %d" % (eh, it.max()))
        assert eh <= (1e-11 if prec == lss.FP64 else 2e-6)


def test_fmm_mixed_eval_reproducible_and_counters(graded):
    """The work queue hands tiles out in cost order, so workgroups meet the
    tiles in a different order every run; the results must still be bitwise
    identical between contexts, and the pair counters consistent."""
    v, t, sig, x = graded
    out = []
    for _ in range(2):
        cf = ctx(v, t, sig, lss.MIXED, lss.FAR_FMM)
        out.append(cf.eval(x))
        st = cf.stats()
        assert 0 < st["last_pairs"] <= st["lane_pairs"] <= 64 * st["last_pairs"]
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_project_graph_reuse(graded, prec):
    """The captured Newton iterations are reused by later projections whose
    buffers, sizes and options match: the same call twice, then a new sigma
    (rebuilt tree, same sizes) and back, each equal bit for bit to a fresh
    context's projection."""
    v, t, sig, _ = graded
    uv = chart_nodes(2)
    say("case: Newton graph reuse, precision %d" % prec)
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    first = cf.project(uv)
    again = cf.project(uv)
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    for s in (0.9 * sig, sig):
        cf.set_sigma(s)
        got = cf.project(uv)
        want = ctx(v, t, s, prec, lss.FAR_FMM).project(uv)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
    for a, b in zip(got, first):
        assert np.array_equal(a, b)


def useful_pairs_brute(v, t, sig, x, cut):
    """Pairs (target, node) with |x - y_k| < cut * sigma_k, by a k-d tree over
    the nodes (every node within cut * max sigma, then each node's own radius)."""
    from scipy.spatial import cKDTree
    y, _ = oracle.nodes(v, t, dunavant6())
    sk = np.repeat(np.asarray(sig, float), len(dunavant6()))
    tree = cKDTree(y)
    n = 0
    for i, cand in enumerate(tree.query_ball_point(x, cut * sk.max(), workers=-1)):
        cand = np.asarray(cand, dtype=np.int64)
        d2 = ((y[cand] - x[i]) ** 2).sum(1)
        n += int(np.count_nonzero(d2 < (cut * sk[cand]) ** 2))
    return n


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_useful_pair_count(graded, prec):
    """With count_useful the evaluation kernels count the pairs inside their
    node's cut radius (section 4.4: the near field is the ball of radius cut
    around the target).  Every such pair lies on a near list, so the count
    equals a brute-force count by distance; the decision u < cut^2 / 2 is taken
    in the kernel's precision, so pairs within rounding of the cut may differ
    (none expected at this size).  Results do not depend on the option."""
    v, t, sig, x = graded
    rng = np.random.default_rng(11)
    xs = x[np.sort(rng.choice(len(x), 2000, replace=False))]
    cut = 8.0 if prec == lss.FP64 else np.sqrt(40.0)
    want = useful_pairs_brute(v, t, sig, xs, cut)
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    p0, g0 = cf.eval(xs)
    assert cf.stats()["useful_pairs"] == 0.0
    cf.set_options(precision=prec, far_field=lss.FAR_FMM, count_useful=1)
    p1, g1 = cf.eval(xs)
    st = cf.stats()
    say("  precision %d useful pairs %.0f (brute force %d), executed %.0f (%.2fx)" % (
        prec, st["useful_pairs"], want, st["last_pairs"], st["last_pairs"] / max(st["useful_pairs"], 1)))
    assert abs(st["useful_pairs"] - want) <= 2 + 1e-7 * want
    assert st["useful_pairs"] <= st["last_pairs"]
    # the dipole-only loop (nodes beyond the cut of every target of a tile)
    # takes none of the pairs inside the cut
    say("  dipole-only pairs %.0f, full-kernel pairs %.0f" % (st["dipole_pairs"], st["last_pairs"] - st["dipole_pairs"]))
    assert 0.0 < st["dipole_pairs"] and st["useful_pairs"] <= st["last_pairs"] - st["dipole_pairs"]
    assert np.array_equal(p0, p1) and np.array_equal(g0, g1)
    cd = ctx(v, t, sig, prec, lss.FAR_DIRECT)
    cd.eval(xs[:100])
    sd = cd.stats()
    assert sd["useful_pairs"] == sd["last_pairs"] == 100 * 12 * len(t)


@pytest.fixture(scope="module")
def volume():
    """Graded bumpy sphere with targets filling a cube around it: many sit in
    coarse empty leaves inside and outside the surface, whose direct lists
    would take whole subtrees without the M2P descent."""
    v, t = bumpy_sphere(30, grade=4.0, lmax=10, nbumps=40, seed=11)
    sig = 0.5 * triangle_diameters(v, t)
    x = box_targets(30000, -1.3, 1.3, seed=12)
    return v, t, sig, x


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_m2p_volume_targets(volume, prec):
    v, t, sig, x = volume
    say("case: volume targets, %d tri, %d targets, precision %d" % (len(t), len(x), prec))
    cd = ctx(v, t, sig, lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(x)
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    pf, gf = cf.eval(x)
    st = cf.stats()
    say("  boxes %d m2l %d m2p %d pairs/target %.0f (nodes %d)" % (
        st["n_boxes"], st["n_m2l"], st["n_m2p"], st["last_pairs"] / len(x), st["n_nodes"]))
    ep, eg = errs(pf, gf, pd, gd)
    say("  vs direct: e_phi %.3e e_grad %.3e" % (ep, eg))
    assert st["n_m2p"] > 0
    assert st["last_pairs"] / len(x) < 0.25 * st["n_nodes"]
    assert ep <= TOL[prec] and eg <= TOL[prec]
    rng = np.random.default_rng(13)
    sel = np.sort(rng.choice(len(x), 400, replace=False))
    po, go = oracle.evaluate(v, t, sig, dunavant6(), x[sel])
    ep, eg = errs(pf[sel], gf[sel], po, go)
    say("  vs oracle (400 sampled): e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_fmm_targets_outside_root_cube(prec):
    """Targets outside the padded root cube take the far field from a
    stackless walk of the tree (multipoles where the M2P test passes, direct
    sums of the leaves where it does not), not a direct sum over the mesh."""
    v, t = icosphere(4)
    sig = 0.05
    xo = shell_targets(3000, 7.0, 12.0, seed=21)         # outside the root cube (half side <= 3.6)
    x = np.concatenate([xo, box_targets(1000, -1.6, 1.6, seed=22)])
    cd = ctx(v, t, sig, lss.FP64, lss.FAR_DIRECT)
    pd, gd = cd.eval(x)
    cf = ctx(v, t, sig, prec, lss.FAR_FMM)
    cf.eval(xo)
    st = cf.stats()
    say("case: outside targets, precision %d: direct pairs/target %.0f of %d nodes" % (
        prec, st["last_pairs"] / len(xo), st["n_nodes"]))
    assert st["last_pairs"] / len(xo) < 0.05 * st["n_nodes"]
    pf, gf = cf.eval(x)
    ep, eg = errs(pf, gf, pd, gd)
    say("  with 1000 volume targets: e_phi %.3e e_grad %.3e" % (ep, eg))
    assert ep <= TOL[prec] and eg <= TOL[prec]
