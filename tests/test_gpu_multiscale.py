"""GPU parity of Phi / grad Phi with the paper's target-attached width
sigma(x) (section 2, eq. sigma2: the Gaussian blend of sigma_j = D_j/lambda
over the triangle centroids), direct FP64 sum, against the oracle: Phi,
grad Phi (with the (dPhi/dsigma) grad sigma term) and sigma(x) within 1e-12
(max error relative to the largest oracle value)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1909_13356_amd as lss
from workloads import (dunavant6, cube_mesh, star_surface, torus_mesh, triangle_diameters,
                       surface_offset_targets, box_targets)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.max(np.abs(np.asarray(a) - b)) / np.max(np.abs(b))


def ctx(v, t, offsets=None):
    c = lss.Context()
    c.set_sources(v, t, dunavant6(), tri_offsets=offsets)
    return c


@pytest.mark.parametrize("lam,sigma0", [(2.5, 0.0), (2.5, 0.15), (1.0, 0.05)])
def test_multiscale_vs_oracle(lam, sigma0):
    v, t = star_surface(8, lmax=8, var0=0.1, seed=6)
    sig = 0.5 * triangle_diameters(v, t)
    x = np.concatenate([surface_offset_targets(v, t, sig, 2000, tmax=3.0, seed=7),
                        box_targets(200, -2.0, 2.0, seed=8)])
    say("case: multiscale sigma(x), star surface %d tri, lambda %g sigma0 %g, %d targets" % (len(t), lam, sigma0, len(x)))
    p, g, s = ctx(v, t).eval_multiscale(x, lam, sigma0)
    po, go, so = oracle.evaluate_multiscale(v, t, dunavant6(), x, lam, sigma0)
    e = rel(p, po), rel(g, go), rel(s, so)
    say("  e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= 1e-12


@pytest.mark.parametrize("far,interp", [(lss.FAR_DIRECT, 0), (lss.FAR_FMM, 1), (lss.FAR_FMM, 2)])
def test_multiscale_batch_of_a_quadratic_torus_and_a_cube(far, interp):
    vt, tt = torus_mesh(16, 8, quadratic=True)
    vc, tc = cube_mesh(4, 2.0, 3.0)
    # the cube as quadratic triangles with their own (unshared) edge midpoints
    mids = 0.5 * (vc[tc[:, [0, 1, 2]]] + vc[tc[:, [1, 2, 0]]]).reshape(-1, 3)
    v = np.concatenate([vt, vc, mids])
    tcq = np.column_stack([tc + len(vt), len(vt) + len(vc) + np.arange(3 * len(tc)).reshape(-1, 3)])
    t6 = np.concatenate([tt, tcq]).astype(np.int32)
    off = np.array([0, len(tt), len(t6)], np.int64)
    x = np.concatenate([box_targets(300, -1.5, 1.5, seed=1), box_targets(300, 1.8, 3.2, seed=3)])
    xm = np.repeat(np.array([0, 1], np.int32), [300, 300])
    say("case: multiscale, batch of a quadratic torus and a cube, far field %d, sigma_interp %d" % (far, interp))
    c = ctx(v, t6, offsets=off)
    c.set_options(precision=lss.FP64, far_field=far, sigma_interp=interp)
    p, g, s = c.eval_multiscale(x, 2.5, 0.0, x_mesh=xm)
    po, go, so = oracle.evaluate_multiscale(v, t6, dunavant6(), x, 2.5, 0.0, tri_offsets=off, x_mesh=xm)
    e = rel(p, po), rel(g, go), rel(s, so)
    say("  e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= 1e-12
    bad = xm.copy()
    bad[3] = 2
    with pytest.raises(lss.LssError) as err:
        c.eval_multiscale(x, 2.5, 0.0, x_mesh=bad)
    assert err.value.code == 1


def test_multiscale_constant_diameter_is_the_constant_sigma_sum_and_device_tensors():
    import torch
    v, t = cube_mesh(6)
    D = np.sqrt(2) / 6
    x = box_targets(1500, -0.5, 1.5, seed=4)
    say("case: multiscale on congruent triangles vs constant sigma; device tensors; errors")
    c = ctx(v, t)
    with pytest.raises(lss.LssError) as err:
        c.eval_multiscale(x, 0.0)
    assert err.value.code == 1
    p, g, s = c.eval_multiscale(x, 2.5)
    assert np.allclose(s, D / 2.5, rtol=1e-13, atol=0)
    c.set_sigma(np.array([D / 2.5]))
    c.set_options(precision=lss.FP64, far_field=lss.FAR_DIRECT)
    p0, g0 = c.eval(x)
    assert rel(p, p0) <= 1e-12 and rel(g, g0) <= 1e-12
    pd, gd, sd = c.eval_multiscale(torch.as_tensor(x, device="cuda"), 2.5)
    torch.cuda.synchronize()
    assert np.array_equal(pd.cpu().numpy(), p) and np.array_equal(gd.cpu().numpy(), g)
    with pytest.raises(lss.LssError) as err:
        lss.Context().eval_multiscale(x, 2.5)
    assert err.value.code == 4


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_multiscale_through_the_octree(prec):
    """sigma(x) through the tree: leaves sized by sigma at the centroids,
    lists built for these targets (a far interaction clears cut * sigma(x) of
    every target in the box), near pairs at the target's width, far field
    from the expansions.  Bars 1e-12 (FP64 settings) and 1e-6 (mixed
    settings: cut sqrt(40) sigma(x), p = 20).  The context's own sigma and
    results are unchanged afterwards."""
    v, t = star_surface(10, lmax=8, var0=0.1, seed=9)
    sig = 0.5 * triangle_diameters(v, t)
    x = np.concatenate([surface_offset_targets(v, t, sig, 6000, tmax=3.0, seed=10),
                        box_targets(500, -2.0, 2.0, seed=11),
                        np.array([[9.0, 0.1, 0.2], [-0.3, 8.0, -1.0]])])        # outside the root cube
    say("case: multiscale sigma(x) through the octree, star surface %d tri, %d targets, precision %d"
        % (len(t), len(x), prec))
    c = ctx(v, t)
    c.set_sigma(sig)
    c.set_options(precision=prec, far_field=lss.FAR_FMM)
    p0, g0 = c.eval(x)
    p, g, s = c.eval_multiscale(x, 2.5, 0.0)
    st = c.stats()
    assert st["n_m2l"] > 0
    po, go, so = oracle.evaluate_multiscale(v, t, dunavant6(), x[::5], 2.5, 0.0)
    bar = 1e-12 if prec == lss.FP64 else 1e-6
    e = rel(p[::5], po), rel(g[::5], go), rel(s[::5], so)
    say("  vs oracle: e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= bar
    cd = ctx(v, t)
    pd, gd, sd = cd.eval_multiscale(x, 2.5, 0.0)               # the direct path on every target
    assert rel(p, pd) <= bar and rel(g, gd) <= bar
    p1, g1 = c.eval(x)
    assert np.array_equal(p1, p0) and np.array_equal(g1, g0)


@pytest.mark.parametrize("sigma0", [0.0, 0.04])
def test_multiscale_octree_on_a_graded_torus(sigma0):
    """A torus whose triangle diameters vary about 30x, so sigma(x) varies
    strongly from one region to the next (sigma0 = 0.04 makes it follow the
    local triangles closely): the octree path against the every-pair path on
    all targets and the oracle on a sample, FP64 settings."""
    from workloads import graded_torus
    v, t = graded_torus(n_tris=12000, seed=21)
    sig = 0.5 * triangle_diameters(v, t)
    x = np.concatenate([surface_offset_targets(v, t, sig, 8000, tmax=3.0, seed=22),
                        box_targets(300, -1.5, 1.5, seed=23)])
    say("case: multiscale through the octree, graded torus %d tri (diameters %.0fx), sigma0 %g, %d targets"
        % (len(t), (2 * sig).max() / (2 * sig).min(), sigma0, len(x)))
    c = ctx(v, t)
    c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM)
    p, g, s = c.eval_multiscale(x, 2.5, sigma0)
    st = c.stats()
    say("  leaves %d m2l %d pairs/target %.0f" % (st["n_leaves"], st["n_m2l"], st["last_pairs"] / len(x)))
    cd = ctx(v, t)
    pd, gd, sd = cd.eval_multiscale(x, 2.5, sigma0)
    e = rel(p, pd), rel(g, gd), rel(s, sd)
    say("  vs every pair: e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= 1e-12
    po, go, so = oracle.evaluate_multiscale(v, t, dunavant6(), x[::40], 2.5, sigma0)
    e = rel(p[::40], po), rel(g[::40], go), rel(s[::40], so)
    say("  vs oracle: e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= 1e-12


def test_sigma_interpolation_against_the_direct_sum():
    """sigma(x) from the Chebyshev cells (sigma_interp = 2) against the direct
    sum (sigma_interp = 1), octree path, on a graded torus with sigma0 =
    sqrt(5) max D: near-surface and box targets, the centre of the hole
    (within 3 sigma0 of the centroids: interpolated), points 4 sigma0 above
    the torus (cells beyond 3 sigma0: direct sum) and far outside the grid
    (direct sum).  sigma within 1e-13, Phi and grad Phi (which carries grad
    sigma) within 1e-12; the automatic choice equals one of the two; the
    oracle on a sample."""
    from workloads import graded_torus
    v, t = graded_torus(n_tris=12000, seed=21)
    sig = 0.5 * triangle_diameters(v, t)
    s0 = np.sqrt(5.0) * (2 * sig).max()
    cen = v[t].mean(1)
    lo, hi = cen.min(0), cen.max(0)
    # two points within 3 sigma0 of the centroids' box (inside the grid) in
    # corner cells more than 3 sigma0 from every centroid, two outside it
    x = np.concatenate([surface_offset_targets(v, t, sig, 8000, tmax=3.0, seed=24),
                        box_targets(300, -1.5, 1.5, seed=25),
                        np.array([[0.0, 0.0, 0.0], [hi[0] + 2.5 * s0, hi[1] + 2.5 * s0, 0.0],
                                  [lo[0] - 2.6 * s0, hi[1] + 2.4 * s0, 0.1], [9.0, 1.0, 2.0], [-40.0, 3.0, 0.0]])])
    say("case: sigma(x) interpolation vs the direct sum, graded torus %d tri, sigma0 %.3f, %d targets"
        % (len(t), s0, len(x)))
    out = {}
    for mode in (1, 2, 0):
        c = ctx(v, t)
        c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM, sigma_interp=mode)
        out[mode] = c.eval_multiscale(x, 2.5, 0.0)
        c.close()
    (pd, gd, sd), (pi, gi, si) = out[1], out[2]
    e = rel(pi, pd), rel(gi, gd), rel(si, sd)
    say("  interpolated vs direct sum: e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert e[0] <= 1e-12 and e[1] <= 1e-12 and e[2] <= 1e-13
    assert not np.array_equal(si, sd)                       # the cells were used
    assert np.array_equal(si[-4:], sd[-4:])                 # the direct sum beyond 3 sigma0 and the grid
    pa, ga, sa = out[0]
    assert np.array_equal(sa, sd) or np.array_equal(sa, si)
    sel = np.concatenate([np.arange(0, 8300, 83), np.arange(8300, len(x))])
    po, go, so = oracle.evaluate_multiscale(v, t, dunavant6(), x[sel], 2.5, 0.0)
    e = rel(pi[sel], po), rel(gi[sel], go), rel(si[sel], so)
    say("  interpolated vs oracle: e_phi %.2e e_grad %.2e e_sigma %.2e" % e)
    assert max(e) <= 1e-12
