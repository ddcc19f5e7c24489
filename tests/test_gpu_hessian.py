"""GPU parity of the Hessian of Phi (direct FP64 sum with the third radial
function) and of the charts' second derivatives and curvatures, against the
oracle.  Bars: Hessian, Phi and grad Phi 1e-12 (max error relative to the
largest oracle value); chart second derivatives and curvatures 1e-10 (they
divide by H . grad Phi and by the first fundamental form)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1909_13356_amd as lss
from workloads import (dunavant6, chart_nodes, icosphere, star_surface, torus_mesh, triangle_diameters,
                       surface_offset_targets, box_targets)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.max(np.abs(np.asarray(a) - b)) / np.max(np.abs(b))


def ctx(v, t, sigma, offsets=None, far=lss.FAR_FMM):
    c = lss.Context()
    c.set_sources(v, t, dunavant6(), tri_offsets=offsets)
    c.set_sigma(np.atleast_1d(np.asarray(sigma, float)))
    c.set_options(precision=lss.FP64, far_field=far)
    return c


@pytest.fixture(scope="module")
def star():
    v, t = star_surface(8, lmax=8, var0=0.1, seed=6)
    sig = 0.5 * triangle_diameters(v, t)
    return v, t, sig


def test_hessian_vs_oracle(star):
    v, t, sig = star
    x = np.concatenate([surface_offset_targets(v, t, sig, 2500, tmax=3.0, seed=7),
                        box_targets(300, -2.0, 2.0, seed=8)])
    say("case: Hessian by the direct sum, star surface %d tri, %d targets" % (len(t), len(x)))
    c = ctx(v, t, sig, far=lss.FAR_DIRECT)
    phi, g, hs = c.eval_hessian(x)
    ho = oracle.hessian(v, t, sig, dunavant6(), x)
    po, go = oracle.evaluate(v, t, sig, dunavant6(), x)
    eh, ep, eg = rel(hs, ho), rel(phi, po), rel(g, go)
    say("  e_hess %.3e e_phi %.3e e_grad %.3e" % (eh, ep, eg))
    assert eh <= 1e-12 and ep <= 1e-12 and eg <= 1e-12


def test_hessian_batch_and_quadratic_skeleton():
    vt, tt = torus_mesh(24, 12, quadratic=True)
    vs, ts = icosphere(2)
    vs6 = np.concatenate([vs, 0.5 * (vs[ts[:, [0, 1, 2]]] + vs[ts[:, [1, 2, 0]]]).reshape(-1, 3)])
    n0 = len(vs)
    mids = n0 + 3 * np.arange(len(ts))[:, None] + np.arange(3)[None]
    ts6 = np.concatenate([ts, mids], axis=1).astype(np.int32)     # unshared edge points at the midpoints
    vs6 = 0.6 * vs6 + np.array([2.5, 0.0, 0.0])
    v = np.concatenate([vt, vs6])
    t = np.concatenate([tt, ts6 + len(vt)]).astype(np.int32)
    off = np.array([0, len(tt), len(t)], np.int64)
    x = np.concatenate([box_targets(600, -1.6, 1.6, seed=2), box_targets(400, 1.8, 3.2, seed=3)])
    xm = np.concatenate([np.zeros(600, np.int32), np.ones(400, np.int32)])
    say("case: Hessian, ragged batch of a quadratic torus and a sphere, %d targets" % len(x))
    c = ctx(v, t, [0.07], offsets=off)
    _, _, hs = c.eval_hessian(x, x_mesh=xm)
    ho = oracle.hessian(v, t, [0.07], dunavant6(), x, tri_offsets=off, x_mesh=xm)
    e = rel(hs, ho)
    say("  e_hess %.3e" % e)
    assert e <= 1e-12
    bad = xm.copy()
    bad[7] = 2
    with pytest.raises(lss.LssError) as err:
        c.eval_hessian(x, x_mesh=bad)
    assert err.value.code == 1


def test_chart_curvature_vs_oracle(star):
    v, t, sig = star
    uv = chart_nodes(4)
    say("case: chart curvature, star surface %d tri, p = 4" % len(t))
    c = ctx(v, t, sig)
    h, x, st, it = c.project(uv)
    assert np.all(st == 0)
    xuu, xuv, xvv, K, Hm = c.chart_curvature(uv, h)
    sel = np.arange(0, len(t), 13)
    idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
    o = oracle.chart_curvature(v, t, sig, dunavant6(), uv, h[idx], sel=sel)
    errs = [rel(a[idx], b) for a, b in zip((xuu, xuv, xvv, K, Hm), o)]
    say("  e_xuu %.2e e_xuv %.2e e_xvv %.2e e_gauss %.2e e_mean %.2e" % tuple(errs))
    assert max(errs) <= 1e-10
    assert np.all(np.isfinite(K)) and np.all(np.isfinite(Hm))


def test_chart_curvature_sphere_and_device_tensors():
    import torch
    v, t = icosphere(4)
    uv = chart_nodes(2)
    say("case: chart curvature on an icosphere, device tensors")
    c = ctx(v, t, [0.05])
    h, x, st, it = c.project(uv)
    assert np.all(st == 0)
    xuu, xuv, xvv, K, Hm = c.chart_curvature(uv, h)
    R = np.linalg.norm(x, axis=1)
    say("  max |K R^2 - 1| %.2e  max |H R - 1| %.2e" % (np.abs(K * R * R - 1).max(), np.abs(Hm * R - 1).max()))
    assert np.abs(K * R * R - 1).max() < 5e-2 and np.abs(Hm * R - 1).max() < 2.5e-2
    hd = torch.as_tensor(h, device="cuda")
    out = c.chart_curvature(torch.as_tensor(uv, device="cuda"), hd)
    torch.cuda.synchronize()
    for a, b in zip(out, (xuu, xuv, xvv, K, Hm)):
        assert np.array_equal(a.cpu().numpy(), b)
    xd = torch.as_tensor(x[:500], device="cuda")
    pd, gd, hsd = c.eval_hessian(xd)
    p, g, hs = c.eval_hessian(x[:500])
    torch.cuda.synchronize()
    assert np.array_equal(hsd.cpu().numpy(), hs) and np.array_equal(pd.cpu().numpy(), p)


@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_hessian_fmm_vs_oracle_and_direct(star, prec):
    """The Hessian through the octree: near lists with the full kernel, M2P
    lists and local expansions with their second derivatives.  Bars: Phi and
    grad as for lss_eval; the Hessian 1e-10 (FP64 settings: the kernel at the
    8 sigma cut differs from the Laplace double layer by 2e-11 in its third
    radial function) and 1e-5 (mixed settings: cut sqrt(40) sigma, p = 20)."""
    v, t, sig = star
    x = np.concatenate([surface_offset_targets(v, t, sig, 4000, tmax=3.0, seed=17),
                        box_targets(400, -2.0, 2.0, seed=18),
                        np.array([[6.0, 0.5, -0.3], [0.2, -7.0, 1.0]])])      # outside the root cube
    say("case: Hessian through the FMM, star surface %d tri, %d targets, precision %d" % (len(t), len(x), prec))
    c = ctx(v, t, sig, far=lss.FAR_FMM)
    c.set_options(precision=prec, far_field=lss.FAR_FMM)
    phi, g, hs = c.eval_hessian(x)
    st = c.stats()
    assert st["n_m2l"] > 0
    cd = ctx(v, t, sig, far=lss.FAR_DIRECT)
    pd, gd, hd = cd.eval_hessian(x)
    ho = oracle.hessian(v, t, sig, dunavant6(), x[::7])
    bar_f = 1e-12 if prec == lss.FP64 else 1e-6
    bar_h = 1e-10 if prec == lss.FP64 else 1e-5
    e = rel(hs, hd), rel(phi, pd), rel(g, gd), rel(hs[::7], ho)
    say("  vs direct: e_hess %.2e e_phi %.2e e_grad %.2e; vs oracle: e_hess %.2e" % e)
    assert e[0] <= bar_h and e[3] <= bar_h and e[1] <= bar_f and e[2] <= bar_f


def test_chart_curvature_through_the_fmm(star):
    v, t, sig = star
    uv = chart_nodes(4)
    say("case: chart curvature through the FMM, star surface %d tri" % len(t))
    c = ctx(v, t, sig, far=lss.FAR_FMM)
    h, x, st, it = c.project(uv)
    assert np.all(st == 0)
    out = c.chart_curvature(uv, h)
    cd = ctx(v, t, sig, far=lss.FAR_DIRECT)
    ref = cd.chart_curvature(uv, h)
    errs = [rel(a, b) for a, b in zip(out, ref)]
    say("  vs direct: e_xuu %.2e e_xuv %.2e e_xvv %.2e e_gauss %.2e e_mean %.2e" % tuple(errs))
    assert max(errs) <= 1e-9


@pytest.mark.parametrize("tile", [128, 256])
def test_hessian_and_sigma_x_fmm_wide_tiles(star, tile):
    """The octree Hessian and sigma(x) kernels at the wider FP64 tiles."""
    v, t, sig = star
    x = surface_offset_targets(v, t, sig, 3000, tmax=3.0, seed=23)
    say("case: Hessian and sigma(x) through the FMM with tile %d" % tile)
    c = ctx(v, t, sig, far=lss.FAR_FMM)
    c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM, tile=tile)
    _, _, hs = c.eval_hessian(x)
    p, g, s = c.eval_multiscale(x, 2.5, 0.0)
    cd = ctx(v, t, sig, far=lss.FAR_DIRECT)
    _, _, hd = cd.eval_hessian(x)
    pd, gd, sd = cd.eval_multiscale(x, 2.5, 0.0)
    e = rel(hs, hd), rel(p, pd), rel(g, gd)
    say("  e_hess %.2e e_phi %.2e e_grad %.2e" % e)
    assert e[0] <= 1e-10 and e[1] <= 1e-12 and e[2] <= 1e-12


def test_chart_curvature_batch_vs_oracle():
    """Two surfaces in one context: every chart's curvature from its own mesh."""
    v1, t1 = star_surface(5, lmax=6, var0=0.1, seed=31)
    v2, t2 = icosphere(2)
    v2 = 0.5 * v2 + np.array([3.0, 0.0, 0.0])
    v = np.concatenate([v1, v2])
    t = np.concatenate([t1, t2 + len(v1)]).astype(np.int32)
    off = np.array([0, len(t1), len(t)], np.int64)
    sig = 0.5 * triangle_diameters(v, t)
    uv = chart_nodes(2)
    say("case: chart curvature on a batch of two surfaces, %d tri" % len(t))
    c = ctx(v, t, sig, offsets=off)
    h, x, st, it = c.project(uv)
    assert np.all(st == 0)
    out = c.chart_curvature(uv, h)
    sel = np.arange(0, len(t), 9)
    idx = (sel[:, None] * len(uv) + np.arange(len(uv))[None]).ravel()
    o = oracle.chart_curvature(v, t, sig, dunavant6(), uv, h[idx], sel=sel, tri_offsets=off)
    errs = [rel(a[idx], b) for a, b in zip(out, o)]
    say("  e_xuu %.2e e_xuv %.2e e_xvv %.2e e_gauss %.2e e_mean %.2e" % tuple(errs))
    assert max(errs) <= 1e-9
