"""lss_eval_noalloc (the allocation-free evaluation) against lss_eval through
the C ABI: the same kernels on the same inputs, so the outputs must be equal
bit for bit.  Two calls in a row, the second with fewer targets, so the
shared static scratch array is reused with stale contents from the first;
direct and octree paths, both precisions, a ragged batch with mesh ids, and
the error cases (host arrays, too many targets, unbuilt context)."""
import sys

import numpy as np
import pytest

import paper_1909_13356_amd as lss
from workloads import (dunavant6, bumpy_sphere, star_surface, triangle_diameters, surface_offset_targets,
                       bbox_targets, configs)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def graded():
    v, t = bumpy_sphere(24, grade=4.0, lmax=10, nbumps=40, seed=17)
    sig = 0.5 * triangle_diameters(v, t)
    x = np.concatenate([surface_offset_targets(v, t, sig, 90000, tmax=3.0, seed=18),
                        bbox_targets(v, 3000, pad=0.5, seed=19)])
    return v, t, sig, x


def _same(c, xd, n):
    import torch
    xs = xd[:n].contiguous()
    p0, g0 = c.eval(xs)
    p1 = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    g1 = torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda")
    c.eval_noalloc(xs, p1, g1)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and torch.equal(g0, g1), n


@pytest.mark.parametrize("far", [lss.FAR_FMM, lss.FAR_DIRECT])
@pytest.mark.parametrize("prec", [lss.FP64, lss.MIXED])
def test_noalloc_matches_eval_twice(graded, far, prec):
    import torch
    v, t, sig, x = graded
    say("case: noalloc vs eval, %d tri, far %d precision %d" % (len(t), far, prec))
    c = lss.Context()
    c.set_sources(v, t, dunavant6())
    c.set_sigma(sig)
    c.set_options(precision=prec, far_field=far)
    c.build()
    xd = torch.as_tensor(x, device="cuda")
    n1 = len(x) if far == lss.FAR_FMM else 20000
    for n in (n1, 4099):                # the second call is smaller: stale scratch from the first
        _same(c, xd, n)
    st0 = c.stats()
    p = torch.empty(777, dtype=torch.float64, device="cuda")
    c.eval_noalloc(xd[:777].contiguous(), p, None)          # grad may be null
    torch.cuda.synchronize()
    assert c.stats()["last_targets"] == st0["last_targets"]   # statistics untouched
    p0, _ = c.eval(xd[:777].contiguous())
    assert torch.equal(p, p0)
    c.close()


def test_noalloc_batch_with_mesh_ids():
    import torch
    meshes = []
    for i, (nu, shift) in enumerate([(10, 0.0), (3, 0.25), (14, -0.1)]):
        v, tt = star_surface(nu, lmax=8, var0=0.1, seed=140 + i)
        v = v + shift
        sig = 0.5 * triangle_diameters(v, tt)
        xx = np.concatenate([surface_offset_targets(v, tt, sig, 2000, tmax=3.0, seed=160 + i),
                             bbox_targets(v, 300, pad=0.25, seed=180 + i)])
        meshes.append(dict(verts=v, tris=tt, sigma=sig, targets=xx))
    b = configs.concat_batch(meshes)
    say("case: noalloc batch of 3 meshes, %d targets" % len(b["targets"]))
    for far in (lss.FAR_FMM, lss.FAR_DIRECT):
        c = lss.Context()
        c.set_sources(b["verts"], b["tris"], dunavant6(), tri_offsets=b["tri_offsets"])
        c.set_sigma(b["sigma"])
        c.set_options(precision=lss.FP64, far_field=far)
        c.build()
        xd = torch.as_tensor(b["targets"], device="cuda")
        md = torch.as_tensor(b["target_mesh"], device="cuda")
        for n in (len(b["targets"]), 1234):
            p0, g0 = c.eval(xd[:n].contiguous(), x_mesh=md[:n].contiguous())
            p1 = torch.empty(n, dtype=torch.float64, device="cuda")
            g1 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
            c.eval_noalloc(xd[:n].contiguous(), p1, g1, x_mesh=md[:n].contiguous())
            torch.cuda.synchronize()
            assert torch.equal(p0, p1) and torch.equal(g0, g1), (far, n)
        bad = md[:10].clone()
        bad[3] = 7
        with pytest.raises(lss.LssError) as e:
            c.eval_noalloc(xd[:10].contiguous(), torch.empty(10, dtype=torch.float64, device="cuda"), None,
                           x_mesh=bad)
        assert e.value.code == 1
        c.close()


def test_noalloc_errors(graded):
    import torch
    v, t, sig, x = graded
    c = lss.Context()
    c.set_sources(v, t, dunavant6())
    c.set_sigma(sig)
    c.set_options(precision=lss.FP64, far_field=lss.FAR_FMM)
    p = torch.empty(10, dtype=torch.float64, device="cuda")
    xd = torch.as_tensor(x[:10], device="cuda")
    with pytest.raises(lss.LssError) as e:
        c.eval_noalloc(xd, p, None)                             # not built: this call does not build
    assert e.value.code == 4
    c.build()
    with pytest.raises(lss.LssError) as e:
        c.eval_noalloc(x[:10], np.empty(10), None)              # host arrays
    assert e.value.code == 1
    big = torch.zeros((524289, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(lss.LssError) as e:
        c.eval_noalloc(big, torch.empty(524289, dtype=torch.float64, device="cuda"), None)
    assert e.value.code == 1 and "LSS_NOALLOC_MAX_TARGETS" in str(e.value)
    c.eval_noalloc(xd, p, None)                                 # the context still works
    torch.cuda.synchronize()
    p0, _ = c.eval(xd)
    assert torch.equal(p, p0)
    c.close()
