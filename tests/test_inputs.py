"""Checks of the seeded input generators (meshes, rules, node sets, targets)."""
from math import factorial

import numpy as np
import pytest

from workloads import (dunavant6, chart_nodes, chart_nodes_45, cube_mesh, icosphere,
                       geodesic_sphere, star_surface, bumpy_sphere, mesh_check,
                       triangle_diameters, refine_1to4, box_targets, shell_targets,
                       surface_offset_targets, configs)


def _exact_monomial(i, j):
    # integral over T0 of u^i v^j
    return factorial(i) * factorial(j) / factorial(i + j + 2)


def test_dunavant6_exact_to_degree6():
    r = dunavant6()
    assert r.shape == (12, 3)
    assert abs(r[:, 2].sum() - 0.5) < 1e-16
    worst = 0.0
    for i in range(7):
        for j in range(7 - i):
            q = np.sum(r[:, 2] * r[:, 0] ** i * r[:, 1] ** j)
            worst = max(worst, abs(q - _exact_monomial(i, j)) / _exact_monomial(i, j))
    assert worst < 1e-14
    # and genuinely degree 6: some degree-7 monomial is not integrated exactly
    errs = [abs(np.sum(r[:, 2] * r[:, 0] ** i * r[:, 1] ** (7 - i)) - _exact_monomial(i, 7 - i))
            for i in range(8)]
    assert max(errs) > 1e-7
    # nodes strictly inside T0, all weights positive
    assert np.all(r[:, :2] > 0) and np.all(r[:, 0] + r[:, 1] < 1) and np.all(r[:, 2] > 0)


def test_chart_nodes_unisolvent():
    golden = dict(l.split(None, 1) for l in open(
        __file__.replace("test_inputs.py", "golden/paper_constants.txt")) if l.strip() and l[0] != "#")
    uv = chart_nodes_45()
    assert len(uv) == int(golden["chart_nodes_order8"]) == 45
    assert np.all(uv > 0) and np.all(uv.sum(1) < 1)
    # Vandermonde on the monomials of total degree <= 8 has full rank
    V = np.stack([uv[:, 0] ** i * uv[:, 1] ** j for i in range(9) for j in range(9 - i)], 1)
    assert np.linalg.matrix_rank(V) == 45
    for p in (1, 2, 4, 8):
        assert len(chart_nodes(p)) == (p + 1) * (p + 2) // 2


@pytest.mark.parametrize("n", [1, 3, 16])
def test_cube_closed_volume(n):
    v, t = cube_mesh(n)
    assert len(t) == 12 * n * n
    closed, vol = mesh_check(v, t)
    assert closed and abs(vol - 1.0) < 1e-14


@pytest.mark.parametrize("nu", [1, 2, 5, 9])
def test_geodesic_counts_closed(nu):
    v, t = geodesic_sphere(nu)
    assert len(t) == 20 * nu * nu and len(v) == 10 * nu * nu + 2
    closed, vol = mesh_check(v, t)
    assert closed and 0 < vol < 4 * np.pi / 3
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)


def test_icosphere_level5():
    v, t = icosphere(5)
    assert len(t) == 20480
    closed, vol = mesh_check(v, t)
    assert closed and abs(vol - 4 * np.pi / 3) < 5e-3


def test_star_and_bumpy_surfaces():
    v, t = star_surface(8, seed=3)
    assert mesh_check(v, t)[0]
    v, t = bumpy_sphere(24, grade=10.0, lmax=16, nbumps=50, seed=1)
    closed, vol = mesh_check(v, t)
    assert closed and vol > 0
    D = triangle_diameters(v, t)
    assert D.max() / D.min() > 50        # graded ~ grade^2
    # every triangle faces outward (star-shaped about the origin)
    p0, p1, p2 = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    assert np.all(np.einsum("ij,ij->i", n, p0 + p1 + p2) > 0)


def test_triangle_diameters():
    v = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0],   # equilateral
                  [0, 0, 1], [3, 0, 1], [0, 4, 1],                   # right: hypotenuse 5
                  [0, 0, 2], [4, 0, 2], [2, 0.5, 2]], float)         # obtuse: longest edge
    t = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    D = triangle_diameters(v, t)
    assert abs(D[0] - 2 / np.sqrt(3)) < 1e-14
    assert abs(D[1] - 5.0) < 1e-14
    assert abs(D[2] - 4.0) < 1e-14


def test_refine_1to4_keeps_closed():
    v, t = refine_1to4(*cube_mesh(2))
    assert len(t) == 4 * 48
    closed, vol = mesh_check(v, t)
    assert closed and abs(vol - 1) < 1e-14


def test_targets_seeded():
    a = box_targets(100, seed=0)
    assert np.array_equal(a, box_targets(100, seed=0))
    assert a.min() >= -0.5 and a.max() <= 1.5
    s = shell_targets(1000, seed=2)
    r = np.linalg.norm(s, axis=1)
    assert r.min() >= 0.5 and r.max() <= 1.5
    v, t = icosphere(2)
    sig = np.full(len(t), 0.05)
    x = surface_offset_targets(v, t, sig, 5000, seed=1, chunk=1000)
    assert x.shape == (5000, 3)
    assert np.abs(np.linalg.norm(x, axis=1) - 1).max() < 0.2


def test_config1_shape():
    c = configs.config1()
    assert len(c["tris"]) == 3072 and len(c["targets"]) == 4096
    assert len(c["tris"]) * len(c["rule"]) == 36864


def test_batch_concat():
    m = [dict(verts=v, tris=t, sigma=np.array([0.1]), targets=box_targets(5, seed=i))
         for i, (v, t) in enumerate([cube_mesh(1), cube_mesh(2)])]
    b = configs.concat_batch(m)
    assert list(b["tri_offsets"]) == [0, 12, 60]
    assert b["tris"].max() == len(b["verts"]) - 1
    assert list(np.bincount(b["target_mesh"])) == [5, 5]


def test_torus_and_quadratic_generators():
    from workloads import torus_mesh, quadratic_from_flat, mesh_check
    v, t = torus_mesh(24, 12, R=1.0, r=0.4)
    closed, vol = mesh_check(v, t)
    assert closed and 0.9 * 2 * np.pi ** 2 * 0.16 < vol < 2 * np.pi ** 2 * 0.16
    v6, t6 = torus_mesh(24, 12, R=1.0, r=0.4, quadratic=True)
    assert t6.shape == (len(t), 6) and len(np.unique(t6)) == len(v6)
    assert np.abs(np.hypot(np.hypot(v6[:, 0], v6[:, 1]) - 1.0, v6[:, 2]) - 0.4).max() < 1e-14
    closed, _ = mesh_check(v6, np.ascontiguousarray(t6[:, :3]))
    assert closed
    # every edge point is shared by the two triangles of its edge
    e = np.concatenate([t6[:, [0, 1, 3]], t6[:, [1, 2, 4]], t6[:, [2, 0, 5]]])
    key = {}
    for a, b, m in e:
        key.setdefault((min(a, b), max(a, b)), set()).add(m)
    assert all(len(s) == 1 for s in key.values())
    vs, ts = icosphere(1)
    vq, tq = quadratic_from_flat(vs, ts, lift=lambda p: p / np.linalg.norm(p, axis=1, keepdims=True))
    assert np.allclose(np.linalg.norm(vq, axis=1), 1.0) and np.array_equal(tq[:, :3], ts)


def test_graded_torus_config3():
    """The C3 skeleton: a closed, consistently outward torus (Euler
    characteristic 0), enclosing about the plain torus's 2 pi^2 R r^2 (the
    bumps add and remove little), about 2e5 triangles, triangle diameters
    graded over at least 90x, no sliver (every angle > 20 degrees); seeded."""
    c = configs.config3()
    v, t = c["verts"], c["tris"]
    closed, vol = mesh_check(v, t)
    assert closed
    assert abs(vol - 2 * np.pi ** 2 * 0.09) < 0.01
    edges = {tuple(sorted(e)) for tri in t.tolist() for e in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0]))}
    assert len(v) - len(edges) + len(t) == 0
    assert 1.8e5 <= len(t) <= 2.6e5
    D = triangle_diameters(v, t)
    assert D.max() / D.min() >= 90
    assert np.allclose(c["sigma"], 0.5 * D) and c["chart_uv"].shape == (45, 2)
    p = v[t]
    ang = []
    for k in range(3):
        a, b = p[:, (k + 1) % 3] - p[:, k], p[:, (k + 2) % 3] - p[:, k]
        ang.append(np.degrees(np.arccos(np.clip((a * b).sum(1) / np.linalg.norm(a, axis=1)
                                                / np.linalg.norm(b, axis=1), -1, 1))))
    assert np.min(ang) > 20.0
    c2 = configs.config3()
    assert np.array_equal(c2["verts"], v) and np.array_equal(c2["tris"], t)
