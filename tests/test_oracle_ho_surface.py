"""Pins of the oracle's degree-R surfaces (eq. nodal, eq. tensorgeom: tensor
Lagrange maps on Gauss-Lobatto nodes; App. A.1: ray against a tensor-product
surface; Sec. 2.8 surface model).

Checked against: the nodal and partition-of-unity properties and polynomial
reproduction; the bilinear oracle on a degree-elevated flat hexagon; the
paraboloid z = c (t1^2 + t2^2) as a quadratic in the ray parameter (two hits);
a cubic graph seen from above (depth and angle law in closed form);
watertightness of a curved hexagon by a point-in-polygon test; and the rule for
a root on a leaf edge (the leaf whose half-open extent holds the root rounded to
the 2^-40 grid).
"""

import math

import numpy as np
import pytest

import synth
from synth.scene import Camera
from test_oracle_surface import _in_polygon, _ortho, _pixel_rays


def _forest_one_tree(fn, R, level=3):
    lv, x, y, tr = synth.surface.uniform_quadtrees(1, level)
    return synth.ho_surface_forest([synth.ho_tree(fn, R)], R, lv, x, y, tr)


@pytest.mark.parametrize("R", [2, 3])
def test_nodality_unity_and_reproduction(oracle_mod, R):
    rng = np.random.default_rng(R)
    eta = synth.gl_nodes(R)
    z = rng.normal(size=((R + 1) ** 2, 3))
    geom = synth.ho_geom([z], R)
    t2, t1 = np.meshgrid(eta, eta, indexing="ij")
    got = oracle_mod.ho_map(geom, 0, np.stack([t1.ravel(), t2.ravel()], 1))
    np.testing.assert_allclose(got, z, atol=1e-14)  # eq. nodal
    const = synth.ho_geom([np.tile([0.3, -1.2, 2.5], ((R + 1) ** 2, 1))], R)
    t = rng.uniform(-0.5, 1.5, (50, 2))
    np.testing.assert_allclose(oracle_mod.ho_map(const, 0, t), np.tile([0.3, -1.2, 2.5], (50, 1)), rtol=1e-13)

    def poly(a, b):
        return np.stack([a ** R - b, a * b ** (R - 1), (a * b) ** R + 0.5], -1)

    g = synth.ho_geom([synth.ho_tree(poly, R)], R)
    np.testing.assert_allclose(oracle_mod.ho_map(g, 0, t), poly(t[:, 0], t[:, 1]), rtol=1e-12, atol=1e-13)


def test_degree_two_flat_hexagon_equals_the_bilinear_oracle(oracle_mod):
    rng = np.random.default_rng(71)
    bil = synth.random_quadtree_forest(rng, synth.hexagon_corners(), 2, 5, 0.5)
    ho = synth.ho_surface_forest(synth.ho_hexagon_trees(2), 2, bil.level, bil.x, bil.y, bil.tree_of_leaf())
    assert np.array_equal(ho.x, bil.x) and np.array_equal(ho.level, bil.level)
    fl = synth.random_surface_fields(rng, bil.nleaves)
    cam = synth.hexagon_cameras(72, 60, background=0.3)[1]
    a = oracle_mod.surface_render(bil, fl, cam, hits=True)
    b = oracle_mod.ho_surface_render(ho, fl, cam, hits=True)
    # away from leaf edges the same leaf, depth and value
    rho, r = _pixel_rays(cam)
    s = -rho[:, 2] / r[:, 2]
    pt = rho + s[:, None] * r
    from test_oracle_surface import _invert_bilinear
    safe = np.zeros(len(s), bool)
    for k in range(2):
        t = _invert_bilinear(synth.hexagon_corners()[k], pt)
        inside = (t >= 0).all(1) & (t <= 1).all(1)
        frac = (t * 32) % 1.0
        safe |= inside & (frac > 1e-6).all(1) & (frac < 1 - 1e-6).all(1)
    assert safe.sum() > 1000
    np.testing.assert_array_equal(a["hit_leaf"][safe, 0], b["hit_leaf"][safe, 0])
    np.testing.assert_allclose(b["hit_s"][safe, 0], a["hit_s"][safe, 0], rtol=1e-12)
    for k in ("A", "B", "I"):
        np.testing.assert_allclose(b[k][safe], a[k][safe], rtol=1e-10, atol=1e-14)


def test_paraboloid_hits_as_a_quadratic(oracle_mod):
    c = 0.8

    def fn(a, b):
        return np.stack([a, b, c * (a * a + b * b)], -1)

    f = _forest_one_tree(fn, 2, level=2)
    fl = synth.Fields("surface", np.full((4, f.nleaves), 0.5, np.float32), np.full((4, f.nleaves), 0.5, np.float32))
    rng = np.random.default_rng(72)
    ntwo = 0
    for trial in range(4):
        d = rng.normal(size=3)
        d[2] = -abs(d[2]) * 0.4
        cam = _ortho(d, [0, 0, 1], [0.5, 0.5, 0.6], 40, 32, 1.3 / 40, zfar=6.0)
        out = oracle_mod.ho_surface_render(f, fl, cam, hits=True)
        rho, r = _pixel_rays(cam)
        for p in range(rho.shape[0]):
            (ox, oy, oz), (rx, ry, rz) = rho[p], r[p]
            qa = c * (rx * rx + ry * ry)
            qb = 2 * c * (ox * rx + oy * ry) - rz
            qc = c * (ox * ox + oy * oy) - oz
            disc = qb * qb - 4 * qa * qc
            if abs(disc) < 1e-6:
                continue  # nearly tangent
            roots = [] if disc < 0 else sorted(np.roots([qa, qb, qc]).real)
            tt = [(ox + sv * rx, oy + sv * ry) for sv in roots]
            if any(min(abs(a), abs(a - 1), abs(b), abs(b - 1)) < 1e-7 for a, b in tt):
                continue  # on the patch border
            exp = [sv for sv, (a, b) in zip(roots, tt) if 0 <= a <= 1 and 0 <= b <= 1 and 1.0 <= sv <= 6.0]
            got = [sv for sv, lf in zip(out["hit_s"][p], out["hit_leaf"][p]) if lf >= 0]
            assert len(got) == len(exp), (trial, p, got, exp)
            np.testing.assert_allclose(got, exp, rtol=1e-10)
            ntwo += len(exp) == 2
    assert ntwo > 10


def test_cubic_graph_from_above(oracle_mod):
    """z = f(t1, t2) of degree 3, vertical rays: depth oz - f, and A = A_s^sqrt(1 + |grad f|^2)."""

    def f3(a, b):
        return a ** 3 - 2 * a * b * b + 0.5 * b ** 3

    f = _forest_one_tree(lambda a, b: np.stack([a, b, f3(a, b)], -1), 3, level=3)
    As, Is = 0.6, 0.7
    fl = synth.Fields("surface", np.full((4, f.nleaves), As, np.float32), np.full((4, f.nleaves), Is, np.float32))
    cam = _ortho([0, 0, -1], [0, 1, 0], [0.5, 0.5, 0.0], 30, 30, 0.9 / 30, dist=3.0, zfar=6.0)
    out = oracle_mod.ho_surface_render(f, fl, cam, hits=True)
    rho, _ = _pixel_rays(cam)
    a, b = rho[:, 0], rho[:, 1]
    np.testing.assert_allclose(out["hit_s"][:, 0], rho[:, 2] - f3(a, b), rtol=1e-12)
    fx = 3 * a * a - 2 * b * b
    fy = -4 * a * b + 1.5 * b * b
    A = float(np.float32(As)) ** np.sqrt(1 + fx * fx + fy * fy)
    np.testing.assert_allclose(out["A"], A, rtol=1e-11)
    np.testing.assert_allclose(out["B"], float(np.float32(Is)) * (1 - A), rtol=1e-11)


def test_curved_hexagon_is_watertight(oracle_mod):
    """Degree 3 lifted hexagon seen from above: x and y stay the bilinear map, so every
    vertical ray inside the hexagon meets exactly one leaf."""
    trees = synth.ho_hexagon_trees(3, lambda x, y: 0.3 * np.sin(2 * x) * np.cos(y))
    f = synth.ho_random_forest(np.random.default_rng(73), trees, 3, 2, 5, 0.45)
    fl = synth.random_surface_fields(np.random.default_rng(74), f.nleaves)
    cam = _ortho([0, 0, -1], [0, 1, 0], [-0.5 + 1e-3 / 3, 0.0, 0.0], 90, 80, 3.9 / 90, dist=3.0, zfar=6.0)
    out = oracle_mod.ho_surface_render(f, fl, cam, hits=True)
    rho, _ = _pixel_rays(cam)
    (xl, yl), (xm, ym), (xr, yr) = synth.surface.HEX_TOP
    hexagon = np.array([(xl, -yl), (xm, -ym), (xr, -yr), (xr, yr), (xm, ym), (xl, yl)])
    inside = _in_polygon(rho[:, :2], hexagon)
    nh = (out["hit_leaf"] >= 0).sum(1)
    assert np.all(nh[inside] == 1) and np.all(nh[~inside] == 0)
    assert inside.sum() > 2000


@pytest.mark.parametrize("R", [2, 3])
def test_edge_rays_go_to_the_leaf_starting_there(oracle_mod, R):
    """A graph x = (t1, t2, f) seen from above: the hit of a vertical ray through (x, y) has parameters (x, y), so
    a ray through a leaf edge or corner must hit exactly one leaf, the one whose half-open extent holds (x, y)
    rounded to the 2^-40 grid: the leaf starting at the edge for offsets within half a grid step (1e-14), the
    geometric one beyond it (1e-12)."""
    f = _forest_one_tree(lambda a, b: np.stack([a, b, 0.2 * a * a - 0.15 * a * b + 0.1 * b], -1), R, level=3)
    fl = synth.random_surface_fields(np.random.default_rng(90 + R), f.nleaves)
    x0 = f.x.astype(np.float64) / (1 << synth.QMAX)
    y0 = f.y.astype(np.float64) / (1 << synth.QMAX)
    g = 2.0 ** 40

    def leaf_at(u, v):
        u, v = round(u * g) / g, round(v * g) / g
        hit = np.nonzero((x0 <= u) & (u < x0 + 0.125) & (y0 <= v) & (v < y0 + 0.125))[0]
        assert len(hit) == 1
        return int(hit[0])

    cases = 0
    for e, t in ((0.5, 0.3), (0.25, 0.875), (0.625, 0.0625)):
        for d in (0.0, 1e-14, -1e-14, 1e-12, -1e-12):
            for u, v in ((e + d, t), (t, e + d), (e + d, e + d)):
                cam = _ortho([0, 0, -1], [0, 1, 0], [u, v, 0.0], 1, 1, 1e-3, dist=3.0, zfar=6.0)
                out = oracle_mod.ho_surface_render(f, fl, cam, hits=True)
                got = out["hit_leaf"][0][out["hit_leaf"][0] >= 0]
                assert len(got) == 1 and int(got[0]) == leaf_at(u, v), (u, v, got)
                cases += 1
    # the rounding decides: 1e-14 below an edge goes to the leaf starting there, 1e-12 below it does not
    assert leaf_at(0.5 - 1e-14, 0.3) == leaf_at(0.5, 0.3) != leaf_at(0.5 - 1e-12, 0.3)
    assert cases == 45
