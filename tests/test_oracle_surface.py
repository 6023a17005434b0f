"""Pins of the oracle's surface rendering (Sec. 2.8 surface model, eq. ABphi;
App. A.1 ray against a bilinear tree patch; Sec. 4.1 hexagon of two quadtrees).

Every check uses a construction of its own: an orthographic grid lookup on a
flat square, a numpy ray-plane intersection with a Newton inversion of the
bilinear map, the saddle z = t1 t2 solved as a quadratic in the ray parameter,
the angle law at known angles, point-in-polygon tests for watertightness, and
two stacked trees folded by hand.
"""

import math

import numpy as np
import pytest

import synth
from synth.scene import Camera

SQUARE = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64)


def _ortho(vh, u, center, w, h, ell, dist=2.0, zfar=4.0, background=0.0):
    vh = np.asarray(vh, np.float64) / np.linalg.norm(vh)
    u = np.asarray(u, np.float64)
    u = u - np.dot(u, vh) * vh
    u /= np.linalg.norm(u)
    t = np.cross(vh, u)
    return Camera(np.asarray(center, np.float64) - dist * vh, vh.copy(), t, u, float(ell), float(zfar), w, h, True,
                  float(background))


def _pixel_rays(cam):
    """Ray origin and direction of every pixel (row j = 0 first), by the camera definition."""
    i = np.arange(cam.w)[None, :].repeat(cam.h, 0).ravel()
    j = np.arange(cam.h)[:, None].repeat(cam.w, 1).ravel()
    a = cam.ell * (i - (cam.w - 1) / 2.0)
    b = cam.ell * (j - (cam.h - 1) / 2.0)
    off = a[:, None] * cam.t[None, :] + b[:, None] * cam.u[None, :]
    n = np.linalg.norm(cam.v)
    if cam.ortho:
        return cam.o[None, :] + off, np.repeat((cam.v / n)[None, :], len(i), 0)
    return np.repeat(cam.o[None, :], len(i), 0), cam.v[None, :] + off


def _const_fields(n, As, Is):
    return synth.Fields("surface", np.full((4, n), As, np.float32), np.full((4, n), Is, np.float32))


def test_flat_square_seen_orthographically(oracle_mod):
    """Opaque leaves of a uniform level-3 quadtree on the unit square: each pixel shows the
    intensity of the leaf under its centre, at depth 2 from the camera."""
    lv, x, y, tr = synth.surface.uniform_quadtrees(1, 3)
    f = synth.surface_forest(SQUARE, lv, x, y, tr)
    rng = np.random.default_rng(1)
    Is = rng.uniform(0.2, 1.0, f.nleaves)
    fl = synth.Fields("surface", np.zeros((4, f.nleaves), np.float32),
                      np.repeat(Is[None, :], 4, 0).astype(np.float32))
    cam = _ortho([0, 0, -1], [1, 0, 0], [0.5, 0.5, 0.0], 64, 64, 1.0 / 56, background=0.3)
    out = oracle_mod.surface_render(f, fl, cam, hits=True)
    rho, r = _pixel_rays(cam)
    p = rho + 2.0 * r
    inside = (p[:, 0] >= 0) & (p[:, 0] <= 1) & (p[:, 1] >= 0) & (p[:, 1] <= 1)
    cell = np.minimum((p[:, 0] * 8).astype(int), 7) + 8 * np.minimum((p[:, 1] * 8).astype(int), 7)
    key = synth.morton_keys(f.x, f.y, f.z)
    leaf_of_cell = np.array([np.searchsorted(key, synth.morton_keys(np.array([(c % 8) << 16], np.uint32),
                                                                      np.array([(c // 8) << 16], np.uint32),
                                                                      np.array([0], np.uint32))[0])
                             for c in range(64)])
    exp_I = np.where(inside, Is[leaf_of_cell[cell]].astype(np.float32), 0.3)
    np.testing.assert_allclose(out["I"], exp_I, rtol=1e-7)
    assert np.all(out["A"][inside] == 0.0) and np.all(out["A"][~inside] == 1.0)
    np.testing.assert_array_equal(out["hit_leaf"][:, 0], np.where(inside, leaf_of_cell[cell], -1))
    np.testing.assert_allclose(out["hit_s"][inside, 0], 2.0, rtol=1e-15)
    assert np.all(out["hit_leaf"][:, 1] == -1)


def _invert_bilinear(P, pt):
    """(t1, t2) with J(t1, t2) = pt (x, y only) by Newton from the centre."""
    t = np.full((pt.shape[0], 2), 0.5)
    a, b, c, d = P[0], P[1] - P[0], P[2] - P[0], P[3] - P[1] - P[2] + P[0]
    for _ in range(60):
        J = a + b * t[:, :1] + c * t[:, 1:] + d * (t[:, :1] * t[:, 1:])
        res = (J - pt)[:, :2]
        j1 = (b + d * t[:, 1:])[:, :2]
        j2 = (c + d * t[:, :1])[:, :2]
        det = j1[:, 0] * j2[:, 1] - j1[:, 1] * j2[:, 0]
        dt1 = (res[:, 0] * j2[:, 1] - res[:, 1] * j2[:, 0]) / det
        dt2 = (j1[:, 0] * res[:, 1] - j1[:, 1] * res[:, 0]) / det
        t[:, 0] -= dt1
        t[:, 1] -= dt2
    return t


def test_flat_hexagon_against_plane_intersection_and_inverse_map(oracle_mod):
    corners = synth.hexagon_corners()
    lv, x, y, tr = synth.surface.uniform_quadtrees(2, 3)
    f = synth.surface_forest(corners, lv, x, y, tr)
    fl = synth.random_surface_fields(np.random.default_rng(2), f.nleaves)
    cam = synth.hexagon_cameras(80, 60)[0]
    out = oracle_mod.surface_render(f, fl, cam, hits=True)
    rho, r = _pixel_rays(cam)
    s = -rho[:, 2] / r[:, 2]
    pt = rho + s[:, None] * r
    key = synth.morton_keys(f.x, f.y, f.z)
    checked = 0
    for k in range(2):
        t = _invert_bilinear(corners[k], pt)
        ok = (t >= 0).all(1) & (t <= 1).all(1)
        # keep away from leaf edges and the tree seam, where rounding may decide
        frac = (t * 8) % 1.0
        ok &= (frac > 1e-6).all(1) & (frac < 1 - 1e-6).all(1)
        for p in np.nonzero(ok)[0]:
            ci = (t[p] * 8).astype(int)
            kk = synth.morton_keys(np.array([ci[0] << 16], np.uint32), np.array([ci[1] << 16], np.uint32),
                                   np.array([0], np.uint32))[0]
            leaf = f.tree_begin[k] + np.searchsorted(key[f.tree_begin[k]:f.tree_begin[k + 1]], kk)
            assert out["hit_leaf"][p, 0] == leaf and out["hit_leaf"][p, 1] == -1
            assert math.isclose(out["hit_s"][p, 0], s[p], rel_tol=1e-12)
            checked += 1
    assert checked > 2000
    # pixels that see no tree see the background
    miss = out["hit_leaf"][:, 0] < 0
    assert miss.any() and np.all(out["I"][miss] == cam.background)


def test_saddle_patch_hits_as_a_quadratic_in_the_ray_parameter(oracle_mod):
    """J(t1, t2) = (t1, t2, t1 t2): along the ray, (rho_x + s r_x)(rho_y + s r_y) = rho_z + s r_z."""
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 1]], np.float64)
    f = synth.surface_forest(P, np.array([0], np.uint8), np.array([0], np.uint32), np.array([0], np.uint32), [0])
    fl = _const_fields(1, 0.5, 0.5)
    rng = np.random.default_rng(3)
    ntwo = 0
    for trial in range(6):
        d = rng.normal(size=3)
        d[2] = abs(d[2]) * 0.3
        cam = _ortho(d, [0, 0, 1] if abs(d[2]) < 0.9 else [1, 0, 0], [0.5, 0.5, 0.25], 48, 40, 1.0 / 30, zfar=6.0)
        out = oracle_mod.surface_render(f, fl, cam, hits=True)
        rho, r = _pixel_rays(cam)
        for p in range(rho.shape[0]):
            (ox, oy, oz), (rx, ry, rz) = rho[p], r[p]
            roots = np.roots([rx * ry, ox * ry + oy * rx - rz, ox * oy - oz])
            roots = np.sort([z.real for z in roots if abs(z.imag) < 1e-12])
            exp = [sv for sv in roots if 0 <= ox + sv * rx <= 1 and 0 <= oy + sv * ry <= 1 and
                   cam_clip(cam)[0] <= sv <= cam_clip(cam)[1]]
            got = [sv for sv, lf in zip(out["hit_s"][p], out["hit_leaf"][p]) if lf >= 0]
            # skip rays grazing the patch border, where rounding decides
            tt = [(ox + sv * rx, oy + sv * ry) for sv in roots]
            if any(min(abs(a), abs(a - 1), abs(b), abs(b - 1)) < 1e-9 for a, b in tt):
                continue
            assert len(got) == len(exp), (trial, p, got, exp)
            np.testing.assert_allclose(got, exp, rtol=1e-9, atol=1e-12)
            ntwo += len(exp) == 2
    assert ntwo > 20


def cam_clip(cam):
    n = np.linalg.norm(cam.v)
    return (n, cam.zfar) if cam.ortho else (1.0, cam.zfar / n)


@pytest.mark.parametrize("phi_deg", [0.0, 40.0, 70.0])
def test_angle_law(oracle_mod, phi_deg):
    """eq. ABphi: A = A_s^(1/cos phi), B = I_s (1 - A); opaque A_s = 0 gives (0, I_s)."""
    phi = math.radians(phi_deg)
    lv, x, y, tr = synth.surface.uniform_quadtrees(1, 2)
    f = synth.surface_forest(SQUARE, lv, x, y, tr)
    cam = _ortho([math.sin(phi), 0, -math.cos(phi)], [0, 1, 0], [0.5, 0.5, 0.0], 32, 32, 1.0 / 150)
    for As, Is in ((0.6, 0.8), (0.0, 0.7), (1.0, 0.9)):
        out = oracle_mod.surface_render(f, _const_fields(f.nleaves, As, Is), cam)
        A = float(np.float32(As)) ** (1.0 / math.cos(phi))
        np.testing.assert_allclose(out["A"], A, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(out["B"], float(np.float32(Is)) * (1 - A), rtol=1e-12, atol=1e-15)


def test_bilinear_corner_values_at_normal_incidence(oracle_mod):
    f = synth.surface_forest(SQUARE, np.array([0], np.uint8), np.array([0], np.uint32), np.array([0], np.uint32), [0])
    As = np.array([[0.9], [0.1], [0.5], [0.3]], np.float32)
    Is = np.array([[0.2], [0.6], [1.0], [0.4]], np.float32)
    cam = _ortho([0, 0, -1], [0, 1, 0], [0.5, 0.5, 0.0], 20, 20, 1.0 / 24)
    out = oracle_mod.surface_render(f, synth.Fields("surface", As, Is), cam, hits=True)
    rho, r = _pixel_rays(cam)
    u, v = rho[:, 0], rho[:, 1]
    w = np.stack([(1 - u) * (1 - v), u * (1 - v), (1 - u) * v, u * v])
    a = (w * As.astype(np.float64)).sum(0)
    b = (w * Is.astype(np.float64)).sum(0) * (1 - a)
    np.testing.assert_allclose(out["A"], a, rtol=1e-12)
    np.testing.assert_allclose(out["B"], b, rtol=1e-12)


def _in_polygon(pts, poly):
    """Strictly inside a convex counter-clockwise polygon."""
    inside = np.ones(len(pts), bool)
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        cr = (b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0])
        inside &= cr > 0
    return inside


def test_hexagon_is_watertight(oracle_mod):
    """Every ray through the hexagon's interior meets exactly one leaf; rays outside none."""
    corners = synth.hexagon_corners()
    f = synth.random_quadtree_forest(np.random.default_rng(4), corners, 2, 6, 0.45)
    fl = _const_fields(f.nleaves, 0.5, 0.5)
    cam = _ortho([0, 0, -1], [0, 1, 0], [-0.5 + 1e-3 / 3, 0.0, 0.0], 150, 130, 3.9 / 150)
    out = oracle_mod.surface_render(f, fl, cam, hits=True)
    rho, _ = _pixel_rays(cam)
    (xl, yl), (xm, ym), (xr, yr) = synth.surface.HEX_TOP
    hexagon = np.array([(xl, -yl), (xm, -ym), (xr, -yr), (xr, yr), (xm, ym), (xl, yl)])
    inside = _in_polygon(rho[:, :2], hexagon)
    nh = (out["hit_leaf"] >= 0).sum(1)
    near_edge = np.zeros(len(nh), bool)
    for k in range(6):
        a, b = hexagon[k], hexagon[(k + 1) % 6]
        e = b - a
        dist = np.abs(e[0] * (rho[:, 1] - a[1]) - e[1] * (rho[:, 0] - a[0])) / np.linalg.norm(e)
        near_edge |= dist < 1e-9
    assert np.all(nh[inside & ~near_edge] == 1)
    assert np.all(nh[~inside & ~near_edge] == 0)
    assert inside.sum() > 5000


def test_two_stacked_trees_fold_nearest_first(oracle_mod):
    top = SQUARE + np.array([0, 0, 0.5])
    corners = np.stack([SQUARE, top])
    lv, x, y, tr = synth.surface.uniform_quadtrees(2, 1)
    f = synth.surface_forest(corners, lv, x, y, tr)
    As = np.where(f.tree_of_leaf() == 0, 0.3, 0.7)
    Is = np.where(f.tree_of_leaf() == 0, 0.9, 0.2)
    fl = synth.Fields("surface", np.repeat(As[None], 4, 0).astype(np.float32),
                      np.repeat(Is[None], 4, 0).astype(np.float32))
    cam = _ortho([0, 0, -1], [0, 1, 0], [0.5, 0.5, 0.0], 16, 16, 1.0 / 20, background=0.25)
    out = oracle_mod.surface_render(f, fl, cam, hits=True)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    a_top, b_top = f32(0.7), f32(0.2) * (1 - f32(0.7))
    a_bot, b_bot = f32(0.3), f32(0.9) * (1 - f32(0.3))
    np.testing.assert_allclose(out["A"], a_top * a_bot, rtol=1e-14)
    np.testing.assert_allclose(out["B"], b_top + a_top * b_bot, rtol=1e-14)
    np.testing.assert_allclose(out["hit_s"][:, 0], 1.5, rtol=1e-15)
    np.testing.assert_allclose(out["hit_s"][:, 1], 2.0, rtol=1e-15)
    assert np.all(f.tree_of_leaf()[out["hit_leaf"][:, 0]] == 1)


def test_mandelbrot_forest_tiles_both_trees():
    f, val = synth.mandelbrot_forest(3, 7)
    area = np.ldexp(1.0, -2 * f.level.astype(np.int64))
    tree = f.tree_of_leaf()
    for k in range(2):
        assert math.isclose(area[tree == k].sum(), 1.0, rel_tol=1e-12)
    keys = synth.morton_keys(f.x, f.y, f.z)
    for k in range(2):
        kk = keys[f.tree_begin[k]:f.tree_begin[k + 1]]
        assert np.all(np.diff(kk.astype(np.int64)) > 0)
    assert val.shape == (4, f.nleaves) and val.min() >= 0 and val.max() == 1.0
    # leaves above the finest level have equal corner values
    coarse = f.level < 7
    assert np.all(val[:, coarse].min(0) == val[:, coarse].max(0))
