"""Surface forests: quadtrees on bilinear tree patches (a 2D forest placed in
3D space by one bilinear map per tree), with per-leaf corner values of the
surface's transparency A_s and intensity I_s, and the Mandelbrot-set data of
the paper's first example (Sec. 4.1).

Leaves are stored as octree leaves with z = 0 (level, x, y anchors in units of
2^-19 of the tree's parameter square), in Morton order within each tree.
geom_params holds 12 doubles per tree, its corners P00, P10, P01, P11 (corner q
at parameter (q & 1, q >> 1)).  Nothing here intersects rays or evaluates the
surface model.
"""

from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .scene import QMAX, Camera, Fields, Forest, _sorted_forest, perspective_camera

# The hexagon of Sec. 4.1: top corners (-23/10, 3/4), (-1/4, 9/5), (13/10, 1)
# in the z = 0 plane, the bottom ones mirrored in y; cut along x = -1/4 into a
# left and a right quadrilateral, one tree each.  The left tree's t1 = 1 edge
# is the right tree's t1 = 0 edge.
HEX_TOP = ((-2.3, 0.75), (-0.25, 1.8), (1.3, 1.0))


def hexagon_corners(z=(0.0, 0.0, 0.0, 0.0, 0.0, 0.0)) -> np.ndarray:
    """[2, 4, 3] tree corners; z: heights of the six hexagon corners (bottom-left,
    bottom-middle, bottom-right, top-left, top-middle, top-right), 0 for the plane."""
    (xl, yl), (xm, ym), (xr, yr) = HEX_TOP
    bl, bm, br = (xl, -yl, z[0]), (xm, -ym, z[1]), (xr, -yr, z[2])
    tl, tm, tr = (xl, yl, z[3]), (xm, ym, z[4]), (xr, yr, z[5])
    return np.array([[bl, bm, tl, tm], [bm, br, tm, tr]], np.float64)


def patch_point(corners: np.ndarray, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """Bilinear map of one tree's 4 corners at parameters (t1, t2): [..., 3]."""
    c = np.asarray(corners, np.float64)
    t1 = np.asarray(t1, np.float64)[..., None]
    t2 = np.asarray(t2, np.float64)[..., None]
    return (c[0] * (1 - t1) * (1 - t2) + c[1] * t1 * (1 - t2) + c[2] * (1 - t1) * t2 + c[3] * t1 * t2)


def surface_forest(corners: np.ndarray, level, x, y, tree) -> Forest:
    corners = np.asarray(corners, np.float64).reshape(-1, 4, 3)
    nt = corners.shape[0]
    return _sorted_forest(level, x, y, np.zeros(len(level), np.uint32), np.asarray(tree, np.int64), "surface",
                          corners.ravel().copy(), nt)


def _children(level, x, y, tree):
    h = (np.uint32(1) << (np.uint32(QMAX) - level.astype(np.uint32) - np.uint32(1))).astype(np.uint32)
    lv = np.repeat(level + 1, 4).astype(np.uint8)
    cx = np.repeat(x, 4) + np.tile(np.array([0, 1, 0, 1], np.uint32), len(x)) * np.repeat(h, 4)
    cy = np.repeat(y, 4) + np.tile(np.array([0, 0, 1, 1], np.uint32), len(y)) * np.repeat(h, 4)
    return lv, cx.astype(np.uint32), cy.astype(np.uint32), np.repeat(tree, 4)


def uniform_quadtrees(ntrees: int, level: int):
    n = 1 << level
    g = np.arange(n, dtype=np.uint32) << np.uint32(QMAX - level)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    lv = np.full(ntrees * n * n, level, np.uint8)
    return lv, np.tile(xx.ravel(), ntrees), np.tile(yy.ravel(), ntrees), np.repeat(np.arange(ntrees), n * n)


def leaf_corner_params(level, x, y):
    """Parameters (t1, t2) of each leaf's 4 corners: two [4, N] arrays."""
    s = 1.0 / (1 << QMAX)
    h = np.ldexp(1.0, -level.astype(np.int64))
    x0, y0 = x.astype(np.float64) * s, y.astype(np.float64) * s
    t1 = np.stack([x0, x0 + h, x0, x0 + h])
    t2 = np.stack([y0, y0, y0 + h, y0 + h])
    return t1, t2


def leaf_corner_points(forest: Forest) -> np.ndarray:
    """World positions of every leaf's 4 corners: [4, N, 3]."""
    corners = forest.geom_params.reshape(-1, 4, 3)
    t1, t2 = leaf_corner_params(forest.level, forest.x, forest.y)
    tree = forest.tree_of_leaf()
    out = np.empty((4, forest.nleaves, 3))
    for k in range(forest.ntrees):
        m = tree == k
        out[:, m] = patch_point(corners[k], t1[:, m], t2[:, m])
    return out


def random_quadtree_forest(rng, corners, lmin=1, lmax=4, p_split=0.5) -> Forest:
    """Quadtrees refined at random from level lmin to lmax."""
    corners = np.asarray(corners, np.float64).reshape(-1, 4, 3)
    lv, x, y, tr = uniform_quadtrees(corners.shape[0], lmin)
    done = [], [], [], []
    for _ in range(lmin, lmax):
        split = rng.random(len(lv)) < p_split
        for acc, a in zip(done, (lv, x, y, tr)):
            acc.append(a[~split])
        lv, x, y, tr = _children(lv[split], x[split], y[split], tr[split])
    for acc, a in zip(done, (lv, x, y, tr)):
        acc.append(a)
    return surface_forest(corners, *(np.concatenate(a) for a in done))


def mandelbrot_count(c: np.ndarray, maxiter: int = 30) -> np.ndarray:
    """Iterations of z <- z^2 + c from z = 0 before |z| > 2 (at most maxiter), over maxiter."""
    c = np.asarray(c, np.complex128)
    z = np.zeros_like(c)
    n = np.zeros(c.shape, np.int32)
    alive = np.ones(c.shape, bool)
    for _ in range(maxiter):
        z[alive] = z[alive] * z[alive] + c[alive]
        esc = alive & (np.abs(z) > 2.0)
        alive &= ~esc
        n[alive] += 1
    return n.astype(np.float64) / maxiter


def _corner_counts(corners, lv, x, y, tr, maxiter):
    t1, t2 = leaf_corner_params(lv, x, y)
    val = np.empty(t1.shape)
    for k in range(corners.shape[0]):
        m = tr == k
        p = patch_point(corners[k], t1[:, m], t2[:, m])
        val[:, m] = mandelbrot_count(p[..., 0] + 1j * p[..., 1], maxiter)
    return val


def mandelbrot_forest(lmin=4, lmax=11, maxiter=30, corners=None):
    """Two quadtrees on the hexagon, uniform at lmin, then every leaf whose four corner
    values (the Mandelbrot iteration count at the corner's (x, y), over maxiter) are not
    all equal is split, up to lmax.  Returns the forest and its corner values [4, N]."""
    corners = hexagon_corners() if corners is None else np.asarray(corners, np.float64).reshape(-1, 4, 3)
    lv, x, y, tr = uniform_quadtrees(corners.shape[0], lmin)
    done = [], [], [], []
    for level in range(lmin, lmax + 1):
        val = _corner_counts(corners, lv, x, y, tr, maxiter)
        split = (val.min(0) != val.max(0)) if level < lmax else np.zeros(len(lv), bool)
        for acc, a in zip(done, (lv, x, y, tr)):
            acc.append(a[~split])
        if not split.any():
            break
        lv, x, y, tr = _children(lv[split], x[split], y[split], tr[split])
    f = surface_forest(corners, *(np.concatenate(a) for a in done))
    return f, _corner_counts(corners, f.level, f.x, f.y, f.tree_of_leaf(), maxiter)


def mandelbrot_fields(values: np.ndarray, instance: int = 0) -> Fields:
    """Transfer functions of the two image instances of Sec. 4.1, as corner values:
    0: opaque, intensity from grey (0.5) to white (1); 1: transparent, highlighting
    iteration counts just below the maximum."""
    s = np.asarray(values, np.float64)
    if instance == 0:
        As = np.zeros_like(s)
        Is = 0.5 + 0.5 * s
    else:
        w = np.exp(-((s - 29.0 / 30.0) / 0.05) ** 2)
        As = 0.85 - 0.6 * w
        Is = 0.1 + 0.9 * w
    return Fields("surface", As.astype(np.float32), Is.astype(np.float32))


def random_surface_fields(rng, n: int, opaque_frac=0.2) -> Fields:
    As = rng.uniform(0.0, 1.0, (4, n))
    As[:, rng.random(n) < opaque_frac] = 0.0
    return Fields("surface", As.astype(np.float32), rng.uniform(0.0, 1.0, (4, n)).astype(np.float32))


def hexagon_cameras(w=1024, h=1024, background=0.2) -> List[Camera]:
    """The two instances: the hexagon seen from above at two angles."""
    c = np.array([-0.5, 0.0, 0.0])
    eye0 = c + 4.2 * np.array([0.25, -0.45, 0.86])
    eye1 = c + 3.8 * np.array([-0.55, 0.35, 0.76])
    return [perspective_camera(eye0, c, [0.0, 0.0, 1.0], 1.0, 60.0, w, h, 10.0, background),
            perspective_camera(eye1, c, [0.0, 0.0, 1.0], 1.0, 60.0, w, h, 10.0, background)]


# ----------------------------------------------------------------------------
# degree-R trees (eq. nodal, eq. tensorgeom)
# ----------------------------------------------------------------------------


def gl_nodes(R: int) -> np.ndarray:
    """Gauss-Lobatto nodes on [0, 1] for degree R (2 or 3)."""
    if R == 2:
        return np.array([0.0, 0.5, 1.0])
    if R == 3:
        a = 0.5 / math.sqrt(5.0)
        return np.array([0.0, 0.5 - a, 0.5 + a, 1.0])
    raise ValueError("degree 2 or 3")


def ho_tree(fn, R: int) -> np.ndarray:
    """Control points z_{m1, m2} = fn(eta_m1, eta_m2) of one tree: [(R+1)^2, 3], m1 fastest."""
    eta = gl_nodes(R)
    t2, t1 = np.meshgrid(eta, eta, indexing="ij")
    return np.asarray(fn(t1.ravel(), t2.ravel()), np.float64).reshape(-1, 3)


def ho_geom(trees, R: int) -> np.ndarray:
    """geom_params of a degree-R surface forest: [R, control points of every tree]."""
    return np.concatenate([[float(R)]] + [np.asarray(t, np.float64).ravel() for t in trees])


def ho_hexagon_trees(R: int, height=None):
    """The hexagon's two trees with the surface lifted to z = height(x, y) (None: flat),
    interpolated at the Gauss-Lobatto grid of degree R."""
    corners = hexagon_corners()
    trees = []
    for k in range(2):
        def fn(t1, t2, k=k):
            p = patch_point(corners[k], t1, t2)
            if height is not None:
                p[:, 2] = height(p[:, 0], p[:, 1])
            return p
        trees.append(ho_tree(fn, R))
    return trees


def ho_surface_forest(trees, R: int, level, x, y, tree) -> Forest:
    nt = len(trees)
    f = _sorted_forest(level, x, y, np.zeros(len(level), np.uint32), np.asarray(tree, np.int64), "surface_ho",
                       ho_geom(trees, R), nt)
    return f


def ho_random_forest(rng, trees, R: int, lmin=1, lmax=4, p_split=0.5) -> Forest:
    """Quadtrees refined at random on degree-R trees."""
    lv, x, y, tr = uniform_quadtrees(len(trees), lmin)
    done = [], [], [], []
    for _ in range(lmin, lmax):
        split = rng.random(len(lv)) < p_split
        for acc, a in zip(done, (lv, x, y, tr)):
            acc.append(a[~split])
        lv, x, y, tr = _children(lv[split], x[split], y[split], tr[split])
    for acc, a in zip(done, (lv, x, y, tr)):
        acc.append(a)
    return ho_surface_forest(trees, R, *(np.concatenate(a) for a in done))
