"""Volume trees of degree R: each tree's reference cube is mapped to space by
a tensor product of degree-R Lagrange polynomials on the Gauss-Lobatto nodes
(eq. nodal, eq. tensorgeom).  A tree is given by its control points, the map's
values at the node triples; geom_params of a volume forest are
``[R, control points of every tree]``, (R+1)^3 points of 3 doubles per tree,
m1 fastest, then m2, then m3.  Data generation only."""

from __future__ import annotations

from typing import List

import numpy as np

from .scene import Camera, Fields, Forest, Scene, _sorted_forest, adaptive_forest, perspective_camera, \
    random_perspective_camera, straddle_refiner, trilinear_fields_from_gaussians, uniform_forest, QMAX
from .surface import gl_nodes


def vol_tree(fn, R: int) -> np.ndarray:
    """Control points fn(eta_m1, eta_m2, eta_m3) of one tree: [(R+1)^3, 3], m1 fastest."""
    eta = gl_nodes(R)
    t3, t2, t1 = np.meshgrid(eta, eta, eta, indexing="ij")
    return np.asarray(fn(t1.ravel(), t2.ravel(), t3.ravel()), np.float64).reshape(-1, 3)


def vol_geom(trees, R: int) -> np.ndarray:
    return np.concatenate([[float(R)]] + [np.asarray(t, np.float64).ravel() for t in trees])


def bent_map(c: float):
    """x = (t1, t2, t3 + c t1^2): a cube whose two faces normal to z are parabolic
    cylinders; degree 2 in t1, so a degree-2 tree reproduces it exactly."""
    def fn(t1, t2, t3):
        return np.stack([t1, t2, t3 + c * t1 * t1], -1)
    return fn


def random_quadratic_map(rng, amp: float):
    """x = t + amp * (a random combination of the monomials t_a^p t_b^q of degree
    at most 2 in every variable): a mildly curved degree-2 tree."""
    coef = rng.uniform(-1.0, 1.0, (3, 3, 3, 3))  # [axis][p1][p2][p3]
    coef[:, 0, 0, 0] = 0.0

    def fn(t1, t2, t3):
        out = np.stack([t1, t2, t3], -1).astype(np.float64)
        for k in range(3):
            acc = np.zeros_like(t1, dtype=np.float64)
            for p1 in range(3):
                for p2 in range(3):
                    for p3 in range(3):
                        if p1 + p2 + p3 > 2:
                            continue
                        acc += coef[k, p1, p2, p3] * t1 ** p1 * t2 ** p2 * t3 ** p3
            out[:, k] += amp * acc
        return out
    return fn


def volume_forest(trees, R: int, base: Forest) -> Forest:
    """The leaves of `base` (a one-tree cube forest, or tree-major leaves with
    tree_begin) on degree-R volume trees."""
    tree = base.tree_of_leaf().astype(np.int64)
    return _sorted_forest(base.level, base.x, base.y, base.z, tree, "volume", vol_geom(trees, R), len(trees))


def volume_scene(seed=0, R=2, lmin=1, lmax=4, ngauss=4, w=64, h=48, amp=0.06, ncams=1, background=0.0,
                 method="rk4") -> Scene:
    """A small adaptive forest on one mildly curved degree-R tree, trilinear fields
    from Gaussians in reference coordinates, perspective cameras."""
    rng = np.random.default_rng([1809, 1334, 5000 + seed])
    centers = rng.uniform(0.0, 1.0, (ngauss, 3))
    sigmas = rng.uniform(0.06, 0.2, ngauss)
    base = adaptive_forest(straddle_refiner(centers, sigmas), lmin, lmax)
    tree = vol_tree(random_quadratic_map(rng, amp), R)
    forest = volume_forest([tree], R, base)
    fields = trilinear_fields_from_gaussians(base, centers, sigmas)
    cams = [random_perspective_camera(rng, w, h, background=background) for _ in range(ncams)]
    return Scene(f"volume{seed}", forest, fields, cams, method, 4, {"centers": centers, "sigmas": sigmas})
