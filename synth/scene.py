"""Seeded generators for forests, fields and cameras.

Conventions shared by every consumer (they are data formats, not method
arithmetic):

* Leaf anchors are integers in units of ``2**-QMAX`` of the tree's reference
  cube; a leaf at level ``l`` spans ``2**(QMAX-l)`` units per axis.
* Leaves are sorted tree-major, then by the Morton (z-order) key of the anchor,
  with the x bit least significant in every bit triple.  Child and corner ids
  follow the same convention: ``c = bx + 2*by + 4*bz``.
* Fields are stored structure-of-arrays: ``kappa[corner][leaf]`` with one
  corner for per-leaf constants and eight corners for trilinear data.
* A camera is the paper's (o, v, t, u, ell, w, h) plus the far distance, an
  orthographic flag and the background intensity.  ``raw()`` packs it into
  the 20 doubles every interface takes.

Seeds follow ``numpy.random.default_rng([1809, 1334, k])`` for workload k.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

QMAX = 19  # deepest representable level; anchors fit in 19 bits per axis


# ----------------------------------------------------------------------------
# data holders
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Forest:
    level: np.ndarray  # uint8 [N]
    x: np.ndarray  # uint32 [N]
    y: np.ndarray  # uint32 [N]
    z: np.ndarray  # uint32 [N]
    tree_begin: np.ndarray  # int64 [ntrees + 1]
    geom: str = "unit_cube"  # or "shell6"
    geom_params: Optional[np.ndarray] = None  # float64, geometry-specific

    @property
    def nleaves(self) -> int:
        return int(self.level.shape[0])

    @property
    def ntrees(self) -> int:
        return int(self.tree_begin.shape[0] - 1)

    def tree_of_leaf(self) -> np.ndarray:
        t = np.zeros(self.nleaves, np.int32)
        for k in range(self.ntrees):
            t[self.tree_begin[k]:self.tree_begin[k + 1]] = k
        return t


@dataclasses.dataclass
class Fields:
    kind: str  # "const", "trilinear", "const_eq" (eps holds the equilibrium intensity I) or "surface"
    kappa: np.ndarray  # float32 [ncorner][N], or [nch][ncorner][N] for several channels
    eps: np.ndarray  # float32, as kappa

    @property
    def ncorner(self) -> int:
        return int(self.kappa.shape[-2])

    @property
    def nch(self) -> int:
        return 1 if self.kappa.ndim == 2 else int(self.kappa.shape[0])

    def channel(self, ch: int) -> "Fields":
        """Single-channel fields of channel ch."""
        if self.kappa.ndim == 2:
            assert ch == 0
            return self
        return Fields(self.kind, self.kappa[ch], self.eps[ch])


def stack_channels(fields: List["Fields"]) -> "Fields":
    """Several single-channel fields of one kind as the channels of one."""
    assert len({f.kind for f in fields}) == 1
    return Fields(fields[0].kind, np.stack([f.kappa for f in fields]), np.stack([f.eps for f in fields]))


@dataclasses.dataclass
class Camera:
    o: np.ndarray
    v: np.ndarray
    t: np.ndarray
    u: np.ndarray
    ell: float
    zfar: float
    w: int
    h: int
    ortho: bool = False
    background: float = 0.0

    def raw(self) -> np.ndarray:
        """The 20-double camera record: o, v, t, u, ell, zfar, w, h, ortho, I_b, 0, 0."""
        r = np.zeros(20, np.float64)
        r[0:3] = self.o
        r[3:6] = self.v
        r[6:9] = self.t
        r[9:12] = self.u
        r[12] = self.ell
        r[13] = self.zfar
        r[14] = self.w
        r[15] = self.h
        r[16] = 1.0 if self.ortho else 0.0
        r[17] = self.background
        return r

    @property
    def npix(self) -> int:
        return int(self.w) * int(self.h)


@dataclasses.dataclass
class Scene:
    name: str
    forest: Forest
    fields: Fields
    cameras: List[Camera]
    method: str  # "analytic" or "rk4"
    substeps: int = 4
    extra: dict = dataclasses.field(default_factory=dict)

    def cams_raw(self) -> np.ndarray:
        return np.stack([c.raw() for c in self.cameras]).astype(np.float64)


# ----------------------------------------------------------------------------
# forests
# ----------------------------------------------------------------------------


def morton_keys(x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Interleave anchor bits (x least significant) into a 57-bit key."""
    x = x.astype(np.uint64)
    y = y.astype(np.uint64)
    z = z.astype(np.uint64)
    key = np.zeros(x.shape, np.uint64)
    one = np.uint64(1)
    for b in range(QMAX):
        bb = np.uint64(b)
        key |= ((x >> bb) & one) << np.uint64(3 * b)
        key |= ((y >> bb) & one) << np.uint64(3 * b + 1)
        key |= ((z >> bb) & one) << np.uint64(3 * b + 2)
    return key


def _sorted_forest(level, x, y, z, tree=None, geom="unit_cube", geom_params=None, ntrees=1):
    level = np.asarray(level, np.uint8)
    x = np.asarray(x, np.uint32)
    y = np.asarray(y, np.uint32)
    z = np.asarray(z, np.uint32)
    if tree is None:
        tree = np.zeros(level.shape, np.int64)
    key = morton_keys(x, y, z)
    order = np.lexsort((key, tree))
    tree = tree[order]
    tb = np.searchsorted(tree, np.arange(ntrees + 1), side="left").astype(np.int64)
    return Forest(level[order], x[order], y[order], z[order], tb, geom, geom_params)


def uniform_forest(level: int) -> Forest:
    n = 1 << level
    g = np.arange(n, dtype=np.uint32) << np.uint32(QMAX - level)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    return _sorted_forest(np.full(n ** 3, level, np.uint8), xx.ravel(), yy.ravel(), zz.ravel())


def gaussian_sum(p: np.ndarray, centers: np.ndarray, sigmas: np.ndarray) -> np.ndarray:
    """Sum of unit-amplitude isotropic Gaussians at points p[..., 3]."""
    s = np.zeros(p.shape[:-1], np.float64)
    for c, sg in zip(centers, sigmas):
        d2 = ((p - c) ** 2).sum(-1)
        s += np.exp(-d2 / (2.0 * sg * sg))
    return s


def _lattice_offsets(m: int) -> np.ndarray:
    g = np.linspace(0.0, 1.0, m)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1)  # [m^3, 3]


def adaptive_forest(refine_fn, lmin: int, lmax: int, chunk: int = 1 << 15) -> Forest:
    """Refine uniformly to ``lmin``, then split a leaf while ``refine_fn`` says so.

    ``refine_fn(lo[n,3], h)`` receives leaf lower corners and the edge length
    (in the unit cube) and returns a bool mask of leaves to split.
    """
    n0 = 1 << lmin
    g = np.arange(n0, dtype=np.int64) << (QMAX - lmin)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    cur = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1)
    out_lv, out_xyz = [], []
    scale = 1.0 / (1 << QMAX)
    for lv in range(lmin, lmax + 1):
        if lv == lmax or cur.shape[0] == 0:
            out_lv.append(np.full(cur.shape[0], lv, np.uint8))
            out_xyz.append(cur)
            break
        h = 1.0 / (1 << lv)
        split = np.zeros(cur.shape[0], bool)
        for a in range(0, cur.shape[0], chunk):
            lo = cur[a:a + chunk].astype(np.float64) * scale
            split[a:a + chunk] = refine_fn(lo, h)
        out_lv.append(np.full(int((~split).sum()), lv, np.uint8))
        out_xyz.append(cur[~split])
        par = cur[split]
        half = 1 << (QMAX - lv - 1)
        kids = []
        for c in range(8):
            off = np.array([(c & 1) * half, ((c >> 1) & 1) * half, ((c >> 2) & 1) * half], np.int64)
            kids.append(par + off)
        cur = np.concatenate(kids, 0) if kids else np.zeros((0, 3), np.int64)
    lv = np.concatenate(out_lv)
    xyz = np.concatenate(out_xyz, 0)
    return _sorted_forest(lv, xyz[:, 0], xyz[:, 1], xyz[:, 2])


def straddle_refiner(centers, sigmas, thresh=0.2, lattice=3):
    offs = _lattice_offsets(lattice)

    def fn(lo, h):
        pts = lo[:, None, :] + h * offs[None, :, :]
        s = gaussian_sum(pts, centers, sigmas)
        return (s.min(1) < thresh) & (s.max(1) > thresh)

    return fn


# ----------------------------------------------------------------------------
# six-tree spherical shell (equiangular cubed sphere)
# ----------------------------------------------------------------------------

SHELL_R0, SHELL_R1 = 0.55, 1.0


def shell_frame(k: int):
    """(e1, e2, e3) of tree k: e3 = +-e_m (m = k // 2, sign + for even k), e1 = e_{m+1}, e2 = e_{m+2}."""
    m, sgn = k // 2, (1.0 if k % 2 == 0 else -1.0)
    e = np.eye(3)
    return e[(m + 1) % 3], e[(m + 2) % 3], sgn * e[m]


def shell_map(k: int, t: np.ndarray, r0=SHELL_R0, r1=SHELL_R1) -> np.ndarray:
    """Equiangular map of tree k: reference t[..., 3] in [0,1]^3 to real space."""
    e1, e2, e3 = shell_frame(k)
    a = np.tan(np.pi / 4 * (2 * t[..., 0] - 1))
    b = np.tan(np.pi / 4 * (2 * t[..., 1] - 1))
    r = r0 + (r1 - r0) * t[..., 2]
    d = a[..., None] * e1 + b[..., None] * e2 + e3
    return (r / np.sqrt(1 + a * a + b * b))[..., None] * d


def shell_params(level: int, r0=SHELL_R0, r1=SHELL_R1) -> np.ndarray:
    """Geometry table: r0, r1, table level L, then tan(pi/4 (2 i / 2^L - 1)) for i = 0 .. 2^L."""
    i = np.arange((1 << level) + 1, dtype=np.float64)
    tab = np.tan(np.pi / 4 * (2 * i / (1 << level) - 1))
    # exact values where they exist: tree boundaries must coincide between trees
    tab[0], tab[-1], tab[(1 << level) // 2] = -1.0, 1.0, 0.0
    return np.concatenate([[r0, r1, float(level)], tab])


def shell_forest(refine_fn, lmin: int, lmax: int, chunk: int = 1 << 15) -> Forest:
    """Six trees refined uniformly to lmin, then while refine_fn(points [n, P, 3]) says so."""
    levels, xs, ys, zs, trees = [], [], [], [], []
    offs = _lattice_offsets(3)
    scale = 1.0 / (1 << QMAX)
    for k in range(6):
        n0 = 1 << lmin
        g = np.arange(n0, dtype=np.int64) << (QMAX - lmin)
        zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
        cur = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], -1)
        for lv in range(lmin, lmax + 1):
            if lv == lmax or cur.shape[0] == 0:
                split = np.zeros(cur.shape[0], bool)
            else:
                h = 1.0 / (1 << lv)
                split = np.zeros(cur.shape[0], bool)
                for a in range(0, cur.shape[0], chunk):
                    lo = cur[a:a + chunk].astype(np.float64) * scale
                    pts = shell_map(k, lo[:, None, :] + h * offs[None, :, :])
                    split[a:a + chunk] = refine_fn(pts)
            keep = cur[~split]
            levels.append(np.full(keep.shape[0], lv, np.uint8))
            xs.append(keep[:, 0]); ys.append(keep[:, 1]); zs.append(keep[:, 2])
            trees.append(np.full(keep.shape[0], k, np.int64))
            if lv == lmax:
                break
            par = cur[split]
            half = 1 << (QMAX - lv - 1)
            kids = [par + np.array([(c & 1) * half, ((c >> 1) & 1) * half, ((c >> 2) & 1) * half], np.int64)
                    for c in range(8)]
            cur = np.concatenate(kids, 0)
    return _sorted_forest(np.concatenate(levels), np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
                          np.concatenate(trees), "shell6", shell_params(lmax), 6)


def shell_corner_points(forest: Forest) -> np.ndarray:
    """Real-space positions of the 8 reference corners of every leaf: [8, N, 3]."""
    scale = 1.0 / (1 << QMAX)
    lo = np.stack([forest.x, forest.y, forest.z], -1).astype(np.float64) * scale
    h = np.ldexp(1.0, -forest.level.astype(np.int64))
    tree = forest.tree_of_leaf()
    r0, r1 = forest.geom_params[0], forest.geom_params[1]
    pts = np.empty((8, forest.nleaves, 3))
    for c in range(8):
        t = lo + h[:, None] * np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1], np.float64)
        for k in range(6):
            sel = tree == k
            pts[c, sel] = shell_map(k, t[sel], r0, r1)
    return pts


def shell_centers(rng, k, r0=SHELL_R0, r1=SHELL_R1):
    d = rng.normal(size=(k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = (r0 ** 3 + rng.uniform(0, 1, k) * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
    return d * r[:, None]


def shell_scene(seed=0, lmin=1, lmax=3, ngauss=4, w=96, h=72, sigma=(0.09, 0.3), dist=3.0, background=0.0,
                rule="volume", name=None) -> "Scene":
    """Six-tree shell with trilinear fields (in reference coordinates) from Gaussians in the shell."""
    rng = np.random.default_rng([1809, 1334, 3] if seed is None else [1809, 1334, 3000 + seed])
    centers = shell_centers(rng, ngauss)
    sigmas = rng.uniform(sigma[0], sigma[1], ngauss)

    def refine(pts):
        s = gaussian_sum(pts, centers, sigmas)
        if rule == "volume":
            return s.max(1) > 0.2
        return (s.min(1) < 0.2) & (s.max(1) > 0.2)

    forest = shell_forest(refine, lmin, lmax)
    pts = shell_corner_points(forest)
    sc = np.stack([gaussian_sum(pts[c], centers, sigmas) for c in range(8)])
    fields = Fields("trilinear", (0.2 + 2.0 * sc).astype(np.float32), (0.1 + 1.0 * sc).astype(np.float32))
    cam = random_perspective_camera(rng, w, h, dist=dist, center=(0.0, 0.0, 0.0), background=background)
    return Scene(name or f"shell{seed}", forest, fields, [cam], "rk4", 4, {"centers": centers, "sigmas": sigmas})


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------


def corner_points(forest: Forest) -> np.ndarray:
    """Unit-cube positions of the 8 corners of every leaf: [8, N, 3]."""
    scale = 1.0 / (1 << QMAX)
    lo = np.stack([forest.x, forest.y, forest.z], -1).astype(np.float64) * scale
    h = np.ldexp(1.0, -forest.level.astype(np.int64))
    pts = np.empty((8, forest.nleaves, 3))
    for c in range(8):
        pts[c] = lo + h[:, None] * np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1], np.float64)
    return pts


def constant_fields(kappa: np.ndarray, eps: np.ndarray) -> Fields:
    return Fields("const", np.asarray(kappa, np.float32)[None, :].copy(),
                  np.asarray(eps, np.float32)[None, :].copy())


def constant_variant(scene: Scene) -> Scene:
    """The scene with each leaf's corner values replaced by their mean, so that
    every leaf holds constant coefficients and renders analytically: the same
    forest, cameras, visibility and pairing, with one (kappa, eps) per leaf."""
    f = scene.fields
    assert f.kind == "trilinear" and f.nch == 1
    fields = constant_fields(f.kappa.astype(np.float64).mean(axis=0), f.eps.astype(np.float64).mean(axis=0))
    return Scene(scene.name + "_const", scene.forest, fields, scene.cameras, "analytic", 1, dict(scene.extra))


def split_shares(forest: Forest, fields: Fields, cuts) -> List[tuple]:
    """One-tree forest cut into contiguous curve-order ranges at the leaf
    indices `cuts`: a list of (Forest, Fields), one per process share."""
    assert forest.ntrees == 1
    bounds = [0] + [int(c) for c in cuts] + [forest.nleaves]
    out = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        f = Forest(forest.level[a:b].copy(), forest.x[a:b].copy(), forest.y[a:b].copy(), forest.z[a:b].copy(),
                   np.array([0, b - a], np.int64), forest.geom, forest.geom_params)
        out.append((f, Fields(fields.kind, fields.kappa[:, a:b].copy(), fields.eps[:, a:b].copy())))
    return out


def equilibrium_fields(kappa: np.ndarray, intensity: np.ndarray) -> Fields:
    """Per-leaf constant absorption and equilibrium intensity I (emission kappa I)."""
    return Fields("const_eq", np.asarray(kappa, np.float32)[None, :].copy(),
                  np.asarray(intensity, np.float32)[None, :].copy())


def trilinear_fields_from_gaussians(forest: Forest, centers, sigmas,
                                    k0=0.2, k1=2.0, e0=0.1, e1=1.0) -> Fields:
    """Linear transfer of the Gaussian sum at each leaf corner to (kappa, eps)."""
    pts = corner_points(forest)
    s = np.empty((8, forest.nleaves))
    for c in range(8):
        s[c] = gaussian_sum(pts[c], centers, sigmas)
    return Fields("trilinear", (k0 + k1 * s).astype(np.float32), (e0 + e1 * s).astype(np.float32))


def perturb_fields(fields: Fields, rng, sigma=0.05) -> Fields:
    dk = rng.normal(0.0, sigma, fields.kappa.shape)
    de = rng.normal(0.0, sigma, fields.eps.shape)
    return Fields(fields.kind, (fields.kappa.astype(np.float64) + dk).astype(np.float32),
                  (fields.eps.astype(np.float64) + de).astype(np.float32))


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------


def _unit(a):
    a = np.asarray(a, np.float64)
    return a / np.linalg.norm(a)


def perspective_camera(eye, target, up, n, fov_deg, w, h, zfar, background=0.0) -> Camera:
    """Camera at ``eye`` looking at ``target``; ell from the horizontal field of view."""
    vh = _unit(np.asarray(target, np.float64) - np.asarray(eye, np.float64))
    up = np.asarray(up, np.float64)
    u = _unit(up - np.dot(up, vh) * vh)
    t = np.cross(vh, u)  # left-handed frame: t x u = -vh
    ell = 2.0 * n * math.tan(math.radians(fov_deg) / 2.0) / w
    return Camera(np.asarray(eye, np.float64), n * vh, t, u, ell, float(zfar), int(w), int(h), False,
                  float(background))


def random_perspective_camera(rng, w, h, dist=2.5, center=(0.5, 0.5, 0.5), n=1.0, fov_deg=42.0,
                              zfar=5.0, background=0.0) -> Camera:
    d = _unit(rng.normal(size=3))
    up = _unit(rng.normal(size=3))
    if abs(np.dot(up, d)) > 0.99:
        up = _unit(np.cross(d, [1.0, 0.0, 0.0]) + 0.1)
    c = np.asarray(center, np.float64)
    return perspective_camera(c + dist * d, c, up, n, fov_deg, w, h, zfar, background)


def orthographic_axis_camera(axis: int, sign: int, w=64, h=64, ell=1.0 / 64, n=1.0, zfar=3.0,
                             center=(0.5, 0.5, 0.5), background=0.0) -> Camera:
    vh = np.zeros(3)
    vh[axis] = float(sign)
    u = np.zeros(3)
    u[(axis + 1) % 3] = 1.0
    t = np.cross(vh, u)
    c = np.asarray(center, np.float64)
    return Camera(c - 2.0 * vh, n * vh, t, u, float(ell), float(zfar), int(w), int(h), True,
                  float(background))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------


def _gaussians(rng, k, smin, smax):
    centers = rng.uniform(0.0, 1.0, (k, 3))
    sigmas = rng.uniform(smin, smax, k)
    return centers, sigmas


def small_scene(seed=0, lmin=2, lmax=5, ngauss=4, w=96, h=72, method="rk4", ncams=1,
                background=0.0, sigma=(0.06, 0.2), ortho=False) -> Scene:
    """A few-thousand-leaf adaptive scene the oracle renders in well under a second."""
    rng = np.random.default_rng([1809, 1334, 1000 + seed])
    centers, sigmas = _gaussians(rng, ngauss, *sigma)
    forest = adaptive_forest(straddle_refiner(centers, sigmas), lmin, lmax)
    if method == "analytic":
        fields = constant_fields(rng.uniform(0.1, 2.0, forest.nleaves),
                                 rng.uniform(0.0, 1.0, forest.nleaves))
    else:
        fields = trilinear_fields_from_gaussians(forest, centers, sigmas)
    cams = []
    for _ in range(ncams):
        if ortho:
            cams.append(orthographic_axis_camera(int(rng.integers(3)), int(rng.choice([-1, 1])),
                                                 w=w, h=h, ell=1.4 / w, background=background))
        else:
            cams.append(random_perspective_camera(rng, w, h, background=background))
    return Scene(f"small{seed}", forest, fields, cams, method, 4,
                 {"centers": centers, "sigmas": sigmas})


def config4_cameras(ncams: int = 64, resolutions=(256, 512, 1024, 2048)) -> List[Camera]:
    """The cameras of workload 4 (drawn from its own seed) without rebuilding the forest."""
    rng = np.random.default_rng([1809, 1334, 4])
    res = rng.choice(list(resolutions), size=ncams)
    return [random_perspective_camera(rng, int(r), int(r)) for r in res]


def config_scene(k: int, w: Optional[int] = None) -> Scene:
    """The five seeded workloads.

    1: uniform level-3 unit cube, per-leaf constants, 64x64 orthographic, analytic.
    2: adaptive levels 4-9 (~1M leaves), trilinear, 1024^2 perspective, RK4 x 4.
    3: six-tree equiangular shell r in [0.55, 1], levels 3-7, trilinear, 2048^2 perspective at distance 3.
    4: the workload-2 forest seen by 64 cameras of uneven resolution.
    5: a workload-2-shaped forest, 512^2, background 0.5, perturbed target fields.
    """
    rng = np.random.default_rng([1809, 1334, k])
    if k == 1:
        forest = uniform_forest(3)
        kappa = rng.uniform(0.1, 2.0, forest.nleaves)
        eps = rng.uniform(0.0, 1.0, forest.nleaves)
        axis = int(rng.integers(3))
        sign = int(rng.choice([-1, 1]))
        cam = orthographic_axis_camera(axis, sign)
        return Scene("config1", forest, constant_fields(kappa, eps), [cam], "analytic", 1,
                     {"axis": axis, "sign": sign})
    if k in (2, 4, 5):
        # workload 4 renders the forest of workload 2 with cameras of its own seed
        frng = np.random.default_rng([1809, 1334, 2]) if k == 4 else rng
        centers, sigmas = _gaussians(frng, 8, 0.03, 0.1)
        forest = adaptive_forest(straddle_refiner(centers, sigmas), 4, 9)
        fields = trilinear_fields_from_gaussians(forest, centers, sigmas)
        extra = {"centers": centers, "sigmas": sigmas}
        if k == 2:
            cams = [random_perspective_camera(rng, w or 1024, w or 1024)]
        elif k == 4:
            res = rng.choice([256, 512, 1024, 2048], size=64)
            cams = [random_perspective_camera(rng, int(r), int(r)) for r in res]
        else:
            cams = [random_perspective_camera(rng, w or 512, w or 512, background=0.5)]
            extra["target_fields"] = perturb_fields(fields, rng, 0.05)
        return Scene(f"config{k}", forest, fields, cams, "rk4", 4, extra)
    if k == 3:
        return shell_scene(None, 3, 7, 8, w or 2048, w or 2048, name="config3")
    raise ValueError(f"workload {k} is not generated here")
