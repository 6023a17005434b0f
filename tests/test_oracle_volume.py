"""Pins of the oracle's degree-R volume trees (Sec. 2.1 curved elements, App. A.1
faces): a tree map that is the identity, or a similarity, of the unit cube must
render as the unit-cube oracle does; a bent cube whose faces are parabolic
cylinders has closed-form chords, so a constant medium has a closed-form image
and the leaves of a forest tile every ray's chord; trilinear fields against
brute-force marching with the closed-form inverse map."""

import numpy as np
import pytest

import synth

R_DEG = (2, 3)


def _identity_tree(R):
    return synth.vol_tree(lambda a, b, c: np.stack([a, b, c], -1), R)


@pytest.mark.parametrize("R", R_DEG)
def test_identity_map_renders_as_the_unit_cube(oracle_mod, R):
    """Control points on the node grid of the identity: the leaves' faces are the cube's, the Newton
    inverse is exact, so the images equal the unit-cube oracle's (RK4 x 4, trilinear) to rounding."""
    O = oracle_mod
    sc = synth.small_scene(3, lmin=1, lmax=3, ngauss=3, w=24, h=18, background=0.3)
    vf = synth.volume_forest([_identity_tree(R)], R, sc.forest)
    rv = O.vol_render(vf, sc.fields, sc.cameras[0], "rk4", 4)
    rc = O.render(sc.forest, sc.fields, sc.cameras[0], "rk4", 4)
    assert rv["segments"] == rc["segments"] > 500 and rv["overlaps"] == 0
    for k in ("A", "B", "I"):
        assert np.abs(rv[k] - rc[k]).max() < 1e-12


def test_similarity_map_renders_as_the_transformed_camera(oracle_mod):
    """x = s Q xi + b (a rotation, a scale, a shift): the cube oracle with the camera taken back by the inverse
    map (lengths shrink by s, so kappa and eps grow by s) renders the same image."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    s, b = 1.7, np.array([0.3, -0.2, 0.5])
    tree = synth.vol_tree(lambda t1, t2, t3: (s * (np.stack([t1, t2, t3], -1) @ Q.T)) + b, 2)
    sc = synth.small_scene(4, lmin=1, lmax=3, ngauss=3, w=20, h=16)
    vf = synth.volume_forest([tree], 2, sc.forest)
    centre = s * (np.array([0.5, 0.5, 0.5]) @ Q.T) + b
    cam = synth.random_perspective_camera(rng, 20, 16, dist=4.0, center=tuple(centre), zfar=8.0)
    rv = O.vol_render(vf, sc.fields, cam, "rk4", 4)
    # the camera in reference coordinates
    inv = lambda p: (np.asarray(p) - b) @ Q / s  # noqa: E731
    back = synth.Camera(inv(cam.o), cam.v @ Q / s, cam.t @ Q, cam.u @ Q, cam.ell / s, cam.zfar / s, cam.w, cam.h,
                        cam.ortho, cam.background)
    fs = synth.Fields(sc.fields.kind, (sc.fields.kappa.astype(np.float64) * s), sc.fields.eps.astype(np.float64) * s)
    rc = O.render(sc.forest, fs, back, "rk4", 4)
    assert rv["segments"] == rc["segments"] > 100
    for k in ("A", "B", "I"):
        assert np.abs(rv[k] - rc[k]).max() < 1e-10


def _bent_chord(c, rho, r, smin, smax):
    """Parameter intervals where rho + s r lies in {0 <= x, y <= 1, 0 <= z - c x^2 <= 1}: the x and y slabs
    are linear in s, z - c x^2 is quadratic."""
    lo, hi = smin, smax
    for k in (0, 1):
        if r[k] == 0.0:
            if not (0.0 <= rho[k] <= 1.0):
                return []
            continue
        a, bb = (0.0 - rho[k]) / r[k], (1.0 - rho[k]) / r[k]
        lo, hi = max(lo, min(a, bb)), min(hi, max(a, bb))
    if not hi > lo:
        return []
    # g(s) = (rho_z + s r_z) - c (rho_x + s r_x)^2 = g2 s^2 + g1 s + g0
    g2, g1, g0 = -c * r[0] ** 2, r[2] - 2.0 * c * rho[0] * r[0], rho[2] - c * rho[0] ** 2
    cuts = [lo, hi]
    for level in (0.0, 1.0):
        for root in np.roots([g2, g1, g0 - level]):
            if abs(root.imag) < 1e-12 and lo < root.real < hi:
                cuts.append(root.real)
    cuts = sorted(cuts)
    out = []
    for a, bb in zip(cuts[:-1], cuts[1:]):
        m = 0.5 * (a + bb)
        g = g2 * m * m + g1 * m + g0
        if 0.0 <= g <= 1.0 and bb > a:
            if out and abs(out[-1][1] - a) < 1e-14:
                out[-1][1] = bb
            else:
                out.append([a, bb])
    return out


def _ray(cam, i, j):
    a = cam.ell * (i - (cam.w - 1) / 2.0)
    b = cam.ell * (j - (cam.h - 1) / 2.0)
    return cam.o.copy(), cam.v + a * cam.t + b * cam.u


@pytest.mark.parametrize("c", [0.25, -0.4])
def test_bent_cube_constant_medium_closed_form(oracle_mod, c):
    """One leaf and a refined forest on the bent cube, constant (kappa, eps): every pixel's A and B are the
    closed form over the ray's chord, exp(-kappa L) and (eps / kappa)(1 - exp(-kappa L))."""
    O = oracle_mod
    cam = synth.perspective_camera([2.2, -1.4, 2.0], [0.5, 0.5, 0.6 + 0.3 * c], [0, 0, 1], 1.0, 40.0, 24, 20, 6.0)
    kap, eps = 1.25, 0.75  # exact in FP32, the fields' storage
    for base in (synth.uniform_forest(0), synth.uniform_forest(2)):
        N = base.nleaves
        vf = synth.volume_forest([synth.vol_tree(synth.bent_map(c), 2)], 2, base)
        fields = synth.constant_fields(np.full(N, kap), np.full(N, eps))
        rv = O.vol_render(vf, fields, cam, "analytic", 1)
        A = np.ones(cam.npix)
        for j in range(cam.h):
            for i in range(cam.w):
                rho, r = _ray(cam, i, j)
                L = sum(b - a for a, b in _bent_chord(c, rho, r, 1.0, 6.0)) * np.linalg.norm(r)
                A[j * cam.w + i] = np.exp(-kap * L)
        assert (A < 0.999).sum() > 50
        assert np.abs(rv["A"] - A).max() < 1e-11
        assert np.abs(rv["B"] - eps / kap * (1.0 - A)).max() < 1e-11


def test_bent_cube_leaves_tile_the_chord(oracle_mod):
    """Over a refined bent cube, every leaf's intervals along a ray (explicit candidates, all leaves) add up
    to the closed-form chord: the faces' crossings and the inside tests lose and double-count nothing."""
    O = oracle_mod
    c = 0.3
    base = synth.uniform_forest(2)
    vf = synth.volume_forest([synth.vol_tree(synth.bent_map(c), 2)], 2, base)
    cam = synth.perspective_camera([1.9, 2.3, 1.6], [0.5, 0.5, 0.65], [0, 0, 1], 1.0, 38.0, 9, 7, 6.0)
    N = base.nleaves
    crossed = 0
    for j in range(cam.h):
        for i in range(cam.w):
            rho, r = _ray(cam, i, j)
            want = sum(b - a for a, b in _bent_chord(c, rho, r, 1.0, 6.0))
            ns, iv = O.vol_cands(vf, cam.raw(), np.arange(N), np.full(N, i), np.full(N, j))
            assert ns.max() <= 2
            got = float(((iv[:, 1] - iv[:, 0]) * (ns >= 1) + (iv[:, 3] - iv[:, 2]) * (ns >= 2)).sum())
            assert abs(got - want) < 1e-11, (i, j, got, want)
            crossed += int(want > 0.0 and (ns > 0).sum() >= 3)
    assert crossed > 20


def test_bent_cube_trilinear_against_marching(oracle_mod):
    """Trilinear fields on a refined bent cube: RK4 x 8 per segment against brute-force marching (midpoint
    steps of the constant-coefficient closed form at points located by the closed-form inverse map)."""
    O = oracle_mod
    c = 0.3
    rng = np.random.default_rng(11)
    base = synth.uniform_forest(2)
    N = base.nleaves
    centers, sigmas = rng.uniform(0, 1, (3, 3)), rng.uniform(0.15, 0.3, 3)
    fields = synth.trilinear_fields_from_gaussians(base, centers, sigmas)
    vf = synth.volume_forest([synth.vol_tree(synth.bent_map(c), 2)], 2, base)
    cam = synth.perspective_camera([2.0, -1.2, 1.8], [0.5, 0.5, 0.65], [0, 0, 1], 1.0, 34.0, 6, 5, 6.0)
    rv = O.vol_render(vf, fields, cam, "rk4", 8)
    kap = fields.kappa.astype(np.float64)
    eps = fields.eps.astype(np.float64)
    lv, xs, ys, zs = base.level, base.x, base.y, base.z
    scale = 1.0 / (1 << synth.QMAX)

    def leaf_of(xi):
        for l in range(N):
            h = 1.0 / (1 << int(lv[l]))
            lo = np.array([xs[l], ys[l], zs[l]]) * scale
            if np.all(xi >= lo) and np.all(xi <= lo + h):
                return l, (xi - lo) / h
        return -1, None

    M = 4000
    for j in range(cam.h):
        for i in range(cam.w):
            rho, r = _ray(cam, i, j)
            A, B = 1.0, 0.0
            for a, b in _bent_chord(c, rho, r, 1.0, 6.0):
                ds = (b - a) / M
                for q in range(M):  # nearest first
                    s = a + (q + 0.5) * ds
                    x = rho + s * r
                    xi = np.array([x[0], x[1], x[2] - c * x[0] ** 2])
                    l, u = leaf_of(np.clip(xi, 0.0, 1.0))
                    w = np.array([(u[0] if k & 1 else 1 - u[0]) * (u[1] if k & 2 else 1 - u[1]) *
                                  (u[2] if k & 4 else 1 - u[2]) for k in range(8)])
                    kk, ee = float(w @ kap[:, l]), float(w @ eps[:, l])
                    dx = ds * np.linalg.norm(r)
                    a_ = np.exp(-kk * dx)
                    b_ = ee / kk * (1 - a_)
                    B = B + A * b_
                    A = A * a_
            p = j * cam.w + i
            assert abs(rv["A"][p] - A) < 2e-6 and abs(rv["B"][p] - B) < 2e-6, (i, j)


def test_random_quadratic_map_inverse_round_trip(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(5)
    tree = synth.vol_tree(synth.random_quadratic_map(rng, 0.08), 2)
    geom = synth.vol_geom([tree], 2)
    xi = rng.uniform(0.0, 1.0, (200, 3))
    x = O.vol_map(geom, 0, xi)
    back, ok = O.vol_inverse(geom, 0, x)
    assert ok and np.abs(back - xi).max() < 1e-13
    # the map interpolates its control points at the node triples (eq. nodal)
    eta = synth.gl_nodes(2)
    t3, t2, t1 = np.meshgrid(eta, eta, eta, indexing="ij")
    nodes = np.stack([t1.ravel(), t2.ravel(), t3.ravel()], -1)
    assert np.abs(O.vol_map(geom, 0, nodes) - tree).max() < 1e-14
