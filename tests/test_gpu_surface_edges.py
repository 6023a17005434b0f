"""GPU parity of degree-R surfaces on the rays that tests with random pixels
avoid (App. A.1 ray against tensor-product surfaces; eq. tensorgeom):

* rays through points on leaf edges and corners, and at parameter offsets of
  1e-3 down to 1e-14 on either side: the same single hit, in the same leaf (the
  leaf whose half-open extent holds the root rounded to the 2^-40 grid, on both
  sides), at the same depth (1e-9) and with the same image (1e-5);
* rays near a tangency of the paraboloid z = c ((t1 - 1/2)^2 + (t2 - 1/2)^2),
  at heights eta above the tangent one from 1e-2 down to 1e-14 (two roots
  2 sqrt(eta / c) apart, in the two leaves meeting at t1 = 1/2) and below it
  (no root): the same hits, leaves and images; the depths agree to about
  1e-16 / sqrt(eta) (1e-9 at eta = 1e-14).  The exactly tangent ray (a double
  root, which rounding turns into a near miss or a near pair) may give 0, 1 or
  2 hits on either side and is not compared.

Each ray is the one pixel of an orthographic 1 x 1 camera, whose ray starts
exactly at the camera's origin.
"""

import numpy as np
import pytest

import synth
from synth.scene import Camera
from test_gpu_parity import PIX_TOL, _torch, rel_err
from test_gpu_surface import _candidates

pytestmark = pytest.mark.gpu


def _ray(o, vh, up=(0.0, 0.0, 1.0), zfar=8.0):
    vh = np.asarray(vh, np.float64) / np.linalg.norm(vh)
    u = np.asarray(up, np.float64)
    u = u - np.dot(u, vh) * vh
    u /= np.linalg.norm(u)
    return Camera(np.asarray(o, np.float64), vh.copy(), np.cross(vh, u), u, 1e-3, zfar, 1, 1, True, 0.0)


def _compare(forest, fields, cams, tags, O, skip=()):
    torch = _torch()
    import paper_1809_01334_amd as P

    print(f"[case] degree-{int(forest.geom_params[0])} surface, {len(cams)} one-pixel rays", flush=True)
    r = P.Renderer(forest, fields, cams, "analytic", 1)
    r.forward()
    hit, sio = r.debug_segments()
    torch.cuda.synchronize()
    ccam, cleaf, _ = _candidates(r)
    n = len(ccam)
    hit = hit[:n].cpu().numpy().astype(np.int64)
    sio = sio[:4 * n].cpu().numpy().reshape(-1, 4)
    r.forward()
    I = r.I.cpu().numpy()
    hits = 0
    for k, cam in enumerate(cams):
        if tags[k] in skip:
            continue
        ref = O.ho_surface_render(forest, fields, cam, hits=True)
        m = ref["hit_leaf"][0] >= 0
        o_leaf, o_s = ref["hit_leaf"][0][m], ref["hit_s"][0][m]
        g_leaf, g_s = [], []
        sel = ccam == k
        for h, l, s in zip(hit[sel], cleaf[sel], sio[sel]):
            for q in range(min(int(h), 2)):
                g_leaf.append(int(l))
                g_s.append(s[2 * q])
        assert sorted(g_leaf) == sorted(o_leaf.tolist()), (tags[k], g_leaf, o_leaf)
        np.testing.assert_allclose(np.sort(g_s), np.sort(o_s), rtol=1e-9, err_msg=tags[k])
        assert rel_err(I[k:k + 1], ref["I"]) <= PIX_TOL, tags[k]
        hits += len(g_leaf)
    return hits


@pytest.mark.parametrize("R", [2, 3])
def test_rays_on_and_near_leaf_edges(oracle_mod, R):
    O = oracle_mod
    rng = np.random.default_rng(700 + R)
    fn = lambda a, b: np.stack([a + 0.1 * b * b, b + 0.05 * a * b,  # noqa: E731
                                0.25 * (a - 0.3) ** 2 - 0.2 * b * b + 0.1 * a * b], -1)
    f = synth.ho_random_forest(rng, [synth.ho_tree(fn, R)], R, 2, 4, 0.5)
    fl = synth.random_surface_fields(rng, f.nleaves, opaque_frac=0.0)
    geom = np.asarray(f.geom_params)
    cams, tags = [], []
    offsets = (1e-3, 1e-6, 1e-9, 1e-11, 1e-12, 1e-13, 1e-14, 0.0, -1e-14, -1e-13, -1e-12, -1e-9, -1e-6)
    for e, t2 in ((0.5, 0.37), (0.25, 0.61), (0.75, 0.13), (0.375, 0.8)):
        for d in offsets:
            for axis in (0, 1):
                t = (e + d, t2) if axis == 0 else (t2, e + d)
                p = O.ho_map(geom, 0, np.array([t]))[0]
                vh = np.array([0.3, -0.2, -1.0])
                cams.append(_ray(p - 3.0 * vh / np.linalg.norm(vh), vh))
                tags.append(f"edge {e} axis {axis} offset {d:+.0e}")
    for e1, e2 in ((0.5, 0.5), (0.25, 0.75), (0.5, 0.25)):
        for d in (1e-9, 1e-12, 1e-14, 0.0, -1e-14, -1e-12):
            p = O.ho_map(geom, 0, np.array([(e1 + d, e2 + d)]))[0]
            vh = np.array([-0.2, 0.35, -1.0])
            cams.append(_ray(p - 3.0 * vh / np.linalg.norm(vh), vh))
            tags.append(f"corner {e1},{e2} offset {d:+.0e}")
    assert _compare(f, fl, cams, tags, O) == len(cams)


@pytest.mark.parametrize("R", [2, 3])
def test_rays_near_a_tangency(oracle_mod, R):
    c, y0 = 0.8, 0.8
    trees = [synth.ho_tree(lambda a, b: np.stack([a, b, c * ((a - 0.5) ** 2 + (b - 0.5) ** 2)], -1), R)]
    f = synth.ho_random_forest(np.random.default_rng(3), trees, R, 1, 3, 0.5)
    fl = synth.random_surface_fields(np.random.default_rng(4), f.nleaves, opaque_frac=0.0)
    zt = c * (y0 - 0.5) ** 2
    etas = (1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14, 0.0, -1e-14, -1e-12, -1e-10, -1e-8, -1e-4)
    cams = [_ray([-1.0, y0, zt + eta], [1.0, 0.0, 0.0]) for eta in etas]
    tags = [f"tangent eta {eta:+.0e}" for eta in etas]
    hits = _compare(f, fl, cams, tags, oracle_mod, skip=("tangent eta +0e+00",))
    assert hits == 2 * 7
