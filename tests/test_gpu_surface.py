"""GPU parity of surface forests (Sec. 2.8 surface model, eq. ABphi; App. A.1
ray against bilinear tree patches; the Mandelbrot hexagon of Sec. 4.1).

Pairing bit for bit against the oracle: for every candidate (visible leaf,
pixel of its rectangle), the number of hits the oracle gives to that leaf at
that pixel and their depths in FP64; every oracle hit lies in a candidate
(the leaf rectangles are conservative).  A, B and I within 1e-5 relative
(floor 1e-3 of the image maximum).
"""

import numpy as np
import pytest

import synth
from synth.scene import Camera
from test_gpu_parity import PIX_TOL, _torch, rel_err

pytestmark = pytest.mark.gpu


def _renderer(forest, fields, cams):
    import paper_1809_01334_amd as P

    print(f"[case] surface N={forest.nleaves} trees={forest.ntrees} cams={[(c.w, c.h) for c in cams]}", flush=True)
    return P.Renderer(forest, fields, cams, "analytic", 1)


def _candidates(r):
    """Camera, leaf and camera-local pixel of every candidate."""
    c = r.vf.read_counts()
    nvis = c["nvis"]
    leaf = r.vf.vis_leaf[:nvis].cpu().numpy().astype(np.int64)
    cam = r.vf.vis_cam[:nvis].cpu().numpy().astype(np.int64)
    rect = r.vf.vis_rect[:4 * nvis].cpu().numpy().reshape(-1, 4).astype(np.int64)
    off = r.vf.cand_offset[:nvis + 1].cpu().numpy()
    w = rect[:, 1] - rect[:, 0] + 1
    v = np.repeat(np.arange(nvis), np.diff(off))
    k = np.arange(off[-1]) - off[v]
    i = rect[v, 0] + k % w[v]
    j = rect[v, 2] + k // w[v]
    width = np.array([wh[0] for wh in r.cams.wh], np.int64)
    return cam[v], leaf[v], j * width[cam[v]] + i


def _check(r, forest, fields, cams, O, pixels=None, cand_sample=None):
    """Pairing (all candidates, or those at `pixels`) and images against the oracle."""
    torch = _torch()
    r.forward()
    hit, sio = r.debug_segments()
    torch.cuda.synchronize()
    ccam, cleaf, cpix = _candidates(r)
    n = len(ccam)
    hit = hit[:n].cpu().numpy().astype(np.int64)
    sio = sio[:4 * n].cpu().numpy().reshape(-1, 4)
    r.forward()
    A, B, I = (t.cpu().numpy() for t in (r.A, r.B, r.I))
    N = forest.nleaves
    total_hits = 0
    for k, cam in enumerate(cams):
        ref = O.surface_render(forest, fields, cam, pixels=pixels, hits=True)
        P_ = cam.w * cam.h
        pix = np.arange(P_) if pixels is None else np.asarray(pixels)
        H = ref["hit_leaf"].shape[1]
        ph = np.repeat(pix, H)
        lh = ref["hit_leaf"].ravel().astype(np.int64)
        sh = ref["hit_s"].ravel()
        m = lh >= 0
        key = ph[m] * N + lh[m]
        order = np.argsort(key, kind="stable")
        key, sh = key[order], sh[m][order]
        sel = ccam == k
        if pixels is not None:
            sel &= np.isin(cpix, pix)
        ck = cpix[sel] * N + cleaf[sel]
        lo = np.searchsorted(key, ck, "left")
        hi = np.searchsorted(key, ck, "right")
        cnt = hi - lo
        assert np.array_equal(hit[sel], cnt), (k, int((hit[sel] != cnt).sum()))
        assert cnt.sum() == len(key), "an oracle hit outside every candidate rectangle"
        s = sio[sel]
        one = cnt >= 1
        two = cnt == 2
        assert np.array_equal(s[one, 0].view(np.uint64), sh[lo[one]].view(np.uint64))
        assert np.array_equal(s[two, 2].view(np.uint64), sh[lo[two] + 1].view(np.uint64))
        total_hits += len(key)
        sl = slice(r.cams.img_off[k], r.cams.img_off[k + 1])
        for nm, x in (("A", A[sl]), ("B", B[sl]), ("I", I[sl])):
            got = x if pixels is None else x[pixels]
            e = rel_err(got, ref[nm])
            assert e <= PIX_TOL, (k, nm, e)
    return total_hits, hit


def _ortho(vh, up, center, w, h, ell, dist=3.0, zfar=6.0, background=0.0):
    vh = np.asarray(vh, np.float64) / np.linalg.norm(vh)
    u = np.asarray(up, np.float64)
    u = u - np.dot(u, vh) * vh
    u /= np.linalg.norm(u)
    return Camera(np.asarray(center, np.float64) - dist * vh, vh.copy(), np.cross(vh, u), u, float(ell),
                  float(zfar), w, h, True, float(background))


def test_flat_hexagon_two_cameras(oracle_mod):
    rng = np.random.default_rng(61)
    f = synth.random_quadtree_forest(rng, synth.hexagon_corners(), 2, 6, 0.45)
    fl = synth.random_surface_fields(rng, f.nleaves)
    cams = synth.hexagon_cameras(96, 80, background=0.3)
    cams[1] = synth.hexagon_cameras(73, 61, background=0.1)[1]
    r = _renderer(f, fl, cams)
    nh, _ = _check(r, f, fl, cams, oracle_mod)
    assert nh > 4000


def test_warped_hexagon_low_angle(oracle_mod):
    """Non-planar bilinear trees seen at a low angle, where rays can cross a tree twice."""
    rng = np.random.default_rng(62)
    corners = synth.hexagon_corners(z=(0.6, -0.5, 0.7, -0.6, 0.5, -0.7))
    f = synth.random_quadtree_forest(rng, corners, 2, 5, 0.5)
    fl = synth.random_surface_fields(rng, f.nleaves)
    cams = [synth.perspective_camera([-0.5 + 3.5, 0.3, 0.35], [-0.5, 0.0, 0.0], [0, 0, 1], 1.0, 60.0, 90, 70,
                                             10.0, 0.2),
            _ortho([0.9, 0.2, -0.15], [0, 0, 1], [-0.5, 0.0, 0.0], 80, 64, 4.2 / 80)]
    r = _renderer(f, fl, cams)
    _check(r, f, fl, cams, oracle_mod)


def test_saddle_double_hits(oracle_mod):
    """J = (t1, t2, t1 t2) refined to level 4, grazing views: pixels with two hits, in
    one leaf or in two."""
    rng = np.random.default_rng(63)
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 1]], np.float64)
    f = synth.random_quadtree_forest(rng, P, 1, 4, 0.6)
    fl = synth.random_surface_fields(rng, f.nleaves, opaque_frac=0.0)
    cams = [_ortho([0.7, -0.7, 0.08], [0, 0, 1], [0.5, 0.5, 0.3], 96, 64, 1.6 / 96),
            _ortho([-0.6, -0.75, 0.12], [0, 0, 1], [0.5, 0.5, 0.3], 64, 48, 1.6 / 64, background=0.5)]
    r = _renderer(f, fl, cams)
    _check(r, f, fl, cams, oracle_mod)
    two = 0
    for cam in cams:
        ref = oracle_mod.surface_render(f, fl, cam, hits=True)
        two += int(((ref["hit_leaf"] >= 0).sum(1) == 2).sum())
    assert two > 50


def test_stacked_trees_and_opaque_front(oracle_mod):
    """Three parallel trees: the fold over roots orders them by depth per pixel."""
    rng = np.random.default_rng(64)
    sq = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64)
    corners = np.stack([sq, sq + [0.1, 0.05, 0.4], sq + [-0.1, 0.0, 0.8]])
    f = synth.random_quadtree_forest(rng, corners, 1, 4, 0.5)
    fl = synth.random_surface_fields(rng, f.nleaves, opaque_frac=0.3)
    cams = [_ortho([0.2, 0.1, -1.0], [0, 1, 0], [0.5, 0.5, 0.4], 72, 72, 1.3 / 72, background=0.6),
            synth.perspective_camera([0.5, -2.0, 2.5], [0.5, 0.5, 0.4], [0, 0, 1], 1.0, 50.0, 64, 56, 10.0)]
    r = _renderer(f, fl, cams)
    _check(r, f, fl, cams, oracle_mod)


@pytest.mark.parametrize("instance", [0, 1])
def test_mandelbrot_small(oracle_mod, instance):
    f, val = synth.mandelbrot_forest(3, 7)
    fl = synth.mandelbrot_fields(val, instance)
    cams = synth.hexagon_cameras(128, 112)
    r = _renderer(f, fl, cams)
    _check(r, f, fl, cams, oracle_mod)


@pytest.mark.parametrize("seed", range(8))
def test_random_warped_trees(oracle_mod, seed):
    """Seeded random cases: one to three bilinear trees with random warped corners (rays may cross a tree twice,
    trees may overlap in depth), random refinement, fields with opaque leaves, and one or two random cameras
    (perspective or orthographic, random background): the full pairing and the images against the oracle."""
    rng = np.random.default_rng([6161, seed])
    ntrees = int(rng.integers(1, 4))
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64)
    corners = np.stack([base + rng.normal(0.0, 0.25, (4, 3)) + [0.0, 0.0, 0.35 * t] for t in range(ntrees)])
    f = synth.random_quadtree_forest(rng, corners, 1, int(rng.integers(3, 6)), 0.5)
    fl = synth.random_surface_fields(rng, f.nleaves, opaque_frac=float(rng.uniform(0.0, 0.4)))
    cams = []
    for _ in range(int(rng.integers(1, 3))):
        w, h = int(rng.integers(30, 90)), int(rng.integers(30, 90))
        if rng.integers(2):
            d = rng.normal(size=3)
            cams.append(_ortho(d, [0, 0, 1] if abs(d[2]) < 0.9 * np.linalg.norm(d) else [1, 0, 0],
                               [0.5, 0.5, 0.35], w, h, 2.2 / w, background=float(rng.uniform(0, 0.5))))
        else:
            cams.append(synth.random_perspective_camera(rng, w, h, dist=3.0, center=(0.5, 0.5, 0.35),
                                                        zfar=8.0, background=float(rng.uniform(0, 0.5))))
    r = _renderer(f, fl, cams)
    nh, _ = _check(r, f, fl, cams, oracle_mod)
    assert nh > 100


def test_surface_rejections_and_graph_replay(oracle_mod):
    torch = _torch()
    import paper_1809_01334_amd as P

    f, val = synth.mandelbrot_forest(3, 5)
    fl = synth.mandelbrot_fields(val, 1)
    cams = synth.hexagon_cameras(64, 48)
    r = _renderer(f, fl, cams)
    r.forward()
    ref = r.I.clone()
    with pytest.raises(P.RcError) as e:
        r.backward(torch.ones_like(r.I))
    assert e.value.status == P._lib.RC_EUNSUPPORTED
    with pytest.raises(P.RcError) as e:
        r.composite_lists()
    assert e.value.status == P._lib.RC_EUNSUPPORTED
    r.capture()
    for _ in range(3):
        r.I.zero_()
        torch.cuda.synchronize()
        r.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.I, ref)


@pytest.mark.timeout(600)
def test_mandelbrot_full_size_sampled(oracle_mod):
    """Levels 4-11 (about 500 k leaves), two 1024^2 instances: pairing of every candidate
    at 2000 sampled pixels per view and the images there."""
    f, val = synth.mandelbrot_forest(4, 11)
    fl = synth.mandelbrot_fields(val, 1)
    cams = synth.hexagon_cameras(1024, 1024)
    r = _renderer(f, fl, cams)
    pix = np.sort(np.random.default_rng(65).choice(1024 * 1024, 2000, replace=False))
    nh, _ = _check(r, f, fl, cams, oracle_mod, pixels=pix)
    assert nh > 1000
