"""GPU parity of degree-R surface forests (eq. nodal, eq. tensorgeom; App. A.1
ray against tensor-product surfaces; App. A.2 boxes; Sec. 2.8 surface model).

The GPU searches each candidate's leaf square with camera-space Bernstein
polynomials (eq. camerapoints) and Newton's method; the oracle subdivides the
whole tree square in world space.  Per candidate, the number of hits the
oracle gives to that leaf at that pixel must match, every oracle hit must lie
in a candidate rectangle, depths agree to 1e-9 relative, and A, B and I to
1e-5 relative (floor 1e-3 of the image maximum).
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import PIX_TOL, _torch, rel_err
from test_gpu_surface import _candidates, _ortho

pytestmark = pytest.mark.gpu


def _check_ho(forest, fields, cams, O, pixels=None):
    torch = _torch()
    import paper_1809_01334_amd as P

    print(f"[case] degree-{int(forest.geom_params[0])} surface N={forest.nleaves} trees={forest.ntrees} "
          f"cams={[(c.w, c.h) for c in cams]}", flush=True)
    r = P.Renderer(forest, fields, cams, "analytic", 1)
    r.forward()
    hit, sio = r.debug_segments()
    torch.cuda.synchronize()
    ccam, cleaf, cpix = _candidates(r)
    n = len(ccam)
    hit = hit[:n].cpu().numpy().astype(np.int64)
    sio = sio[:4 * n].cpu().numpy().reshape(-1, 4)
    assert hit.max(initial=0) <= 2
    r.forward()
    A, B, I = (t.cpu().numpy() for t in (r.A, r.B, r.I))
    N = forest.nleaves
    total = 0
    for k, cam in enumerate(cams):
        ref = O.ho_surface_render(forest, fields, cam, pixels=pixels, hits=True)
        pix = np.arange(cam.w * cam.h) if pixels is None else np.asarray(pixels)
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
        if not np.array_equal(hit[sel], cnt):
            bad = np.nonzero(hit[sel] != cnt)[0]
            for b in bad[:8]:
                print(f"[mismatch] cam {k} pixel {cpix[sel][b]} leaf {cleaf[sel][b]} gpu {hit[sel][b]} "
                      f"{sio[sel][b, [0, 2]]} oracle {cnt[b]} {sh[lo[b]:hi[b]]} "
                      f"pixel hits {ref['hit_s'][np.searchsorted(pix, cpix[sel][b])]}", flush=True)
            raise AssertionError((k, len(bad)))
        assert cnt.sum() == len(key), "an oracle hit outside every candidate rectangle"
        s = sio[sel]
        one, two = cnt >= 1, cnt == 2
        np.testing.assert_allclose(s[one, 0], sh[lo[one]], rtol=1e-9)
        np.testing.assert_allclose(s[two, 2], sh[lo[two] + 1], rtol=1e-9)
        total += len(key)
        sl = slice(r.cams.img_off[k], r.cams.img_off[k + 1])
        for nm, x in (("A", A[sl]), ("B", B[sl]), ("I", I[sl])):
            got = x if pixels is None else x[pixels]
            e = rel_err(got, ref[nm])
            assert e <= PIX_TOL, (k, nm, e)
    return total


@pytest.mark.parametrize("R", [2, 3])
def test_lifted_hexagon(oracle_mod, R):
    rng = np.random.default_rng(80 + R)
    trees = synth.ho_hexagon_trees(R, lambda x, y: 0.35 * np.sin(2 * x) * np.cos(1.5 * y))
    f = synth.ho_random_forest(rng, trees, R, 2, 5, 0.45)
    fl = synth.random_surface_fields(rng, f.nleaves)
    cams = [synth.hexagon_cameras(88, 72, background=0.3)[0],
            synth.perspective_camera([2.8, 1.2, 1.0], [-0.5, 0.0, 0.0], [0, 0, 1], 1.0, 55.0, 70, 60, 10.0, 0.1)]
    assert _check_ho(f, fl, cams, oracle_mod) > 3000


def test_paraboloid_cups_two_hits(oracle_mod):
    """z = c (t1^2 + t2^2) patches seen from the side: rays entering and leaving a cup."""
    rng = np.random.default_rng(82)
    c = 0.8
    trees = [synth.ho_tree(lambda a, b: np.stack([a, b, c * ((a - 0.5) ** 2 + (b - 0.5) ** 2)], -1), 2),
             synth.ho_tree(lambda a, b: np.stack([a + 1.2, b, 0.1 + c * ((a - 0.5) ** 2 + (b - 0.5) ** 2)], -1), 2)]
    f = synth.ho_random_forest(rng, trees, 2, 1, 4, 0.5)
    fl = synth.random_surface_fields(rng, f.nleaves, opaque_frac=0.0)
    cams = [_ortho([0.15, 1.0, -0.1], [0, 0, 1], [1.1, 0.5, 0.2], 96, 40, 2.6 / 96),
            _ortho([-0.1, 1.0, -0.2], [0, 0, 1], [1.1, 0.5, 0.2], 64, 32, 2.6 / 64, background=0.4)]
    _check_ho(f, fl, cams, oracle_mod)
    two = 0
    for cam in cams:
        ref = oracle_mod.ho_surface_render(f, fl, cam, hits=True)
        two += int(((ref["hit_leaf"] >= 0).sum(1) >= 2).sum())
    assert two > 30


def test_cubic_graph_orthographic_and_mandelbrot_data(oracle_mod):
    """A degree-3 graph carrying the Mandelbrot corner data of its (x, y)."""
    def fn(a, b):
        x = -2.2 + 2.8 * a
        y = -1.4 + 2.8 * b
        return np.stack([x, y, 0.2 * (a ** 3 - 2 * a * b * b + 0.5 * b ** 3)], -1)

    rng = np.random.default_rng(83)
    f = synth.ho_random_forest(rng, [synth.ho_tree(fn, 3)], 3, 3, 6, 0.5)
    pts = synth.leaf_corner_points(synth.surface_forest(
        np.array([fn(np.array([0.0]), np.array([0.0]))[0], fn(np.array([1.0]), np.array([0.0]))[0],
                  fn(np.array([0.0]), np.array([1.0]))[0], fn(np.array([1.0]), np.array([1.0]))[0]]),
        f.level, f.x, f.y, np.zeros(f.nleaves, np.int64)))
    val = synth.mandelbrot_count(pts[..., 0] + 1j * pts[..., 1])
    fl = synth.mandelbrot_fields(val, 1)
    cams = [_ortho([0.1, -0.2, -1.0], [0, 1, 0], [-0.8, 0.0, 0.0], 80, 80, 3.0 / 80),
            synth.perspective_camera([-0.8, -3.0, 2.5], [-0.8, 0.0, 0.0], [0, 0, 1], 1.0, 55.0, 72, 64, 10.0)]
    _check_ho(f, fl, cams, oracle_mod)


@pytest.mark.timeout(600)
def test_lifted_hexagon_full_size_sampled(oracle_mod):
    """Degree 2, the Mandelbrot refinement (levels 4-9) on the lifted hexagon, 1024^2, 1500 sampled pixels."""
    R = 2
    trees = synth.ho_hexagon_trees(R, lambda x, y: 0.35 * np.sin(2 * x) * np.cos(1.5 * y))
    base, val = synth.mandelbrot_forest(4, 9)
    f = synth.ho_surface_forest(trees, R, base.level, base.x, base.y, base.tree_of_leaf())
    fl = synth.mandelbrot_fields(val, 1)
    cams = synth.hexagon_cameras(1024, 1024)[:1]
    pix = np.sort(np.random.default_rng(84).choice(1024 * 1024, 1500, replace=False))
    assert _check_ho(f, fl, cams, oracle_mod, pixels=pix) > 500
