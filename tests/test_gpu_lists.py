"""GPU parity of share compositing (Sec. 3.3 coarsening stopped at a share's
maximal complete subtrees, Sec. 3.5 per-pixel lists, Sec. 2.5 cutting and
averaging overlapping segments) against the oracle.

Per-pixel entry counts and intervals are compared bit for bit (the intervals
are the oracle's FP64 slab values rounded to float), A and B within 1e-5; the
merged images of a partition within 1e-5 of the full render.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import PIX_TOL, _torch, rel_err

pytestmark = pytest.mark.gpu


def _depth_order(off, ent):
    """Permutation putting every pixel's entries in (s_in, s_out, A, B) order of their float values."""
    off = np.asarray(off, np.int64)
    e = np.asarray(ent).reshape(-1, 4).astype(np.float32)
    pix = np.repeat(np.arange(off.size - 1), np.diff(off))
    return np.lexsort((e[:, 3], e[:, 2], e[:, 1], e[:, 0], pix))


def _share_lists(scene, forest, fields, method, substeps):
    import paper_1809_01334_amd as P

    r = P.Renderer(forest, fields, scene.cameras, method, substeps)
    off, ent = r.forward_lists()
    _torch().cuda.synchronize()
    return r, off, ent


def _check_lists(r, off, ent, scene, forest, fields, O):
    off_h = off.cpu().numpy()
    ent_h = ent.cpu().numpy()
    assert off_h[0] == 0 and off_h[-1] == ent_h.shape[0]
    for k, cam in enumerate(scene.cameras):
        lo, hi = int(r.cams.img_off[k]), int(r.cams.img_off[k + 1])
        ro, re_ = O.share_lists(forest, fields, cam, scene.method, scene.substeps)
        go = off_h[lo:hi + 1] - off_h[lo]
        np.testing.assert_array_equal(go, ro)  # entries per pixel
        g = ent_h[off_h[lo]:off_h[hi]]
        g = g[_depth_order(go, g)]
        q = np.asarray(re_, np.float64).reshape(-1, 4)
        q = q[_depth_order(ro, q)]
        np.testing.assert_array_equal(g[:, :2], q[:, :2].astype(np.float32))  # intervals
        for c in (2, 3) if q.shape[0] else ():
            err = rel_err(g[:, c], q[:, c])
            assert err <= PIX_TOL, (k, c, err)
    return ent_h.shape[0]


@pytest.mark.parametrize("ncuts", [0, 3])
def test_share_lists_match_oracle(oracle_mod, ncuts):
    _torch()
    sc = synth.small_scene(41, ncams=2, w=56, h=44, background=0.3)
    rng = np.random.default_rng(41)
    N = sc.forest.nleaves
    cuts = sorted(rng.choice(np.arange(1, N), ncuts, replace=False)) if ncuts else []
    for i, (f, fl) in enumerate(synth.split_shares(sc.forest, sc.fields, cuts)):
        print(f"[case] share {i} of {ncuts + 1}: {f.nleaves} leaves", flush=True)
        r, off, ent = _share_lists(sc, f, fl, sc.method, sc.substeps)
        _check_lists(r, off, ent, sc, f, fl, oracle_mod)
        if ncuts == 0:
            # the whole forest is one unit, the root: at most one entry per pixel
            assert int(np.diff(off.cpu().numpy()).max()) == 1


def test_merged_partition_equals_full_render(oracle_mod):
    torch = _torch()
    import paper_1809_01334_amd as P

    sc = synth.small_scene(42, ncams=2, w=64, h=52, background=0.25)
    N = sc.forest.nleaves
    cuts = [N // 5, N // 2 + 3, N // 2 + 4, 4 * N // 5]
    shares = synth.split_shares(sc.forest, sc.fields, cuts)
    lists, rs = [], []
    for i, (f, fl) in enumerate(shares):
        print(f"[case] partition share {i}: {f.nleaves} leaves", flush=True)
        r, off, ent = _share_lists(sc, f, fl, sc.method, sc.substeps)
        lists.append((off, ent))
        rs.append(r)
    A, B, I, ov = P.merge_lists(rs[0].cams, lists)
    torch.cuda.synchronize()
    assert ov == 0  # shares meet at shared faces with equal depths
    A, B, I = (t.cpu().numpy() for t in (A, B, I))
    for k, cam in enumerate(sc.cameras):
        sl = slice(rs[0].cams.img_off[k], rs[0].cams.img_off[k + 1])
        ref = oracle_mod.render(sc.forest, sc.fields, cam, sc.method, sc.substeps)
        for nm, x in (("A", A[sl]), ("B", B[sl]), ("I", I[sl])):
            err = rel_err(x, ref[nm])
            assert err <= PIX_TOL, (k, nm, err)


def test_single_leaf_and_single_level_shares(oracle_mod):
    """Shares of one leaf and of one sibling group: units are the leaves themselves."""
    _torch()
    sc = synth.small_scene(43, w=40, h=36)
    N = sc.forest.nleaves
    seen = 0
    for a, b in ((0, 1), (N - 1, N), (N // 2, N // 2 + 1), (1, 9), (N // 2, N // 2 + 8)):
        f, fl = synth.split_shares(sc.forest, sc.fields, [c for c in (a, b) if 0 < c < N])[1 if a > 0 else 0]
        print(f"[case] leaves [{a}, {b}): {f.nleaves}", flush=True)
        r, off, ent = _share_lists(sc, f, fl, sc.method, sc.substeps)
        seen += _check_lists(r, off, ent, sc, f, fl, oracle_mod)  # an invisible share has no entries
    assert seen > 0


def _synthetic_lists(rng, P_, nlists, max_per):
    """Per-pixel lists of constant-medium entries, each list sorted with disjoint
    (sometimes touching) intervals, the lists overlapping one another; some entries
    transparent (A = 1), some opaque (A = 0), some of zero length (opaque surfaces),
    and some pixels with one entry repeated in every list."""
    out = []
    for _ in range(nlists):
        cnt = rng.integers(0, max_per + 1, P_)
        off = np.zeros(P_ + 1, np.int64)
        off[1:] = np.cumsum(cnt)
        rows = []
        for c in cnt:
            b = np.sort(rng.uniform(1.0, 5.0, 2 * c))
            for q in range(1, c):
                if rng.random() < 0.3:
                    b[2 * q] = b[2 * q - 1]  # touching the previous entry
            rows.extend(zip(b[0::2], b[1::2]))
        m = int(off[-1])
        iv = np.asarray(rows, np.float64).reshape(m, 2)
        flat = rng.random(m) < 0.05
        iv[flat, 1] = iv[flat, 0]
        ln = iv[:, 1] - iv[:, 0]
        beta = rng.uniform(0.0, 3.0, m)
        beta[rng.random(m) < 0.1] = 0.0
        gamma = rng.uniform(0.0, 1.0, m)
        A = np.exp(-beta * ln)
        B = np.where(beta > 0, gamma / np.maximum(beta, 1e-30) * (1 - A), gamma * ln)
        opaque = (rng.random(m) < 0.05) | flat
        A[opaque] = 0.0
        B[flat] = gamma[flat]
        out.append((off, np.stack([iv[:, 0], iv[:, 1], A, B], 1).astype(np.float32)))
    # pixels whose first entry is the same in every list
    for p in rng.choice(P_, P_ // 20, replace=False):
        if all(o[p + 1] - o[p] == 1 for o, _ in out):
            for o, e in out[1:]:
                e[o[p]] = out[0][1][out[0][0][p]]
    return out


@pytest.mark.parametrize("nlists,max_per", [(1, 4), (3, 3), (16, 1)])
def test_merge_of_overlapping_lists_matches_oracle(oracle_mod, nlists, max_per):
    torch = _torch()
    import paper_1809_01334_amd as P

    rng = np.random.default_rng(44 + nlists)
    cam = synth.random_perspective_camera(rng, 61, 47, background=0.6)
    cams = P.rc_camera_prepare(cam.raw()[None, :], torch.device("cuda:0"))
    lists = _synthetic_lists(rng, cams.npix, nlists, max_per)
    print(f"[case] merge {nlists} lists, {sum(e.shape[0] for _, e in lists)} entries", flush=True)
    dev = [(torch.from_numpy(o).cuda(), torch.from_numpy(e.reshape(-1)).cuda()) for o, e in lists]
    A, B, I, ov = P.merge_lists(cams, dev)
    torch.cuda.synchronize()
    ref = oracle_mod.merge_lists([(o, e.astype(np.float64)) for o, e in lists], cams.npix,
                                 background=cam.background)
    assert ov == ref["overlaps"] and (ov == 0 if nlists == 1 else ov > 0)
    for nm, x in (("A", A), ("B", B), ("I", I)):
        err = rel_err(x.cpu().numpy(), ref[nm])
        assert err <= PIX_TOL, (nm, err)


def test_merge_rejects_bad_list_counts():
    torch = _torch()
    import paper_1809_01334_amd as P
    from paper_1809_01334_amd import _lib as L

    cam = synth.random_perspective_camera(np.random.default_rng(45), 8, 8)
    cams = P.rc_camera_prepare(cam.raw()[None, :], torch.device("cuda:0"))
    off = torch.zeros(cams.npix + 1, dtype=torch.int64, device="cuda:0")
    ent = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    with pytest.raises(ValueError):
        P.merge_lists(cams, [(off, ent)] * (L.RC_MAXLISTS + 1))
    A, B, I, ov = P.merge_lists(cams, [(off, ent)])
    assert ov == 0 and float(A.min()) == 1.0 and float(B.abs().max()) == 0.0


@pytest.mark.timeout(600)
def test_headline_workload_in_eight_shares(oracle_mod):
    """The full-size adaptive workload (1024^2) cut into 8 equal leaf ranges, as bench.py
    times it: the merged image against the full render on every pixel and against the
    oracle on 3000 sampled pixels; one share's lists against the oracle's on every pixel."""
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.config_scene(2)
    cam = scene.cameras[0]
    N = scene.forest.nleaves
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4)
    r.forward()
    shares = synth.split_shares(scene.forest, scene.fields, [N * k // 8 for k in range(1, 8)])
    lists, rs = [], []
    for i, (f, fl) in enumerate(shares):
        print(f"[case] headline share {i}: {f.nleaves} leaves", flush=True)
        ri = P.Renderer(f, fl, scene.cameras, "rk4", 4)
        lists.append(ri.forward_lists())
        rs.append(ri)
    A, B, I, ov = P.merge_lists(r.cams, lists)
    torch.cuda.synchronize()
    assert ov == 0
    for nm, x, y in (("A", A, r.A), ("B", B, r.B), ("I", I, r.I)):
        err = rel_err(x.cpu().numpy(), y.cpu().numpy())
        assert err <= PIX_TOL, ("full render", nm, err)
    pix = np.sort(np.random.default_rng(46).choice(cam.npix, 3000, replace=False))
    ref = oracle_mod.render(scene.forest, scene.fields, cam, "rk4", 4, pixels=pix)
    for nm, x in (("A", A), ("B", B), ("I", I)):
        err = rel_err(x.cpu().numpy()[pix], ref[nm])
        assert err <= PIX_TOL, ("oracle", nm, err)
    f, fl = shares[3]
    print(f"[case] headline share 3 lists against the oracle", flush=True)
    assert _check_lists(rs[3], *lists[3], scene, f, fl, oracle_mod) > 0
