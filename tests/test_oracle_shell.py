"""Pins of the oracle's curved six-tree shell geometry (Sec. 2.1, smooth per-tree maps).

Checked against what the geometry fixes independently: the map/inverse round
trip, ray/sphere chords computed here with numpy, the constant-medium closed
form across the hollow core, conservativeness of the lenient boxes under an
independent projection, and brute-force marching.
"""

import math

import numpy as np

import synth


def _rays(cam):
    v = np.asarray(cam.v)
    n = np.linalg.norm(v)
    for j in range(cam.h):
        for i in range(cam.w):
            a, b = cam.ell * (i - (cam.w - 1) / 2), cam.ell * (j - (cam.h - 1) / 2)
            yield j * cam.w + i, cam.o, v + a * cam.t + b * cam.u, 1.0, cam.zfar / n


def _ball_chord(rho, r, R, smin, smax):
    A, B, C = r @ r, rho @ r, rho @ rho - R * R
    D = B * B - A * C
    if D <= 0:
        return None
    s1, s2 = (-B - math.sqrt(D)) / A, (-B + math.sqrt(D)) / A
    return max(s1, smin), min(s2, smax)


def _shell_length(rho, r, smin, smax, r0=synth.SHELL_R0, r1=synth.SHELL_R1):
    o = _ball_chord(rho, r, r1, smin, smax)
    if o is None or o[1] <= o[0]:
        return 0.0
    L = o[1] - o[0]
    i = _ball_chord(rho, r, r0, smin, smax)
    if i is not None:
        a, b = max(i[0], o[0]), min(i[1], o[1])
        if b > a:
            L -= b - a
    return L * np.linalg.norm(r)


def test_map_and_inverse_round_trip(oracle_mod):
    O = oracle_mod
    geom = synth.shell_params(4)
    rng = np.random.default_rng(3)
    for k in range(6):
        for _ in range(50):
            t = rng.uniform(0.001, 0.999, 3)
            x = O.shell_map(geom, k, t)
            np.testing.assert_allclose(x, synth.shell_map(k, t[None])[0], rtol=1e-13, atol=1e-14)
            np.testing.assert_allclose(O.shell_inverse(geom, k, x), t, rtol=0, atol=1e-12)
            assert synth.SHELL_R0 - 1e-12 <= np.linalg.norm(x) <= synth.SHELL_R1 + 1e-12


def test_tan_table_is_the_map_at_dyadic_parameters():
    geom = synth.shell_params(5)
    L = int(geom[2])
    tab = geom[3:]
    i = np.arange((1 << L) + 1)
    np.testing.assert_allclose(tab, np.tan(np.pi / 4 * (2 * i / (1 << L) - 1)), rtol=0, atol=2e-16)
    assert tab[0] == -1.0 and tab[-1] == 1.0 and tab[(1 << L) // 2] == 0.0


def test_shell_segments_tile_the_shell(oracle_mod):
    """kappa = 0, eps = 1: B is the ray's length inside the shell, hollow core excluded."""
    O = oracle_mod
    sc = synth.shell_scene(1, lmin=1, lmax=3, w=40, h=30, dist=2.2)
    N = sc.forest.nleaves
    fields = synth.Fields("trilinear", np.zeros((8, N), np.float32), np.ones((8, N), np.float32))
    cam = sc.cameras[0]
    r = O.render(sc.forest, fields, cam)
    assert r["overlaps"] == 0 and r["segments"] > 0
    for p, rho, rr, smin, smax in _rays(cam):
        L = _shell_length(rho, rr, smin, smax)
        assert abs(r["B"][p] - L) < 1e-10, (p, r["B"][p], L)


def test_constant_medium_across_the_hollow_core(oracle_mod):
    O = oracle_mod
    sc = synth.shell_scene(2, lmin=1, lmax=2, w=36, h=28, dist=2.5)
    N = sc.forest.nleaves
    kap, eps, bg = 1.7, 0.6, 0.3
    fields = synth.Fields("trilinear", np.full((8, N), kap, np.float32), np.full((8, N), eps, np.float32))
    cam = sc.cameras[0]
    cam.background = bg
    r = O.render(sc.forest, fields, cam)
    kf, ef = float(np.float32(kap)), float(np.float32(eps))
    for p, rho, rr, smin, smax in _rays(cam):
        L = _shell_length(rho, rr, smin, smax)
        A = math.exp(-kf * L)
        I = ef / kf * (1 - A) + A * bg
        assert abs(r["I"][p] - I) < 2e-5, (p, r["I"][p], I)


def test_lenient_boxes_are_conservative(oracle_mod):
    O = oracle_mod
    sc = synth.shell_scene(3, lmin=1, lmax=3, w=64, h=48, dist=2.6)
    cam = sc.cameras[0]
    f = sc.forest
    rect, _ = O.prune(f, cam.raw())
    tree = f.tree_of_leaf()
    rng = np.random.default_rng(5)
    v = np.asarray(cam.v)
    n = np.linalg.norm(v)
    for l in rng.choice(f.nleaves, 200, replace=False):
        lo = np.array([f.x[l], f.y[l], f.z[l]], np.float64) * 2.0 ** -synth.QMAX
        h = 2.0 ** -int(f.level[l])
        pts = synth.shell_map(int(tree[l]), lo + h * rng.uniform(0, 1, (400, 3)))
        d = pts - cam.o
        X, Y, Z = d @ cam.t, d @ cam.u, d @ (v / n)
        px = X / Z * n / cam.ell + (cam.w - 1) / 2
        py = Y / Z * n / cam.ell + (cam.h - 1) / 2
        i0, i1, j0, j1 = rect[0, l]
        ins = (px >= -0.5) & (px <= cam.w - 0.5) & (py >= -0.5) & (py <= cam.h - 0.5)
        if i0 > i1:
            # an empty rectangle: no sample point may project onto a pixel centre
            assert not np.any(ins & (np.abs(px - np.round(px)) < 1e-9) & (np.abs(py - np.round(py)) < 1e-9))
            continue
        assert np.all(px[ins] > i0 - 1) and np.all(px[ins] < i1 + 1)
        assert np.all(py[ins] > j0 - 1) and np.all(py[ins] < j1 + 1)


def test_at_most_two_intervals_and_two_occur(oracle_mod):
    O = oracle_mod
    sc = synth.shell_scene(4, lmin=1, lmax=2, w=48, h=40, dist=2.2)
    nseg, sio = O.shell_pairs(sc.forest, sc.cameras[0].raw())
    assert nseg.max() == 2 and nseg.min() == 0
    two = sio[nseg == 2]
    assert np.all(two[:, 1] > two[:, 0]) and np.all(two[:, 2] >= two[:, 1]) and np.all(two[:, 3] > two[:, 2])


def test_brute_force_marching_converges_on_the_shell(oracle_mod):
    O = oracle_mod
    sc = synth.shell_scene(5, lmin=1, lmax=2, ngauss=2, w=20, h=16)
    ref = O.render(sc.forest, sc.fields, sc.cameras[0])
    errs = [np.abs(O.march(sc.forest, sc.fields, sc.cameras[0], M=M)["I"] - ref["I"]).max() for M in (100, 400, 1600)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 5e-4, errs
