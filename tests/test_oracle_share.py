"""Pins of the oracle's share compositing (Sec. 3.3 coarsening of one process's
share to its maximal subtrees, Sec. 3.5 per-pixel lists, Sec. 2.5 cutting and
averaging overlapping segments).

Checked against independent definitions: maximal subtrees by brute-force volume
coverage of the share's leaves, the merged lists of a partition against the
full-forest image, and closed forms of a constant medium for overlapping and
duplicated entries.
"""

import math

import numpy as np

import synth

Q = synth.QMAX


def _volumes(forest):
    return np.ldexp(1.0, -3 * forest.level.astype(np.int64))


def test_units_are_the_maximal_covered_subtrees(oracle_mod):
    O = oracle_mod
    sc = synth.small_scene(31, lmin=2, lmax=5, w=16, h=16)
    f = sc.forest
    rng = np.random.default_rng(31)
    for cuts in ([f.nleaves // 3, 2 * f.nleaves // 3], sorted(rng.choice(np.arange(1, f.nleaves), 4, replace=False))):
        for sf, _ in synth.split_shares(f, sc.fields, cuts):
            ul, ux, uy, uz = O.share_units(sf)
            keys = synth.morton_keys(sf.x, sf.y, sf.z)
            vol = _volumes(sf)
            assert math.isclose(np.ldexp(1.0, -3 * ul.astype(np.int64)).sum(), vol.sum(), rel_tol=1e-12)
            for l, x, y, z in zip(ul, ux, uy, uz):
                # the unit is covered exactly by the share's leaves inside it
                span = 1 << (3 * (Q - int(l)))
                k0 = int(synth.morton_keys(np.array([x]), np.array([y]), np.array([z]))[0])
                inside = (keys >= k0) & (keys < k0 + span)
                assert math.isclose(vol[inside].sum(), 8.0 ** -int(l), rel_tol=1e-12)
                # its parent is not (maximality), unless it is the root
                if l > 0:
                    pspan = span * 8
                    pk0 = k0 - k0 % pspan
                    pin = (keys >= pk0) & (keys < pk0 + pspan)
                    assert vol[pin].sum() < 8.0 ** -(int(l) - 1) * (1 - 1e-12)


def test_merged_share_lists_equal_the_full_image(oracle_mod):
    O = oracle_mod
    sc = synth.small_scene(32, w=48, h=40, background=0.4)
    cam = sc.cameras[0]
    full = O.render(sc.forest, sc.fields, cam, "rk4", 4)
    cuts = [sc.forest.nleaves // 4, sc.forest.nleaves // 2 + 7, 3 * sc.forest.nleaves // 4]
    lists = [O.share_lists(f, fl, cam, "rk4", 4) for f, fl in synth.split_shares(sc.forest, sc.fields, cuts)]
    m = O.merge_lists(lists, cam.npix, background=cam.background)
    assert m["overlaps"] == 0
    for k in ("A", "B", "I"):
        np.testing.assert_allclose(m[k], full[k], rtol=1e-12, atol=1e-14)
    # one share holding the whole forest is one unit, the root: one entry per hit pixel
    off, ent = O.share_lists(sc.forest, sc.fields, cam, "rk4", 4)
    assert np.diff(off).max() == 1
    np.testing.assert_allclose(ent[:, 3], full["B"][np.diff(off) == 1], rtol=1e-12)


def test_cut_and_average_of_overlapping_segments(oracle_mod):
    """A constant medium over [0, 2] and over [1, 3] merge into the medium over [0, 3];
    a duplicated entry averages to itself; touching entries fold plainly."""
    O = oracle_mod
    beta, gamma = 0.7, 0.3

    def medium(a, b):
        A = math.exp(-beta * (b - a))
        return [a, b, A, gamma / beta * (1 - A)]

    ab, ov = O.merge_pixel([medium(0, 2), medium(1, 3)])
    ref = medium(0, 3)
    assert ov == 1 and math.isclose(ab[0], ref[2], rel_tol=1e-13) and math.isclose(ab[1], ref[3], rel_tol=1e-13)
    ab, ov = O.merge_pixel([medium(0.5, 1.5), medium(0.5, 1.5)])
    assert ov == 1 and math.isclose(ab[0], medium(0.5, 1.5)[2], rel_tol=1e-13)
    ab, ov = O.merge_pixel([medium(0, 1), medium(1, 2.5), medium(2.5, 3)])
    assert ov == 0 and math.isclose(ab[0], ref[2], rel_tol=1e-13) and math.isclose(ab[1], ref[3], rel_tol=1e-13)
    # one segment nested inside a longer one
    ab, ov = O.merge_pixel([medium(0, 3), medium(1, 2)])
    assert ov == 1 and math.isclose(ab[0], ref[2], rel_tol=1e-13) and math.isclose(ab[1], ref[3], rel_tol=1e-13)


def test_merge_of_more_than_two_overlapping_entries(oracle_mod):
    """Where several entries cover a depth, the average runs over all of them: three
    copies of one medium on overlapping intervals give the medium over their union;
    three different media on one interval give the geometric mean of the A and the
    arithmetic mean of the B; a zero-length opaque entry inside a medium is folded
    whole at its depth."""
    O = oracle_mod

    def medium(a, b, beta=0.7, gamma=0.3):
        A = math.exp(-beta * (b - a))
        return [a, b, A, gamma / beta * (1 - A)]

    ab, ov = O.merge_pixel([medium(0, 2), medium(1, 3), medium(1.5, 2.5)])
    ref = medium(0, 3)
    assert ov == 2
    assert math.isclose(ab[0], ref[2], rel_tol=1e-13) and math.isclose(ab[1], ref[3], rel_tol=1e-13)
    media = [medium(1, 2, 0.5, 0.2), medium(1, 2, 1.5, 0.9), medium(1, 2, 3.0, 0.1)]
    ab, ov = O.merge_pixel(media)
    assert ov == 2
    assert math.isclose(ab[0], (media[0][2] * media[1][2] * media[2][2]) ** (1 / 3), rel_tol=1e-13)
    assert math.isclose(ab[1], sum(m[3] for m in media) / 3, rel_tol=1e-13)
    Is = 0.8
    ab, ov = O.merge_pixel([medium(0, 2), [1.0, 1.0, 0.0, Is]])
    near = medium(0, 1)
    assert ov == 0 and ab[0] == 0.0 and math.isclose(ab[1], near[3] + near[2] * Is, rel_tol=1e-13)
