"""rc_render, the forward with the intra-tile fold (leaf segments folded into
their parents' records in registers and LDS), against rc_segments followed by
rc_composite: images and node records bit for bit on the same seeded inputs,
on every field kind, integrator and substep count it fuses, on ragged and
mixed camera sets, shares with absent children and the full-size workloads;
the adjoint after it; graph replays.  The images themselves are checked
against the oracle by the parity tests, which render through rc_render."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _two_call(r):
    torch = _torch()
    r.prune()
    r.segments()
    r.composite()
    torch.cuda.synchronize()
    nrec = r.counts["nrec"]
    return [t.clone() for t in (r.A, r.B, r.I)] + [r.rec_node[:2 * nrec].clone()]


def _fused(r):
    torch = _torch()
    # poison every output, so that anything rc_render leaves unwritten shows
    for t in (r.A, r.B, r.I, r.rec_node):
        t.fill_(float("nan"))
    r.prune()
    r.render_step()
    torch.cuda.synchronize()
    nrec = r.counts["nrec"]
    return [r.A, r.B, r.I, r.rec_node[:2 * nrec]]


def _check(scene, method=None, substeps=None, expect_fused=True, **kw):
    torch = _torch()
    import paper_1809_01334_amd as P

    method = method or scene.method
    substeps = substeps or scene.substeps
    print(f"[case] {scene.name}: N={scene.forest.nleaves} cams={len(scene.cameras)} {method}x{substeps}", flush=True)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, method, substeps, **kw)
    assert r.fused == expect_fused
    want = _two_call(r)
    got = _fused(r)
    for nm, a, b in zip(("A", "B", "I", "rec_node"), got, want):
        assert torch.equal(a, b), (scene.name, nm, float((a - b).abs().max()))
    return r


@pytest.mark.parametrize("seed,w,h,ncams,substeps", [(0, 96, 72, 1, 4), (1, 101, 77, 2, 4), (2, 130, 47, 3, 1),
                                                     (3, 64, 64, 1, 2), (4, 55, 41, 2, 8), (5, 73, 59, 1, 3)])
def test_trilinear_rk4(seed, w, h, ncams, substeps):
    scene = synth.small_scene(60 + seed, w=w, h=h, ncams=ncams, background=0.3 * (seed % 2))
    _check(scene, "rk4", substeps)


@pytest.mark.parametrize("method,substeps", [("analytic", 1), ("rk4", 4), ("rk4", 5)])
def test_constant_fields(method, substeps):
    scene = synth.constant_variant(synth.small_scene(70, w=88, h=66, ncams=2, background=0.4))
    _check(scene, method, substeps)


def test_equilibrium_fields():
    base = synth.small_scene(71, w=80, h=60)
    rng = np.random.default_rng(71)
    N = base.forest.nleaves
    scene = synth.Scene("equilibrium", base.forest,
                        synth.equilibrium_fields(rng.uniform(0.1, 2.0, N), rng.uniform(0.0, 1.0, N)),
                        base.cameras, "analytic", 1)
    _check(scene)


def test_orthographic_and_mixed_small_views():
    """300 views of 1..9 x 1..9 pixels alternating perspective and orthographic: windows of records and
    items straddle cameras and camera modes."""
    rng = np.random.default_rng(7070)
    scene = synth.small_scene(72, lmin=2, lmax=4)
    cams = []
    for k in range(300):
        w, h = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        if k % 2 == 0:
            cams.append(synth.random_perspective_camera(rng, w, h, background=float(rng.uniform(0, 0.5))))
        else:
            cams.append(synth.orthographic_axis_camera(int(rng.integers(3)), int(rng.choice([-1, 1])), w=w, h=h,
                                                       ell=1.4 / max(w, h), background=float(rng.uniform(0, 0.5))))
    scene.cameras = cams
    _check(scene)
    scene.cameras = [synth.orthographic_axis_camera(a, s, w=70, h=50, ell=1.4 / 70) for a, s in ((0, 1), (2, -1))]
    _check(scene)


def test_shallow_and_degenerate_forests():
    """A one-level forest (the root's children are leaves: the root pass integrates them), a two-level
    forest, one camera seeing nothing, a 1x1 image and near-plane clipping; a forest of one leaf falls back
    to the two calls."""
    for lv in (1, 2):
        forest = synth.uniform_forest(lv)
        N = forest.nleaves
        rng = np.random.default_rng(80 + lv)
        cams = [synth.random_perspective_camera(rng, 40, 30), synth.random_perspective_camera(rng, 1, 1, dist=1.2),
                synth.perspective_camera([0.5, 0.5, 3.0], [0.5, 0.5, 9.0], [0, 1, 0], 1.0, 42, 20, 10, 5.0),
                synth.perspective_camera([0.5, 0.45, 1.3], [0.5, 0.5, 0.0], [0, 1, 0], 0.6, 70, 33, 31, 2.0)]
        for fields, method in ((synth.constant_fields(rng.uniform(0.1, 2, N), rng.uniform(0, 1, N)), "analytic"),
                               (synth.trilinear_fields_from_gaussians(forest, rng.uniform(0, 1, (3, 3)),
                                                                      rng.uniform(0.1, 0.3, 3)), "rk4")):
            _check(synth.Scene(f"uniform{N}", forest, fields, cams, method, 4))
    forest = synth.uniform_forest(0)
    fields = synth.constant_fields(np.array([1.3]), np.array([0.6]))
    cams = [synth.random_perspective_camera(np.random.default_rng(9), 30, 20)]
    _check(synth.Scene("one_leaf", forest, fields, cams, "analytic", 1), expect_fused=False)


def test_shares_with_absent_children():
    """Curve-order leaf ranges of a forest: their node tables hold absent children."""
    scene = synth.small_scene(73, w=90, h=70, ncams=2)
    N = scene.forest.nleaves
    for f, fl in synth.split_shares(scene.forest, scene.fields, [N // 3, N // 3 + 17, (2 * N) // 3]):
        _check(synth.Scene("share", f, fl, scene.cameras, "rk4", 4))


def test_not_fused_paths_match_two_calls():
    """Several channels and the integrator variants run the two calls inside rc_render."""
    scene = synth.small_scene(74, w=60, h=40)
    _check(scene, "gauss2", 2, expect_fused=False)
    _check(scene, "rk4", 2, expect_fused=False, c_rk=0.3)
    f = scene.fields
    two = synth.stack_channels([f, synth.Fields(f.kind, (f.kappa * 0.5).astype(np.float32), f.eps)])
    _check(synth.Scene("two_channels", scene.forest, two, scene.cameras, "rk4", 4), expect_fused=False)


def test_adjoint_after_fused_forward():
    """The adjoint after rc_render (which leaves no leaf records: the renderer runs rc_segments first) equals
    the adjoint after the two calls, bit for bit."""
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.small_scene(75, w=70, h=50, background=0.5)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4)
    g = torch.rand(r.cams.npix, generator=torch.Generator().manual_seed(75)).cuda()
    r.forward(leaf_records=True)
    dk0, de0 = (t.clone() for t in r.backward(g))
    r.forward(leaf_records=False)
    assert not r.leaf_records
    dk1, de1 = r.backward(g)
    torch.cuda.synchronize()
    assert torch.equal(dk0, dk1) and torch.equal(de0, de1)


def test_graph_replays_of_fused_forward():
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.small_scene(76, w=100, h=80, ncams=2, background=0.2)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4, use_render=True)
    want = [t.clone() for t in r.forward()]
    r.capture()
    for _ in range(4):
        r.forward(leaf_records=True)  # eager work between replays
        for t in (r.A, r.B, r.I):
            t.fill_(0.0)
        torch.cuda.synchronize()
        r.replay()
        torch.cuda.synchronize()
        for a, b in zip((r.A, r.B, r.I), want):
            assert torch.equal(a, b)


@pytest.mark.timeout(600)
def test_full_size_workloads_bitwise():
    """The 1024^2 adaptive workload (RK4 x 4, trilinear), the same view with one (kappa, eps) per leaf in
    closed form, and the 64 views of uneven resolution: rc_render against the two calls, bit for bit."""
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.config_scene(2)
    r = _check(scene)
    _check(synth.constant_variant(scene), "analytic", 1, index=r.index)
    cams = synth.config4_cameras()
    print(f"[case] 64 views, {sum(c.npix for c in cams)} pixels", flush=True)
    rb = P.Renderer(r.forest, r.fields, cams, "rk4", 4, index=r.index)
    want = _two_call(rb)
    got = _fused(rb)
    for nm, a, b in zip(("A", "B", "I", "rec_node"), got, want):
        assert torch.equal(a, b), nm


def test_fused_forward_against_the_oracle(oracle_mod):
    """rc_render's images against the FP64 oracle directly: workload 1 (closed form, orthographic) and an
    adaptive scene with three cameras and background (RK4 x 4)."""
    _torch()
    import paper_1809_01334_amd as P

    for scene in (synth.config_scene(1), synth.small_scene(77, w=90, h=70, ncams=3, background=0.3)):
        r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps, use_render=True)
        assert r.fused
        A, B, I = (t.cpu().numpy() for t in r.forward())
        assert not r.leaf_records
        for k, cam in enumerate(scene.cameras):
            ref = oracle_mod.render(scene.forest, scene.fields, cam, scene.method, scene.substeps)
            sl = slice(r.cams.img_off[k], r.cams.img_off[k + 1])
            for x, y in ((A[sl], ref["A"]), (B[sl], ref["B"]), (I[sl], ref["I"])):
                den = np.maximum(np.abs(y), 1e-3 * max(np.abs(y).max(), 1e-30))
                assert float((np.abs(x - y) / den).max()) <= 1e-5


def test_fused_forward_without_leaf_records():
    """rc_render with rec_leaf = NULL where it fuses (the leaf records are not needed): the same images and
    node records as with them, on a forest with leaves at several levels (fused and plain passes) and on a
    one-level forest (the root pass integrates the leaves)."""
    torch = _torch()
    import paper_1809_01334_amd as P

    for scene in (synth.small_scene(78, lmin=3, lmax=5, w=64, h=48, ncams=2),
                  synth.Scene("uniform8", synth.uniform_forest(1), synth.constant_fields(np.linspace(0.2, 1.5, 8),
                                                                                          np.linspace(0.1, 0.9, 8)),
                              [synth.random_perspective_camera(np.random.default_rng(78), 30, 20)], "analytic", 1)):
        r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps)
        assert r.fused
        want = _two_call(r)
        for t in (r.A, r.B, r.I, r.rec_node):
            t.fill_(float("nan"))
        r.prune()
        P.rc_render(r.forest, r.index, r.fields, r.cams, r.vf, r.method, r.substeps, None, r.rec_node, r.A, r.B, r.I)
        torch.cuda.synchronize()
        got = [r.A, r.B, r.I, r.rec_node[:2 * r.counts["nrec"]]]
        for a, b in zip(got, want):
            assert torch.equal(a, b)
