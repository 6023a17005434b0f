"""Compositing with skipped levels (rc_tuning.fold_skip): the pass above a run
of skipped levels folds them itself, in the association of the level passes
(a node's value is the fold of its children's values, nearest first, from the
identity; Sec. 2.4, Sec. 3.3), so the images are bit for bit those of the
plain coarsening, and so are the node records of the levels still written.
The adjoint after such a forward restores the records it reads."""

import numpy as np
import pytest

import synth
from test_gpu_parity import _torch, many_small_views

pytestmark = pytest.mark.gpu

MASKS = (0b10, 0b100, 0b110, 0b1000, 0b1010, 0b1100, 0b10100, 0b101010, 0b11011010)


def _levels_records(r):
    """Node records per written level: {level: float32 array} from rec_node and the slot table."""
    torch = _torch()
    torch.cuda.synchronize()
    off = r.vf.node_offset[:r.nslots + 1].cpu().numpy()
    rec = r.rec_node[:2 * int(off[-1])].cpu().numpy().reshape(-1, 2)
    lb = r.index.level_begin()
    ncams = r.cams.ncams
    out, s = {}, 0
    for l in range(1, r.index.maxlevel):
        n = ncams * (lb[l + 1] - lb[l])
        out[l] = rec[off[s]:off[s + n]]
        s += n
    return out


def _check_masks(r, render=True):
    torch = _torch()
    import paper_1809_01334_amd as P

    r.tuning.fold_skip = 0
    r.forward()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (r.A, r.B, r.I)]
    ref_levels = _levels_records(r)
    for m in MASKS:
        r.tuning.fold_skip = m
        r.composite()
        torch.cuda.synchronize()
        for a, b in zip((r.A, r.B, r.I), ref):
            assert torch.equal(a, b), m
        got = _levels_records(r)
        for l, v in ref_levels.items():
            if not (m >> l) & 1:
                assert np.array_equal(got[l].view(np.uint32), v.view(np.uint32)), (m, l)
        if render:
            r.render_step()
            torch.cuda.synchronize()
            for a, b in zip((r.A, r.B, r.I), ref):
                assert torch.equal(a, b), ("render", m)
    r.tuning.fold_skip = 0
    assert r.index.maxlevel >= 4


def test_adaptive_scene_three_cameras():
    import paper_1809_01334_amd as P

    sc = synth.small_scene(4, lmin=1, lmax=6, ngauss=4, w=96, h=72)
    rng = np.random.default_rng(9)
    cams = [sc.cameras[0], synth.random_perspective_camera(rng, 57, 131, background=0.3),
            synth.random_perspective_camera(rng, 200, 40)]
    print(f"[case] small scene N={sc.forest.nleaves}, 3 cameras", flush=True)
    _check_masks(P.Renderer(sc.forest, sc.fields, cams, "rk4", 4))


def test_tiny_views_mixed_in_every_wave():
    """300 views of 1..9 pixels: waves of the walking passes hold several cameras and nodes."""
    import paper_1809_01334_amd as P

    sc = many_small_views(303, 300)
    print(f"[case] 300 tiny views N={sc.forest.nleaves}", flush=True)
    _check_masks(P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 2))


def test_full_size_view_and_constant_fields():
    import paper_1809_01334_amd as P

    sc = synth.config_scene(2)
    print(f"[case] config 2, N={sc.forest.nleaves}", flush=True)
    _check_masks(P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4), render=False)


def test_run_limit_and_ignored_bits():
    torch = _torch()
    import paper_1809_01334_amd as P

    sc = synth.small_scene(5, lmin=1, lmax=6, w=48, h=40)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4)
    r.forward()
    ref = r.I.clone()
    r.tuning.fold_skip = 0b1110  # three consecutive levels
    with pytest.raises(P.RcError) as e:
        r.composite()
    assert e.value.status == P._lib.RC_EINVAL
    # bit 0 (the root) and levels at or below the deepest internal level are ignored
    r.tuning.fold_skip = 1 | (1 << r.index.maxlevel) | (1 << 30)
    r.composite()
    torch.cuda.synchronize()
    assert torch.equal(r.I, ref)


def test_adjoint_after_a_skipping_forward():
    """backward() after a fold_skip forward rewrites the node records first: gradients bit for bit those after a
    plain forward; the graph of forward + backward keeps every record."""
    torch = _torch()
    import paper_1809_01334_amd as P

    sc = synth.small_scene(6, lmin=1, lmax=5, w=64, h=48, background=0.2)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4)
    g = torch.linspace(-1.0, 1.0, r.cams.npix, device=r.device)
    r.forward()
    dk0, de0 = (t.clone() for t in r.backward(g))
    r.tuning.fold_skip = 0b1010
    r.forward()
    assert not r.node_records
    dk1, de1 = r.backward(g)
    assert torch.equal(dk0, dk1) and torch.equal(de0, de1)
    kap = r.fields.kappa.clone().requires_grad_(True)
    eps = r.fields.eps.clone().requires_grad_(True)
    I = P.render(kap, eps, r)
    (I * g).sum().backward()
    assert torch.equal(kap.grad, dk0) and torch.equal(eps.grad, de0)
    r.capture(backward=True, dLdI=g)
    for _ in range(2):
        r.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.g_dk, dk0) and torch.equal(r.g_de, de0)
