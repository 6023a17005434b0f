"""Several channels per call (the paper converts each RGB channel to its own
(A, B), Sec. 4.1): channel-major fields, records and images.

On the unit cube with the closed form or fixed-step RK4, one pairing serves
every channel; each channel must match a single-channel render of its own
fields to 1e-6 (a different kernel instantiation may round differently) and
the oracle to 1e-5.  Other paths (the shell, the integrator variants) take one
channel at a time and must match bit for bit.  The adjoint runs per channel.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import PIX_TOL, GRAD_TOL, _torch, rel_err

pytestmark = pytest.mark.gpu


def _render(scene_fields, scene, method, substeps, c_rk=0.0):
    import paper_1809_01334_amd as P

    r = P.Renderer(scene.forest, scene_fields, scene.cameras, method, substeps, c_rk=c_rk)
    r.forward()
    _torch().cuda.synchronize()
    return r


def _channels(rng, scene, nch, kind):
    N = scene.forest.nleaves
    out = []
    for _ in range(nch):
        if kind == "const":
            out.append(synth.constant_fields(rng.uniform(0.1, 3.0, N), rng.uniform(0.0, 1.0, N)))
        else:
            out.append(synth.Fields("trilinear", rng.uniform(0.1, 2.5, (8, N)).astype(np.float32),
                                    rng.uniform(0.0, 1.0, (8, N)).astype(np.float32)))
    return out


@pytest.mark.parametrize("kind,method,substeps", [("trilinear", "rk4", 4), ("const", "analytic", 1),
                                                  ("trilinear", "rk4", 2), ("const", "rk4", 4)])
def test_fused_channels_match_single_channel_renders(oracle_mod, kind, method, substeps):
    rng = np.random.default_rng(90 + substeps)
    scene = synth.small_scene(90, ncams=2, w=70, h=52, background=0.3)
    nch = 3 if kind == "trilinear" else 2
    chans = _channels(rng, scene, nch, kind)
    print(f"[case] {nch} channels {kind} {method} x{substeps}", flush=True)
    r = _render(synth.stack_channels(chans), scene, method, substeps)
    P_ = r.cams.npix
    for ch, fl in enumerate(chans):
        one = _render(fl, scene, method, substeps)
        for nm in ("A", "B", "I"):
            got = getattr(r, nm)[ch * P_:(ch + 1) * P_]
            ref = getattr(one, nm)
            e = rel_err(got.cpu().numpy(), ref.cpu().numpy())
            print(f"  channel {ch} {nm}: max rel diff to the single-channel render {e:.2e}", flush=True)
            assert e <= 1e-6, (ch, nm, e)
        I = r.I[ch * P_:(ch + 1) * P_].cpu().numpy()
        for k, cam in enumerate(scene.cameras):
            ref = oracle_mod.render(scene.forest, fl, cam, method, substeps)
            e = rel_err(I[r.cams.img_off[k]:r.cams.img_off[k + 1]], ref["I"])
            assert e <= PIX_TOL, (ch, k, e)


def _fused_vs_per_channel(r):
    """Images and node records of the fused rc_composite_channels against rc_composite per channel."""
    torch = _torch()
    r.composite()
    torch.cuda.synchronize()
    A, B, I = (t.clone() for t in (r.A, r.B, r.I))
    nodes = r.rec_node.clone()
    for t in (r.A, r.B, r.I, r.rec_node):
        t.fill_(-7.0)
    r.composite_per_channel()
    torch.cuda.synchronize()
    assert torch.equal(r.A, A) and torch.equal(r.B, B) and torch.equal(r.I, I)
    nrec, cap = r.vf.read_counts()["nrec"], r.vf.cap_rec
    for ch in range(r.fields.nch):
        sl = slice(ch * 2 * cap, ch * 2 * cap + 2 * nrec)
        assert torch.equal(r.rec_node[sl], nodes[sl]), ch


@pytest.mark.parametrize("nch", [2, 3])
def test_fused_composite_is_bitwise_per_channel(nch):
    """rc_composite_channels folds all channels in one pass: bit for bit rc_composite on each channel's blocks
    (three cameras, one of them straddled by waves; a forest of one leaf; a one-level forest)."""
    rng = np.random.default_rng(100 + nch)
    scene = synth.small_scene(100 + nch, ncams=3, w=67, h=49, background=0.4)
    print(f"[case] fused composite, {nch} channels, 3 cameras", flush=True)
    _fused_vs_per_channel(_render(synth.stack_channels(_channels(rng, scene, nch, "trilinear")), scene, "rk4", 4))
    for forest in (synth.uniform_forest(0), synth.uniform_forest(1)):
        N = forest.nleaves
        cams = [synth.random_perspective_camera(rng, 40, 30), synth.random_perspective_camera(rng, 23, 17)]
        sc = synth.Scene(f"uniform{N}", forest, synth.constant_fields(np.ones(N), np.ones(N)), cams, "analytic", 1)
        print(f"[case] fused composite, {nch} channels, {N} leaves", flush=True)
        _fused_vs_per_channel(_render(synth.stack_channels(_channels(rng, sc, nch, "const")), sc, "analytic", 1))


def test_fused_composite_many_small_views():
    """300 views of 1..9 x 1..9 pixels and three channels: the fused fold's per-lane descriptor path, bit for bit
    against rc_composite per channel."""
    from test_gpu_parity import many_small_views

    scene = many_small_views(307, 300)
    rng = np.random.default_rng(307)
    print("[case] fused composite, 3 channels, 300 small views", flush=True)
    _fused_vs_per_channel(_render(synth.stack_channels(_channels(rng, scene, 3, "trilinear")), scene, "rk4", 4))


@pytest.mark.parametrize("which", ["shell", "gauss2"])
def test_channel_loop_paths(oracle_mod, which):
    rng = np.random.default_rng(95)
    if which == "shell":
        scene = synth.shell_scene(9, lmin=1, lmax=3, w=64, h=48, dist=2.6)
        N = scene.forest.nleaves
        base = scene.fields
        chans = [base, synth.Fields("trilinear", (base.kappa * rng.uniform(0.5, 1.5)).astype(np.float32),
                                    (base.eps * rng.uniform(0.5, 1.5)).astype(np.float32))]
        method, sub = "rk4", 4
    else:
        scene = synth.small_scene(96, w=64, h=48)
        chans = _channels(rng, scene, 2, "trilinear")
        method, sub = "gauss2", 4
    print(f"[case] channel loop on {which}", flush=True)
    r = _render(synth.stack_channels(chans), scene, method, sub)
    P_ = r.cams.npix
    for ch, fl in enumerate(chans):
        one = _render(fl, scene, method, sub)
        assert bool((r.I[ch * P_:(ch + 1) * P_] == one.I).all()), ch


def test_adjoint_per_channel_and_autograd():
    torch = _torch()
    import paper_1809_01334_amd as P

    rng = np.random.default_rng(97)
    scene = synth.small_scene(97, w=60, h=44, background=0.2)
    chans = _channels(rng, scene, 3, "trilinear")
    print("[case] 3-channel adjoint", flush=True)
    r = _render(synth.stack_channels(chans), scene, "rk4", 4)
    P_ = r.cams.npix
    g = torch.from_numpy(rng.uniform(-1, 1, 3 * P_).astype(np.float32)).cuda()
    dk, de = r.backward(g)
    torch.cuda.synchronize()
    for ch, fl in enumerate(chans):
        one = _render(fl, scene, "rk4", 4)
        dk1, de1 = one.backward(g[ch * P_:(ch + 1) * P_].contiguous())
        torch.cuda.synchronize()
        assert rel_err(dk[ch].cpu().numpy(), dk1.cpu().numpy()) <= GRAD_TOL / 10, ch
        assert rel_err(de[ch].cpu().numpy(), de1.cpu().numpy()) <= GRAD_TOL / 10, ch
    # the autograd wrapper sees all channels at once
    kappa = r.fields.kappa.clone().requires_grad_(True)
    eps = r.fields.eps.clone().requires_grad_(True)
    I = P.render(kappa, eps, r)
    (I * g).sum().backward()
    assert torch.allclose(kappa.grad, dk, rtol=1e-5, atol=1e-7) and torch.allclose(eps.grad, de, rtol=1e-5, atol=1e-7)
