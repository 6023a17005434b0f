"""GPU parity at the full sizes of the batched and the adjoint workloads.

* 64 cameras of resolutions from {256, 512, 1024, 2048}^2 on the 839959-leaf adaptive
  forest, rendered in one launch sequence: the chunk tables (written from the ranges at
  this size) against a search of the offsets, sampled pixels of four views against the
  oracle (1e-5), and two views bit for bit against rendering them alone.
* The same 64 views in the benchmark's launch configuration (tuning cache, one HIP graph
  replayed): bit for bit the default configuration's images.  The 1024^2 view likewise, with
  its forward + adjoint graph against an eager backward (bit for bit) and the oracle (1e-4).
* The 512^2 adjoint workload (785604 leaves, background 0.5): the loss
  L = sum (I - I_target)^2 over 2000 sampled pixels, dL/dI taken from the oracle's images
  and handed to both adjoints; the gradients with respect to all per-corner coefficients
  within 1e-4.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import GRAD_TOL, PIX_TOL, _check_child_desc, _check_chunk_tables, _torch, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_batched_64_views_full_size(oracle_mod):
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.config_scene(2)
    cams = synth.config4_cameras()
    print(f"[case] 64 views, {sum(c.npix for c in cams)} pixels, N={scene.forest.nleaves}", flush=True)
    rb = P.Renderer(scene.forest, scene.fields, cams, "rk4", 4)
    A, B, I = (t.clone() for t in rb.forward())
    torch.cuda.synchronize()
    # past 2^22 visible pairs and slots the chunk tables are written from the ranges: same tables as a search
    c = rb.vf.read_counts()
    assert c["nvis"] > 1 << 22 and rb.nslots > 1 << 22
    _check_chunk_tables(rb, rb.vf.cand_offset[:c["nvis"] + 1].cpu().numpy(), c)
    _check_child_desc(rb, sample=1 << 20)
    rng = np.random.default_rng(44)
    sizes = [c.w for c in cams]
    views = sorted({sizes.index(s) for s in set(sizes)})[:4]
    for k in views:
        cam = cams[k]
        pix = np.sort(rng.choice(cam.npix, 1000, replace=False))
        ref = oracle_mod.render(scene.forest, scene.fields, cam, "rk4", 4, pixels=pix)
        lo = rb.cams.img_off[k]
        for nm, x, y in (("A", A, ref["A"]), ("B", B, ref["B"]), ("I", I, ref["I"])):
            got = x[lo:lo + cam.npix].cpu().numpy()[pix]
            e = rel_err(got, y)
            assert e <= PIX_TOL, (k, cam.w, nm, e)
    for k in views[:2]:
        rs = P.Renderer(rb.forest, rb.fields, [cams[k]], "rk4", 4, index=rb.index)
        _, _, Is = rs.forward()
        sl = slice(rb.cams.img_off[k], rb.cams.img_off[k + 1])
        assert torch.equal(Is, I[sl]), k


@pytest.mark.timeout(600)
def test_batched_64_views_bench_configuration(oracle_mod):
    """The 64 views as the benchmark times them: launch shapes and skipped levels from the
    workload's entry in the package's tuning cache, the forward captured in one HIP graph and
    replayed.  A, B and I of every replay equal, bit for bit, those of an eager forward with
    the default launch shapes and every level written, and sampled pixels of the largest view
    match the oracle."""
    torch = _torch()
    import json
    import os

    import paper_1809_01334_amd as P
    from paper_1809_01334_amd import _lib as L
    from paper_1809_01334_amd.tune import signature

    scene = synth.config_scene(2)
    cams = synth.config4_cameras()
    r = P.Renderer(scene.forest, scene.fields, cams, "rk4", 4)
    A0, B0, I0 = (t.clone() for t in r.forward())
    cache = os.path.join(os.path.dirname(P.__file__), "tuning.json")
    sig = signature(r)
    known = json.load(open(cache))
    assert sig in known, f"no tuning cache entry for {sig}"
    tuned = known[sig]["tuning"]
    print(f"[case] 64 views in the tuned configuration {tuned}, one HIP graph", flush=True)
    assert tuned["fold_skip"] != 0  # the walk of skipped levels runs at full size
    r.tuning = L.RcTuning(**tuned)
    r.capture()
    for rep in range(3):
        A, B, I = r.replay()
        torch.cuda.synchronize()
        assert torch.equal(A, A0) and torch.equal(B, B0) and torch.equal(I, I0), rep
        r.prune()  # eager work between the replays
        torch.cuda.synchronize()
    k = max(range(len(cams)), key=lambda i: cams[i].npix)
    cam = cams[k]
    pix = np.sort(np.random.default_rng(45).choice(cam.npix, 1000, replace=False))
    ref = oracle_mod.render(scene.forest, scene.fields, cam, "rk4", 4, pixels=pix)
    lo = r.cams.img_off[k]
    got = I[lo:lo + cam.npix].cpu().numpy()[pix]
    assert rel_err(got, ref["I"]) <= PIX_TOL


@pytest.mark.timeout(600)
def test_single_view_bench_configuration(oracle_mod):
    """The 1024^2 view as the benchmark times it: the tuning cache's launch shapes, skipped
    levels and leaf-adjoint grid; the forward, and the forward + adjoint, each captured in one
    HIP graph and replayed.  The forward's replays equal an eager forward with the default
    launch shapes bit for bit; the captured gradients equal an eager backward on the same grid
    bit for bit and match the oracle's gradient of a loss on 2000 sampled pixels."""
    torch = _torch()
    import json
    import os

    import paper_1809_01334_amd as P
    from paper_1809_01334_amd import _lib as L
    from paper_1809_01334_amd.tune import signature

    scene = synth.config_scene(2)
    cam = scene.cameras[0]
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4)
    A0, B0, I0 = (t.clone() for t in r.forward())
    known = json.load(open(os.path.join(os.path.dirname(P.__file__), "tuning.json")))
    sig = signature(r)
    assert sig in known, f"no tuning cache entry for {sig}"
    tuned = known[sig]["tuning"]
    print(f"[case] one 1024^2 view in the tuned configuration {tuned}", flush=True)
    r.tuning = L.RcTuning(**tuned)
    r.capture()
    for rep in range(2):
        A, B, I = r.replay()
        torch.cuda.synchronize()
        assert torch.equal(A, A0) and torch.equal(B, B0) and torch.equal(I, I0), rep
    pix = np.sort(np.random.default_rng(46).choice(cam.npix, 2000, replace=False))
    go = np.random.default_rng(47).standard_normal(2000).astype(np.float32)
    g = torch.zeros(r.cams.npix, dtype=torch.float32, device=r.device)
    g[torch.from_numpy(pix).to(r.device)] = torch.from_numpy(go).to(r.device)
    r.forward()
    dk, de = (t.clone() for t in r.backward(g))
    torch.cuda.synchronize()
    r.capture(backward=True, dLdI=g)
    for rep in range(2):
        r.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.g_dk, dk) and torch.equal(r.g_de, de), rep
    gk, ge = oracle_mod.grad(scene.forest, scene.fields, cam, go.astype(np.float64), "rk4", 4, pixels=pix)
    assert np.abs(gk).max() > 0 and np.abs(ge).max() > 0
    ek = rel_err(dk.cpu().numpy().T, gk)
    ee = rel_err(de.cpu().numpy().T, ge)
    assert ek <= GRAD_TOL and ee <= GRAD_TOL, (ek, ee)


@pytest.mark.timeout(600)
def test_adjoint_workload_full_size_sampled_loss(oracle_mod):
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.config_scene(5)
    cam = scene.cameras[0]
    tf = scene.extra["target_fields"]
    print(f"[case] adjoint workload N={scene.forest.nleaves} {cam.w}x{cam.h}", flush=True)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps)
    r.forward()
    pix = np.sort(np.random.default_rng(55).choice(cam.npix, 2000, replace=False))
    # dL/dI from the oracle's own images: I and I_target differ by a small
    # perturbation, so the difference is taken in FP64 once and handed to both
    # adjoints (the GPU's input may come from the oracle, never the reverse)
    ref = oracle_mod.render(scene.forest, scene.fields, cam, scene.method, scene.substeps, pixels=pix)
    reft = oracle_mod.render(scene.forest, tf, cam, scene.method, scene.substeps, pixels=pix)
    go = 2.0 * (ref["I"] - reft["I"])
    g = torch.zeros(r.cams.npix, dtype=torch.float32, device=r.device)
    g[torch.from_numpy(pix).to(r.device)] = torch.from_numpy(go.astype(np.float32)).to(r.device)
    dk, de = r.backward(g.contiguous())
    torch.cuda.synchronize()
    gk, ge = oracle_mod.grad(scene.forest, scene.fields, cam, go.astype(np.float32).astype(np.float64),
                             scene.method, scene.substeps, pixels=pix)
    assert np.abs(gk).max() > 0 and np.abs(ge).max() > 0
    ek = rel_err(dk.cpu().numpy().T, gk)
    ee = rel_err(de.cpu().numpy().T, ge)
    assert ek <= GRAD_TOL and ee <= GRAD_TOL, (ek, ee)


@pytest.mark.timeout(900)
def test_adjoint_workload_end_to_end(oracle_mod):
    """The 512^2 adjoint workload end to end, each side differentiating its own images:
    L = sum over the whole view of (I - I_target)^2, I and I_target rendered in FP32 on the
    GPU through the autograd wrapper (dL/dI = 2 (I - I_target) formed by torch in FP32) and
    in FP64 by the oracle.

    The GPU's dL/dI carries the FP32 error of both images.  With both images within the
    pixel tolerance, |dI_p| <= PIX_TOL max(|I_p|, 1e-3 max|I|) (checked first), the error
    of dL/dI at p is at most e_p = 2 PIX_TOL (max(|I_p|, f) + max(|I*_p|, f*)), and it moves
    the gradient of coefficient theta by at most sum_p e_p |dI_p/dtheta| (the oracle's
    weighted absolute sensitivities).  The tolerance per coefficient is that bound plus
    the adjoint's own GRAD_TOL max(|g*|, 1e-3 max|g*|), the bar of the adjoint-only test."""
    torch = _torch()
    import paper_1809_01334_amd as P

    scene = synth.config_scene(5)
    cam = scene.cameras[0]
    tf = scene.extra["target_fields"]
    print(f"[case] adjoint workload end to end N={scene.forest.nleaves} {cam.w}x{cam.h}", flush=True)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps)
    rt = P.Renderer(r.forest, P.DeviceFields.from_synth(tf, r.device), scene.cameras, scene.method,
                    scene.substeps, index=r.index)
    kap = r.fields.kappa.clone().requires_grad_(True)
    eps = r.fields.eps.clone().requires_grad_(True)
    I = P.render(kap, eps, r)
    It = P.render(rt.fields.kappa, rt.fields.eps, rt)
    loss = ((I - It) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = oracle_mod.render(scene.forest, scene.fields, cam, scene.method, scene.substeps)
    reft = oracle_mod.render(scene.forest, tf, cam, scene.method, scene.substeps)
    Ig, Itg = I.detach().cpu().numpy(), It.detach().cpu().numpy()
    assert rel_err(Ig, ref["I"]) <= PIX_TOL and rel_err(Itg, reft["I"]) <= PIX_TOL
    go = 2.0 * (ref["I"] - reft["I"])
    gk, ge = oracle_mod.grad(scene.forest, scene.fields, cam, go, scene.method, scene.substeps)

    def floored(x):
        return np.maximum(np.abs(x), 1e-3 * np.abs(x).max())

    e = 2.0 * PIX_TOL * (floored(ref["I"]) + floored(reft["I"]))
    ak, ae = oracle_mod.grad_abs(scene.forest, scene.fields, cam, e, scene.method, scene.substeps)
    dk = kap.grad.cpu().numpy().T
    de = eps.grad.cpu().numpy().T
    worst = []
    for nm, got, want, bound in (("kappa", dk, gk, ak), ("eps", de, ge, ae)):
        tol = GRAD_TOL * floored(want) + bound
        err = np.abs(got - want)
        worst.append((nm, float((err / tol).max()), rel_err(got, want)))
        assert np.all(err <= tol), (nm, float((err / tol).max()))
    print(f"[measured] end-to-end gradient error / tolerance, and the plain relative error: {worst}", flush=True)
