"""Seeded random combinations of the options, checked against the oracle.

Each case draws a small adaptive forest, one to three cameras of random sizes (perspective or orthographic,
random background), an integrator (closed form, RK4, Gauss or Simpson over 1 to 8 pieces, or the recursion),
and one or two channels.  Every channel's images are compared with the oracle's within 1e-5; where the
adjoint applies, the gradients of L = sum (I - I*)^2 over the first camera's pixels within 1e-4.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import GRAD_TOL, PIX_TOL, _torch, rel_err

pytestmark = pytest.mark.gpu


def _draw(seed):
    rng = np.random.default_rng([4242, seed])
    method = ["analytic", "rk4", "gauss2", "simpson", "recursion"][seed % 5]  # each four times over 20 seeds
    ortho = bool(rng.integers(2))
    scene = synth.small_scene(300 + seed, lmin=int(rng.integers(1, 3)), lmax=int(rng.integers(3, 6)), ortho=ortho,
                              w=int(rng.integers(20, 70)), h=int(rng.integers(20, 70)),
                              ncams=int(rng.integers(1, 4)), background=float(rng.uniform(0.0, 0.6)),
                              method="analytic" if method == "analytic" else "rk4")
    N = scene.forest.nleaves
    nch = int(rng.integers(1, 3))
    chans = []
    for _ in range(nch):
        if method == "analytic":
            chans.append(synth.constant_fields(rng.uniform(0.1, 3.0, N), rng.uniform(0.0, 1.0, N)))
        else:
            chans.append(synth.Fields("trilinear", rng.uniform(0.1, 2.5, (8, N)).astype(np.float32),
                                      rng.uniform(0.0, 1.0, (8, N)).astype(np.float32)))
    c_rk = 0.0
    if method == "analytic":
        meth, sub = "analytic", 1
    elif method == "recursion":
        meth, sub, c_rk = str(rng.choice(["rk4", "gauss2", "simpson"])), int(rng.choice([1, 2])), 0.05
    else:
        meth, sub = method, int(rng.choice([1, 2, 4, 8]))
    return scene, chans, meth, sub, c_rk


@pytest.mark.parametrize("seed", range(20))
def test_random_configuration(oracle_mod, seed):
    torch = _torch()
    import paper_1809_01334_amd as P

    scene, chans, meth, sub, c_rk = _draw(seed)
    print(f"[case] seed {seed}: N={scene.forest.nleaves} cams={[(c.w, c.h, c.ortho) for c in scene.cameras]} "
          f"{meth} x{sub} c_rk={c_rk} channels={len(chans)}", flush=True)
    fields = chans[0] if len(chans) == 1 else synth.stack_channels(chans)
    r = P.Renderer(scene.forest, fields, scene.cameras, meth, sub, c_rk=c_rk)
    _, _, I = r.forward()
    torch.cuda.synchronize()
    npix = r.cams.npix
    A, B, Ia = (t.cpu().numpy() for t in (r.A, r.B, r.I))
    for ch, fl in enumerate(chans):
        for k, cam in enumerate(scene.cameras):
            ref = oracle_mod.render(scene.forest, fl, cam, meth, sub, c_rk=c_rk)
            sl = slice(ch * npix + r.cams.img_off[k], ch * npix + r.cams.img_off[k + 1])
            for nm, x in (("A", A), ("B", B), ("I", Ia)):
                e = rel_err(x[sl], ref[nm])
                assert e <= PIX_TOL, (seed, ch, k, nm, e)
    # gradients over the first camera's pixels (the other cameras' dL/dI are zero)
    rng = np.random.default_rng([4243, seed])
    cam = scene.cameras[0]
    lo, hi = r.cams.img_off[0], r.cams.img_off[1]
    g = np.zeros(len(chans) * npix, np.float32)
    targets = []
    for ch in range(len(chans)):
        t = rng.uniform(0.0, 0.3, hi - lo)
        targets.append(t)
        g[ch * npix + lo:ch * npix + hi] = 2.0 * (Ia[ch * npix + lo:ch * npix + hi] - t)
    dk, de = r.backward(torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    # [leaf][corner] per channel; a single channel has no channel axis
    dk, de = dk.cpu().numpy(), de.cpu().numpy()
    if len(chans) == 1:
        dk, de = dk[None], de[None]
    for ch, fl in enumerate(chans):
        ref = oracle_mod.render(scene.forest, fl, cam, meth, sub, c_rk=c_rk)
        gk, ge = oracle_mod.grad(scene.forest, fl, cam, 2.0 * (ref["I"] - targets[ch]), meth, sub, c_rk=c_rk)
        ek = rel_err(dk[ch].T, gk)
        ee = rel_err(de[ch].T, ge)
        assert ek <= GRAD_TOL and ee <= GRAD_TOL, (seed, ch, ek, ee)
