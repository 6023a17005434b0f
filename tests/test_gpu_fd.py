"""The GPU adjoint against central finite differences of the GPU forward.

L = sum_p w_p I_p with fixed random weights; for random directions d in the
per-corner (kappa, eps) coefficients, (L(c + h d) - L(c - h d)) / 2h from two
FP32 forwards must match the adjoint's directional derivative dL/dc . d.  The
loss is summed in FP64 on the host, and h is large enough that FP32 rounding of
the images stays well below the tolerance.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import _torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method,substeps", [("analytic", 1), ("rk4", 4), ("rk4", 1), ("gauss2", 4), ("simpson", 2)])
def test_adjoint_matches_central_differences(method, substeps):
    torch = _torch()
    import paper_1809_01334_amd as P

    sc = synth.small_scene(51, w=72, h=56, background=0.4)
    rng = np.random.default_rng(51)
    N = sc.forest.nleaves
    if method == "analytic":
        sc.fields = synth.constant_fields(rng.uniform(0.2, 3.0, N), rng.uniform(0.0, 1.0, N))
    print(f"[case] finite differences {method} x{substeps}, N={N}", flush=True)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, method, substeps)
    k0 = r.fields.kappa.clone()
    e0 = r.fields.eps.clone()
    w = torch.from_numpy(rng.uniform(-1.0, 1.0, r.cams.npix).astype(np.float32)).cuda()

    def loss(k, e):
        r.set_fields(k, e)
        r.forward()
        torch.cuda.synchronize()
        return float((w.double() * r.I.double()).sum().item())

    r.set_fields(k0, e0)
    r.forward()
    dk, de = r.backward(w)
    torch.cuda.synchronize()
    for trial in range(3):
        dkd = torch.from_numpy(rng.normal(size=k0.shape).astype(np.float32)).cuda()
        ded = torch.from_numpy(rng.normal(size=e0.shape).astype(np.float32)).cuda()
        h = 2e-2
        fd = (loss(k0 + h * dkd, e0 + h * ded) - loss(k0 - h * dkd, e0 - h * ded)) / (2 * h)
        ad = float((dk.double() * dkd.double()).sum().item() + (de.double() * ded.double()).sum().item())
        assert abs(fd - ad) <= 2e-3 * max(abs(ad), 1e-6), (method, substeps, trial, fd, ad)
