"""GPU parity on the curved six-tree shell (Sec. 2.1 smooth per-tree maps).

Visibility (lenient boxes) and pairing (the number of intervals and both
intervals in FP64) bit for bit against the oracle; A, B and I within 1e-5
relative (floor 1e-3 of the image maximum).  The GPU maps RK4 points back to
reference coordinates by FP64 Newton, the oracle by the closed-form inverse.
"""

import numpy as np
import pytest

import synth
from test_gpu_parity import PIX_TOL, _check_images, _check_prune, _renderer, _torch

pytestmark = pytest.mark.gpu


def _check_shell_pairing(r, scene, O, cams, leaves, off, sample=None):
    hit, sio = r.debug_segments()
    for k, cam in enumerate(scene.cameras):
        vsel = np.flatnonzero(cams == k)
        if sample is not None and len(vsel) > sample:
            vsel = np.sort(np.random.default_rng(k).choice(vsel, sample, replace=False))
        if len(vsel) == 0:
            continue
        n_ref, s_ref = O.shell_pairs(scene.forest, cam.raw(), leaves[vsel])
        idx = np.concatenate([np.arange(off[v], off[v + 1]) for v in vsel])
        assert len(idx) == len(n_ref)
        ti = _torch().from_numpy(idx).to(hit.device)
        n_gpu = hit[ti].cpu().numpy()
        s_gpu = sio.view(-1, 4)[ti].cpu().numpy()
        assert np.array_equal(n_gpu, n_ref), (scene.name, k, int((n_gpu != n_ref).sum()))
        assert np.array_equal(s_gpu.view(np.uint64), s_ref.view(np.uint64)), (scene.name, k)
        assert n_ref.max() <= 2
    return hit


@pytest.mark.parametrize("seed,lmin,lmax,w,h", [(0, 1, 3, 96, 72), (1, 2, 4, 120, 90), (2, 1, 2, 61, 47)])
def test_shell_small_parity(oracle_mod, seed, lmin, lmax, w, h):
    scene = synth.shell_scene(seed, lmin=lmin, lmax=lmax, w=w, h=h, dist=2.4)
    r = _renderer(scene)
    r.forward()
    cams, leaves, off = _check_prune(r, scene, oracle_mod)
    hit = _check_shell_pairing(r, scene, oracle_mod, cams, leaves, off)
    assert int((hit[:int(off[-1])] == 2).sum().item()) > 0  # rays that cross the hollow core
    r.forward()
    _check_images(r, scene, oracle_mod)


@pytest.mark.parametrize("seed", range(6))
def test_shell_random_cases(oracle_mod, seed):
    """Seeded random cases: refinement depth, one or two cameras at random distances and sizes (rays through
    the hollow core), background, RK4 with 1, 2 or 4 substeps or constant fields in closed form."""
    rng = np.random.default_rng([7171, seed])
    lmin = int(rng.integers(1, 3))
    scene = synth.shell_scene(40 + seed, lmin=lmin, lmax=lmin + int(rng.integers(1, 3)),
                              w=int(rng.integers(30, 90)), h=int(rng.integers(30, 90)),
                              dist=float(rng.uniform(1.6, 3.5)), background=float(rng.uniform(0.0, 0.5)))
    if rng.integers(2):
        N = scene.forest.nleaves
        scene.fields = synth.constant_fields(rng.uniform(0.1, 2.0, N), rng.uniform(0.0, 1.0, N))
        scene.method, scene.substeps = "analytic", 1
    else:
        scene.substeps = int(rng.choice([1, 2, 4]))
    if rng.integers(2):
        w, h = int(rng.integers(20, 60)), int(rng.integers(20, 60))
        scene.cameras.append(synth.random_perspective_camera(rng, w, h, dist=float(rng.uniform(1.6, 3.0)),
                                                             center=(0.0, 0.0, 0.0)))
    r = _renderer(scene)
    r.forward()
    cams, leaves, off = _check_prune(r, scene, oracle_mod)
    _check_shell_pairing(r, scene, oracle_mod, cams, leaves, off)
    r.forward()
    _check_images(r, scene, oracle_mod)


def test_shell_constant_analytic_background_and_two_cameras(oracle_mod):
    scene = synth.shell_scene(5, lmin=1, lmax=3, w=80, h=64, dist=2.8, background=0.4)
    rng = np.random.default_rng(55)
    N = scene.forest.nleaves
    scene.fields = synth.constant_fields(rng.uniform(0.1, 2.0, N), rng.uniform(0.0, 1.0, N))
    scene.method = "analytic"
    scene.cameras.append(synth.random_perspective_camera(rng, 47, 33, dist=2.2, center=(0.0, 0.0, 0.0),
                                                         background=0.1))
    r = _renderer(scene)
    r.forward()
    cams, leaves, off = _check_prune(r, scene, oracle_mod)
    _check_shell_pairing(r, scene, oracle_mod, cams, leaves, off)
    r.forward()
    _check_images(r, scene, oracle_mod)


def test_shell_rk4_substep_counts(oracle_mod):
    scene = synth.shell_scene(6, lmin=1, lmax=3, w=64, h=48, dist=2.6)
    for ns in (1, 2, 8):
        scene.substeps = ns
        r = _renderer(scene)
        r.forward()
        _check_images(r, scene, oracle_mod)


def test_shell_adjoint_is_rejected(oracle_mod):
    import paper_1809_01334_amd as P

    scene = synth.shell_scene(7, lmin=1, lmax=2, w=32, h=24)
    r = _renderer(scene)
    r.forward()
    torch = _torch()
    with pytest.raises(P.RcError) as e:
        r.backward(torch.ones_like(r.I))
    assert e.value.status == P._lib.RC_EUNSUPPORTED


def test_shell_graph_replay_matches_eager(oracle_mod):
    torch = _torch()
    scene = synth.shell_scene(8, lmin=1, lmax=3, w=72, h=54, dist=2.5)
    r = _renderer(scene)
    r.forward()
    ref = r.I.clone()
    r.capture()
    for _ in range(3):
        r.I.zero_()
        torch.cuda.synchronize()
        r.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.I, ref)


@pytest.mark.timeout(400)
def test_shell_full_size_sampled(oracle_mod):
    """The 2048x2048, levels 3-7 shell (about 5.2 M leaves): pairing on sampled
    leaves, pixels on a sample of 3000."""
    scene = synth.config_scene(3)
    r = _renderer(scene)
    r.forward()
    cams, leaves, off = _check_prune(r, scene, oracle_mod)
    _check_shell_pairing(r, scene, oracle_mod, cams, leaves, off, sample=300)
    r.forward()
    pix = np.sort(np.random.default_rng(33).choice(2048 * 2048, 3000, replace=False))
    _check_images(r, scene, oracle_mod, pixels=pix)
