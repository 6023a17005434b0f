"""The allocation-free prune (rc_prune_visible_static) against rc_prune_visible:
every output of the visible forest bit for bit, on two calls in a row on one
device (the second on a smaller forest with fewer cameras, so the shared
device scratch still holds the first call's data), and the images rendered
from the static prune's tables equal to the plain path's."""

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _outputs(vf, r):
    """The defined part of every vforest array, as host numpy arrays."""
    c = vf.read_counts()
    nv, nc, nr = c["nvis"], c["ncand"], c["nrec"]
    nslots, ncams, N = r.nslots, r.cams.ncams, r.forest.nleaves
    out = {
        "counts": vf.counts.cpu().numpy(),
        "vis_leaf": vf.vis_leaf[:nv], "vis_cam": vf.vis_cam[:nv], "vis_rect": vf.vis_rect[:4 * nv],
        "cand_offset": vf.cand_offset[:nv + 1], "leaf_vis": vf.leaf_vis[:ncams * N],
        "node_rect": vf.node_rect[:4 * nslots], "node_offset": vf.node_offset[:nslots + 1],
        "cand_chunk": vf.cand_chunk[:(nc + 63) // 64], "rec_chunk": vf.rec_chunk[:(nr + 63) // 64],
        "child_desc": vf.child_desc[:ncams * r.index.ninternal * 8 * 4],
    }
    return {k: (v if isinstance(v, np.ndarray) else v.cpu().numpy()) for k, v in out.items()}


def _poisoned_vforest(r):
    """A vforest of r's capacities with every array filled with -7, so that the
    entries a call leaves unwritten (the descriptors of invisible nodes) compare
    equal and anything else shows."""
    import paper_1809_01334_amd as P

    vf = P.VForest(r.device, r.forest.nleaves, r.cams.ncams, r.nslots, r.vf.cap_vis, r.vf.cap_cand, r.vf.cap_rec,
                   r.index.ninternal)
    for t in (vf.vis_leaf, vf.vis_cam, vf.vis_rect, vf.cand_offset, vf.leaf_vis, vf.node_rect, vf.node_offset,
              vf.cand_chunk, vf.rec_chunk, vf.child_desc):
        t.fill_(-7)
    return vf


def _static_prune(r):
    from paper_1809_01334_amd import _lib as L

    torch = _torch()
    vf = _poisoned_vforest(r)
    st = ctypes.c_void_p(torch.cuda.current_stream(r.device).cuda_stream)
    L.call("rc_prune_visible_static", ctypes.byref(r.forest.struct), ctypes.byref(r.index.struct),
           ctypes.c_void_p(r.cams.buf.data_ptr()), r.cams.ncams, ctypes.byref(vf.struct), st)
    torch.cuda.synchronize()
    return vf


def _plain_prune(r):
    import paper_1809_01334_amd as P

    torch = _torch()
    vf = _poisoned_vforest(r)
    P.rc_prune_visible(r.forest, r.index, r.cams, vf, r.ws)
    torch.cuda.synchronize()
    return vf


def test_static_prune_matches_prune_on_two_calls():
    torch = _torch()
    import paper_1809_01334_amd as P

    big = synth.small_scene(31, lmin=2, lmax=6, ngauss=5, w=160, h=120, ncams=3)
    small = synth.small_scene(32, lmin=1, lmax=4, ngauss=3, w=40, h=30, ncams=1)
    assert small.forest.nleaves < big.forest.nleaves
    results = []
    for scene in (big, small):
        print(f"[case] static prune: N={scene.forest.nleaves} cams={len(scene.cameras)}", flush=True)
        r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps)
        want = _outputs(_plain_prune(r), r)
        vf = _static_prune(r)
        got = _outputs(vf, r)
        assert want["counts"][3] == 0 and want["counts"][0] > 0
        for k in want:
            assert np.array_equal(got[k], want[k]), k
        # the static tables render the same images as the plain path's
        r.segments()
        r.composite()
        torch.cuda.synchronize()
        I0 = r.I.clone()
        r.vf, saved = vf, r.vf
        r.segments()
        r.composite()
        torch.cuda.synchronize()
        assert torch.equal(r.I, I0)
        r.vf = saved
        results.append(int(want["counts"][1]))
    assert results[1] < results[0]


def test_static_prune_rejects_oversize_before_the_gpu():
    """Beyond RC_STATIC_SCRATCH_BYTES the call returns RC_EWORKSPACE, checked on
    the host before anything is enqueued."""
    _torch()
    import paper_1809_01334_amd as P
    from paper_1809_01334_amd import _lib as L

    scene = synth.small_scene(33, lmin=1, lmax=3, ngauss=2, w=16, h=16)
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, scene.method, scene.substeps)
    f = L.RcForest.from_buffer_copy(r.forest.struct)
    f.nleaves = 10_000_000  # 80 MB of rectangles alone
    f.tree_begin = None
    st = L.lib().rc_prune_visible_static(ctypes.byref(f), ctypes.byref(r.index.struct),
                                         ctypes.c_void_p(r.cams.buf.data_ptr()), 1, ctypes.byref(r.vf.struct), None)
    assert st == L.RC_EWORKSPACE
