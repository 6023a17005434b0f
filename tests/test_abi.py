"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1809_01334_amd import _lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("librc.so not built")
    return L


def test_library_exports_every_declared_entry_point():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "rc.h")).read()
    declared = set(re.findall(r"^\s*(?:rc_status|size_t|int64_t|const char \*)\s*(rc_\w+)\(", header, re.M))
    assert {"rc_prune_visible", "rc_segments", "rc_composite", "rc_segments_backward"} <= declared
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS)


def test_status_names():
    L = _lib()
    assert L.strerror(0) == "ok"
    for s in (-1, -2, -3, -4, -5, -6):
        assert L.strerror(s) != "unknown status"


def test_camera_validation_rejects_bad_cameras():
    L = _lib()
    lib = L.lib()
    good = synth.random_perspective_camera(np.random.default_rng(1), 64, 48).raw()
    npix = ctypes.c_int64(0)

    def prep(raw):
        raw = np.ascontiguousarray(raw, np.float64)
        # a non-null device pointer is never dereferenced when validation fails
        return lib.rc_camera_prepare(raw.ctypes.data_as(ctypes.c_void_p), 1, ctypes.c_void_p(16),
                                     ctypes.byref(npix), None)

    bad = []
    r = good.copy(); r[13] = 0.5; bad.append(r)            # zfar <= n
    r = good.copy(); r[14] = 0; bad.append(r)              # w = 0
    r = good.copy(); r[15] = 40000; bad.append(r)          # h too large
    r = good.copy(); r[12] = -1.0; bad.append(r)           # ell <= 0
    r = good.copy(); r[6:9] *= 2.0; bad.append(r)          # t not unit
    r = good.copy(); r[6:9] = -r[6:9]; bad.append(r)       # right-handed frame
    r = good.copy(); r[3:6] = 0.0; bad.append(r)           # n = 0
    r = good.copy(); r[0] = np.nan; bad.append(r)
    for raw in bad:
        assert prep(raw) == L.RC_EINVAL
    assert lib.rc_camera_prepare(None, 1, ctypes.c_void_p(16), ctypes.byref(npix), None) == L.RC_EINVAL


def test_null_and_unsupported_arguments():
    L = _lib()
    lib = L.lib()
    assert lib.rc_forest_index(None, None, None, 0, None) == L.RC_EINVAL
    f = L.RcForest(1, 0, 0, None, None, None, None, None)  # no leaves
    ix = L.RcIndex()
    assert lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None) == L.RC_EINVAL
    f = L.RcForest(2, 0, 8, None, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    assert lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None) == L.RC_EUNSUPPORTED
    f = L.RcForest(1, 0, 8, None, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    assert lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None) == L.RC_EWORKSPACE
    # analytic integration needs constant fields; more than 64 substeps is rejected
    fl = L.RcFields(L.RC_FIELD_TRILINEAR, 1, ctypes.c_void_p(16), ctypes.c_void_p(16))
    vf = L.RcVforest()
    integ = L.RcIntegrator(L.RC_INT_ANALYTIC, 1)
    assert lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), ctypes.c_void_p(16), 1, ctypes.byref(vf),
                           ctypes.byref(integ), ctypes.c_void_p(16), None, None, None, None) == L.RC_EUNSUPPORTED
    integ = L.RcIntegrator(L.RC_INT_RK4, 65)
    assert lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), ctypes.c_void_p(16), 1, ctypes.byref(vf),
                           ctypes.byref(integ), ctypes.c_void_p(16), None, None, None, None) == L.RC_EINVAL
    # 1 .. RC_MAXCH channels
    integ = L.RcIntegrator(L.RC_INT_RK4, 4)
    for nch in (0, L.RC_MAXCH + 1):
        fl = L.RcFields(L.RC_FIELD_CONST, nch, ctypes.c_void_p(16), ctypes.c_void_p(16))
        assert lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), ctypes.c_void_p(16), 1, ctypes.byref(vf),
                               ctypes.byref(integ), ctypes.c_void_p(16), None, None, None, None) == L.RC_EINVAL
        p = ctypes.c_void_p(16)
        assert lib.rc_composite_channels(ctypes.byref(f), ctypes.byref(ix), p, 1, ctypes.byref(vf), nch, p, p, 1,
                                         p, p, p, None, None) == L.RC_EINVAL


def test_sizes_are_consistent():
    L = _lib()
    lib = L.lib()
    assert lib.rc_camera_bytes(3) == 3 * lib.rc_camera_bytes(1) > 0
    ix = L.RcIndex()
    ix.maxlevel = 3
    for l, b in enumerate([0, 1, 9, 73, 73]):
        ix.level_begin[l] = b
    assert lib.rc_node_slots(ctypes.byref(ix), 2) == 2 * (73 - 1)
    f = L.RcForest(1, 0, 1000, None, None, None, None, None)
    b1 = lib.rc_workspace_bytes(ctypes.byref(f), None, 1, None)
    b4 = lib.rc_workspace_bytes(ctypes.byref(f), ctypes.byref(ix), 64, None)
    assert b4 >= b1 > 0


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle and fails loudly without librc."""
    pkg = os.path.join(ROOT, "paper_1809_01334_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src, fn


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """sizeof and offsetof of every struct in rc.h, from a C probe built with gcc."""
    import shutil
    import subprocess

    from paper_1809_01334_amd import _lib as L

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"rc_forest": L.RcForest, "rc_fields": L.RcFields, "rc_integrator": L.RcIntegrator,
               "rc_tuning": L.RcTuning, "rc_index": L.RcIndex, "rc_vforest": L.RcVforest}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            if fname.startswith("pad"):
                continue
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    for line in filter(None, out):
        cname, fname, val = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if fname == "sizeof" else getattr(py, fname).offset
        assert int(val) == want, (cname, fname, int(val), want)


def test_shell_forest_validation():
    """The six-tree shell needs six trees, their leaf offsets and the geometry table."""
    L = _lib()
    lib = L.lib()
    ix = L.RcIndex()
    p = ctypes.c_void_p(16)
    tb6 = np.array([0, 2, 4, 6, 8, 10, 12], np.int64)
    ptb6 = tb6.ctypes.data_as(ctypes.c_void_p)

    def status(ntrees, tb, table, n=12):
        f = L.RcForest(ntrees, L.RC_GEOM_SHELL6, n, tb, p, p, p, p, table)
        return lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None)

    assert status(1, ptb6, p) == L.RC_EINVAL          # one tree
    assert status(6, None, p) == L.RC_EINVAL          # no tree offsets
    assert status(6, ptb6, None) == L.RC_EINVAL       # no geometry table
    bad = np.array([0, 2, 4, 3, 8, 10, 12], np.int64)  # offsets not monotone
    assert status(6, bad.ctypes.data_as(ctypes.c_void_p), p) == L.RC_EINVAL
    assert status(6, ptb6, p, n=11) == L.RC_EINVAL    # last offset != leaves
    assert status(6, ptb6, p) == L.RC_EWORKSPACE      # valid forest, no workspace
    f = L.RcForest(6, 7, 12, ptb6, p, p, p, p, p)     # unknown geometry
    assert lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None) == L.RC_EUNSUPPORTED


def test_integrator_validation():
    """Gauss, Simpson and the recursion need a power-of-two piece count; the
    equilibrium-intensity fields take the closed form only."""
    L = _lib()
    lib = L.lib()
    p = ctypes.c_void_p(16)
    f = L.RcForest(1, 0, 8, None, p, p, p, p)
    vf = L.RcVforest()

    def seg(kind, method, sub, c_rk=0.0):
        fl = L.RcFields(kind, 1, p, p)
        integ = L.RcIntegrator(method, sub, c_rk)
        return lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), p, 1, ctypes.byref(vf), ctypes.byref(integ), p,
                               None, None, None, None)

    T, C, E = L.RC_FIELD_TRILINEAR, L.RC_FIELD_CONST, L.RC_FIELD_CONST_EQ
    assert seg(T, L.RC_INT_GAUSS2, 3) == L.RC_EINVAL
    assert seg(T, L.RC_INT_SIMPSON, 6) == L.RC_EINVAL
    assert seg(T, L.RC_INT_RK4, 3, 0.5) == L.RC_EINVAL       # recursion: power of two
    assert seg(T, L.RC_INT_RK4, 4, -0.1) == L.RC_EINVAL
    assert seg(T, L.RC_INT_RK4, 4, float("nan")) == L.RC_EINVAL
    assert seg(T, 7, 4) == L.RC_EUNSUPPORTED
    assert seg(T, L.RC_INT_ANALYTIC, 1) == L.RC_EUNSUPPORTED
    assert seg(E, L.RC_INT_RK4, 4) == L.RC_EUNSUPPORTED
    assert seg(E, L.RC_INT_GAUSS2, 4) == L.RC_EUNSUPPORTED
    # valid combinations get past validation and stop at the empty vforest
    for kind, method, sub, c_rk in ((T, L.RC_INT_GAUSS2, 4, 0.0), (C, L.RC_INT_SIMPSON, 2, 0.3),
                                    (E, L.RC_INT_ANALYTIC, 1, 0.0), (T, L.RC_INT_RK4, 3, 0.0)):
        assert seg(kind, method, sub, c_rk) == L.RC_EINVAL  # null vforest arrays


def test_visible_pair_capacity_is_limited_to_31_bits():
    """The chunk table stores pair indices as int32, so a capacity of 2^31 or
    more is refused before any device work."""
    L = _lib()
    lib = L.lib()
    p = ctypes.c_void_p(16)
    f = L.RcForest(1, 0, 8, None, p, p, p, p)
    fl = L.RcFields(L.RC_FIELD_TRILINEAR, 1, p, p)
    integ = L.RcIntegrator(L.RC_INT_RK4, 4, 0.0)

    def seg(cap_vis):
        vf = L.RcVforest()
        vf.cap_vis, vf.cap_cand, vf.cap_rec = cap_vis, 64, 0
        for nm in ("vis_leaf", "vis_cam", "vis_rect", "cand_offset", "leaf_vis", "counts"):
            setattr(vf, nm, p)
        return lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), p, 1, ctypes.byref(vf), ctypes.byref(integ), p,
                               None, None, None, None)

    assert seg(2 ** 31) == L.RC_EUNSUPPORTED
    assert seg(2 ** 31 - 1) == L.RC_EUNSUPPORTED
    assert seg(-1) == L.RC_EINVAL


def test_surface_validation():
    """Surface forests take 1 to 6 trees with a corner table, surface data only, and the
    closed-form surface model; the adjoint rejects them."""
    L = _lib()
    lib = L.lib()
    ix = L.RcIndex()
    p = ctypes.c_void_p(16)
    tb = np.array([0, 4, 8], np.int64)
    ptb = tb.ctypes.data_as(ctypes.c_void_p)

    def index_status(ntrees, tb_, table, n=8):
        f = L.RcForest(ntrees, L.RC_GEOM_SURFACE, n, tb_, p, p, p, p, table)
        return lib.rc_forest_index(ctypes.byref(f), ctypes.byref(ix), None, 0, None)

    assert index_status(0, ptb, p) == L.RC_EINVAL
    t7 = np.arange(8, dtype=np.int64)
    assert index_status(7, t7.ctypes.data_as(ctypes.c_void_p), p, n=7) == L.RC_EINVAL
    assert index_status(2, ptb, None) == L.RC_EINVAL
    assert index_status(2, None, p) == L.RC_EINVAL
    assert index_status(2, ptb, p) == L.RC_EWORKSPACE

    vf = L.RcVforest()
    for name in ("vis_leaf", "vis_cam", "vis_rect", "cand_offset", "leaf_vis", "counts", "cand_chunk"):
        setattr(vf, name, p)

    def seg(geom, ntrees, tb_, table, kind, method):
        f = L.RcForest(ntrees, geom, 8, tb_, p, p, p, p, table)
        fl = L.RcFields(kind, 1, p, p)
        integ = L.RcIntegrator(method, 1, 0.0)
        return lib.rc_segments(ctypes.byref(f), ctypes.byref(fl), p, 1, ctypes.byref(vf), ctypes.byref(integ), p,
                               None, None, None, None)

    S, A = L.RC_FIELD_SURFACE, L.RC_INT_ANALYTIC
    assert seg(L.RC_GEOM_SURFACE, 2, ptb, p, S, L.RC_INT_RK4) == L.RC_EUNSUPPORTED      # no ODE on a surface
    assert seg(L.RC_GEOM_SURFACE, 2, ptb, p, L.RC_FIELD_CONST, A) == L.RC_EUNSUPPORTED  # volume data
    assert seg(L.RC_GEOM_UNIT_CUBE, 1, None, None, S, A) == L.RC_EUNSUPPORTED           # surface data on a cube
    f = L.RcForest(2, L.RC_GEOM_SURFACE, 8, ptb, p, p, p, p, p)
    fl = L.RcFields(S, 1, p, p)
    integ = L.RcIntegrator(A, 1, 0.0)
    st = lib.rc_segments_backward(ctypes.byref(f), ctypes.byref(ix), ctypes.byref(fl), p, 1, ctypes.byref(vf),
                                  ctypes.byref(integ), p, p, 1, p, p, p, p, p, 0, p, 0, None, None)
    assert st == L.RC_EUNSUPPORTED


def test_node_slot_count_is_limited_to_31_bits():
    """The record chunk table stores (level, camera, node) slot indices as int32,
    so a slot count of 2^31 - 1 or more is refused before any device work."""
    L = _lib()
    lib = L.lib()
    p = ctypes.c_void_p(16)
    f = L.RcForest(1, 0, 8, None, p, p, p, p)
    vf = L.RcVforest()
    for nm in ("vis_leaf", "vis_cam", "vis_rect", "cand_offset", "leaf_vis", "node_rect", "node_offset", "counts",
               "cand_chunk", "rec_chunk", "child_desc"):
        setattr(vf, nm, p)
    vf.cap_vis, vf.cap_cand, vf.cap_rec = 64, 64, 64

    def prune(internal_below_root, ncams):
        ix = L.RcIndex()
        ix.child, ix.level, ix.x, ix.y, ix.z, ix.tree = p, p, p, p, p, p
        ix.maxlevel = 2
        ix.level_begin[0], ix.level_begin[1] = 0, 1
        for l in range(2, len(ix.level_begin)):
            ix.level_begin[l] = 1 + internal_below_root
        ix.ninternal = ix.cap_internal = 1 + internal_below_root
        assert lib.rc_node_slots(ctypes.byref(ix), ncams) == ncams * internal_below_root
        return lib.rc_prune_visible(ctypes.byref(f), ctypes.byref(ix), p, ncams, ctypes.byref(vf), None, 0, None)

    assert prune(2 ** 27, 16) == L.RC_EUNSUPPORTED        # 2^31 slots
    assert prune(2 ** 31 - 1, 1) == L.RC_EUNSUPPORTED     # 2^31 - 1 slots
    assert prune(2 ** 31 - 2, 1) == L.RC_EWORKSPACE       # the largest count passes, then needs a workspace


def test_static_prune_limits_its_scratch():
    """The allocation-free prune refuses, before any device work, a call whose
    workspace would exceed RC_STATIC_SCRATCH_BYTES (about 8 M items), and checks
    its arguments like rc_prune_visible."""
    L = _lib()
    lib = L.lib()
    p = ctypes.c_void_p(16)
    vf = L.RcVforest()
    for nm in ("vis_leaf", "vis_cam", "vis_rect", "cand_offset", "leaf_vis", "node_rect", "node_offset", "counts",
               "cand_chunk", "rec_chunk", "child_desc"):
        setattr(vf, nm, p)
    vf.cap_vis, vf.cap_cand, vf.cap_rec = 64, 64, 64
    ix = L.RcIndex()
    ix.child, ix.level, ix.x, ix.y, ix.z, ix.tree = p, p, p, p, p, p
    ix.maxlevel = 1
    ix.level_begin[0] = 0
    for l in range(1, len(ix.level_begin)):
        ix.level_begin[l] = 1
    ix.ninternal = ix.cap_internal = 1

    def prune(nleaves, ncams):
        f = L.RcForest(1, 0, nleaves, None, p, p, p, p)
        want = lib.rc_workspace_bytes(ctypes.byref(f), ctypes.byref(ix), ncams, None)
        st = lib.rc_prune_visible_static(ctypes.byref(f), ctypes.byref(ix), p, ncams, ctypes.byref(vf), None)
        return st, want

    st, want = prune(9_000_000, 1)
    assert want > L.RC_STATIC_SCRATCH_BYTES and st == L.RC_EWORKSPACE
    st, want = prune(1_000_000, 9)
    assert want > L.RC_STATIC_SCRATCH_BYTES and st == L.RC_EWORKSPACE
    assert lib.rc_prune_visible_static(None, ctypes.byref(ix), p, 1, ctypes.byref(vf), None) == L.RC_EINVAL
    f = L.RcForest(1, 0, 8, None, p, p, p, p)
    assert lib.rc_prune_visible_static(ctypes.byref(f), ctypes.byref(ix), None, 1, ctypes.byref(vf), None) == \
        L.RC_EINVAL
