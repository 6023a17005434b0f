"""ctypes wrapper of the FP64 CPU oracle (rc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It compiles
``rc_oracle.c`` with gcc (no FP contraction, no fast-math) into
``liboracle.so`` next to this file.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
D = ctypes.c_double


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_prune.restype = I64
        L.or_prune.argtypes = [I64, P, P, P, P, I32, P, P]
        L.or_node_rect.restype = I32
        L.or_node_rect.argtypes = [I32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P, P]
        L.or_pairs.restype = I64
        L.or_pairs.argtypes = [I64, P, P, P, P, P, P, P, P, I64]
        L.or_render.restype = I32
        L.or_render.argtypes = [I64, P, P, P, P, I32, P, P, I32, I32, D, P, I64, P, P, P, P, P, P]
        L.or_grad.restype = I32
        L.or_grad.argtypes = [I64, P, P, P, P, I32, P, P, I32, I32, D, P, I64, P, P, P, P]
        L.or_grad_abs.restype = I32
        L.or_grad_abs.argtypes = [I64, P, P, P, P, I32, P, P, I32, I32, D, P, I64, P, P, P, P]
        L.or_segment.restype = I32
        L.or_segment.argtypes = [I32, P, P, ctypes.c_uint8, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, P, P, D, D, I32, I32, D, P, P]
        L.or_march.restype = I32
        L.or_march.argtypes = [I64, P, P, P, P, I32, P, P, P, I32, P, P, P]
        L.or_shell_prune.restype = I64
        L.or_shell_prune.argtypes = [I64, I32, P, P, P, P, P, P, P, P]
        L.or_shell_pairs.restype = I64
        L.or_shell_pairs.argtypes = [I64, P, I32, P, P, P, P, P, P, P, P, P, I64]
        L.or_shell_render.restype = I32
        L.or_shell_render.argtypes = [I64, I32, P, P, P, P, P, P, I32, P, P, I32, I32, D, P, I64, P, P, P, P, P, P]
        L.or_shell_march.restype = I32
        L.or_shell_march.argtypes = [I64, I32, P, P, P, P, P, P, I32, P, P, P, I32, P, P, P]
        L.or_share_units.restype = I64
        L.or_share_units.argtypes = [I64, P, P, P, P, P, P, P, P, I64]
        L.or_share_lists.restype = I64
        L.or_share_lists.argtypes = [I64, P, P, P, P, I32, P, P, I32, I32, D, P, P, P, I64]
        L.or_merge_pixel.restype = I64
        L.or_merge_pixel.argtypes = [I64, P, P]
        L.or_merge_sorted.restype = I64
        L.or_merge_sorted.argtypes = [I64, P, P, P]
        L.or_surface_render.restype = I32
        L.or_ho_surface_render.restype = I32
        L.or_ho_surface_render.argtypes = [I64, I32, P, P, P, P, P, P, P, P, I64, P, P, P, P, P, P, I32]
        L.or_ho_map.argtypes = [P, I32, I64, P, P]
        L.or_vol_cands.restype = I32
        L.or_vol_cands.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, P]
        L.or_vol_render.restype = I32
        L.or_vol_render.argtypes = [I64, I32, P, P, P, P, P, P, I32, P, P, I32, I32, P, I64, P, P, P, P, P, P]
        L.or_vol_map.argtypes = [P, I32, I64, P, P]
        L.or_vol_inverse.restype = I32
        L.or_vol_inverse.argtypes = [P, I32, I64, P, P]
        L.or_surface_render.argtypes = [I64, I32, P, P, P, P, P, P, P, P, I64, P, P, P, P, P, P]
        L.or_shell_map.argtypes = [P, I32, P, P]
        L.or_shell_inverse.argtypes = [P, I32, P, P]
        for nm in ("or_combine", "or_average"):
            getattr(L, nm).argtypes = [P, P, P]
        L.or_inverse.argtypes = [P, P]
        L.or_split.argtypes = [P, D, P, P]
        L.or_physical.argtypes = [P, D, P]
        L.or_rk4_step.argtypes = [P, P, D, P]
        _lib = L
    return _lib


def threads(n=None) -> int:
    """The OpenMP thread count the oracle runs with; with n, set it first."""
    lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _forest_args(forest):
    lv = _c(forest.level, np.uint8)
    x = _c(forest.x, np.uint32)
    y = _c(forest.y, np.uint32)
    z = _c(forest.z, np.uint32)
    return lv, x, y, z


def _field_args(fields, kappa=None, eps=None):
    """Field kind 1: trilinear corners; 0: constant (kappa, eps); 2: constant
    (kappa, equilibrium intensity I) with eps = kappa I (eq. BIrelation)."""
    k = _c(fields.kappa if kappa is None else kappa, np.float64)
    e = _c(fields.eps if eps is None else eps, np.float64)
    kind = 1 if k.shape[0] == 8 else (2 if getattr(fields, "kind", "") == "const_eq" else 0)
    return kind, k, e


# ---------------------------------------------------------------- group ops


def combine(near, far):
    a, b, o = _c(near, np.float64), _c(far, np.float64), np.zeros(2)
    lib().or_combine(_p(a), _p(b), _p(o))
    return o


def inverse(s):
    a, o = _c(s, np.float64), np.zeros(2)
    lib().or_inverse(_p(a), _p(o))
    return o


def split(s, frac1):
    a, o1, o2 = _c(s, np.float64), np.zeros(2), np.zeros(2)
    lib().or_split(_p(a), float(frac1), _p(o1), _p(o2))
    return o1, o2


def average(s1, s2):
    a, b, o = _c(s1, np.float64), _c(s2, np.float64), np.zeros(2)
    lib().or_average(_p(a), _p(b), _p(o))
    return o


def physical(s, dx):
    a, o = _c(s, np.float64), np.zeros(2)
    lib().or_physical(_p(a), float(dx), _p(o))
    return o


def rk4_step(beta4, gamma4, h):
    b, g, o = _c(beta4, np.float64), _c(gamma4, np.float64), np.zeros(2)
    lib().or_rk4_step(_p(b), _p(g), float(h), _p(o))
    return o


def segment(kind, kap, eps, level, x, y, z, rho, r, s_in, s_out, method, substeps=4, c_rk=0.0):
    """(A, B) and d(A, B)/d(kappa corners, eps corners) of one segment."""
    nc = 8 if kind == 1 else 1
    k, e = _c(kap, np.float64), _c(eps, np.float64)
    rh, rr = _c(rho, np.float64), _c(r, np.float64)
    ab, dab = np.zeros(2), np.zeros((2, 2 * nc))
    lib().or_segment(int(kind), _p(k), _p(e), int(level), int(x), int(y), int(z), _p(rh), _p(rr),
                     float(s_in), float(s_out), int(method), int(substeps), float(c_rk), _p(ab), _p(dab))
    return ab, dab


# ---------------------------------------------------------------- geometry


def _shell(forest):
    return getattr(forest, "geom", "unit_cube") == "shell6"


def _shell_args(forest):
    return (forest.ntrees, _c(forest.tree_begin, np.int64), _c(forest.geom_params, np.float64))


def prune(forest, cams_raw):
    """rect[cam][leaf] = (i0, i1, j0, j1); empty rectangles are (1, 0, 1, 0)."""
    cams = _c(np.atleast_2d(cams_raw), np.float64)
    lv, x, y, z = _forest_args(forest)
    rect = np.zeros((cams.shape[0], forest.nleaves, 4), np.int32)
    if _shell(forest):
        nt, tb, gp = _shell_args(forest)
        nvis = 0
        for k in range(cams.shape[0]):
            out = np.zeros((forest.nleaves, 4), np.int32)
            nvis += lib().or_shell_prune(forest.nleaves, nt, _p(tb), _p(gp), _p(lv), _p(x), _p(y), _p(z),
                                         _p(_c(cams[k], np.float64)), _p(out))
            rect[k] = out
        return rect, int(nvis)
    nvis = lib().or_prune(forest.nleaves, _p(lv), _p(x), _p(y), _p(z), cams.shape[0], _p(cams), _p(rect))
    return rect, int(nvis)


def node_rect(level, x, y, z, cam_raw):
    cam = _c(cam_raw, np.float64)
    rect = np.zeros(4, np.int32)
    vis = lib().or_node_rect(int(level), int(x), int(y), int(z), _p(cam), _p(rect))
    return rect, bool(vis)


def shell_pairs(forest, cam_raw, leaves=None):
    """Shell pairing: per candidate the number of intervals (0..2) and [s_in0, s_out0, s_in1, s_out1]."""
    lv, x, y, z = _forest_args(forest)
    nt, tb, gp = _shell_args(forest)
    lst = np.arange(forest.nleaves, dtype=np.int64) if leaves is None else _c(leaves, np.int64)
    cam = _c(cam_raw, np.float64)
    L = lib()
    args = (lst.shape[0], _p(lst), nt, _p(tb), _p(gp), _p(lv), _p(x), _p(y), _p(z), _p(cam))
    ncand = L.or_shell_pairs(*args, None, None, 0)
    nseg = np.zeros(max(ncand, 1), np.uint8)
    sio = np.zeros((max(ncand, 1), 4), np.float64)
    L.or_shell_pairs(*args, _p(nseg), _p(sio), ncand)
    return nseg[:ncand], sio[:ncand]


def pairs(forest, cam_raw, leaves=None):
    """Candidate pairing in (leaf, row-major pixel) order for the listed leaves."""
    lv, x, y, z = _forest_args(forest)
    lst = np.arange(forest.nleaves, dtype=np.int64) if leaves is None else _c(leaves, np.int64)
    cam = _c(cam_raw, np.float64)
    L = lib()
    ncand = L.or_pairs(lst.shape[0], _p(lst), _p(lv), _p(x), _p(y), _p(z), _p(cam), None, None, 0)
    hit = np.zeros(max(ncand, 1), np.uint8)
    sio = np.zeros((max(ncand, 1), 2), np.float64)
    L.or_pairs(lst.shape[0], _p(lst), _p(lv), _p(x), _p(y), _p(z), _p(cam), _p(hit), _p(sio), ncand)
    return hit[:ncand], sio[:ncand]


# ---------------------------------------------------------------- render / grad

METHODS = {"analytic": 0, "rk4": 1, "gauss2": 2, "simpson": 3}


def render(forest, fields, cam, method="rk4", substeps=4, pixels=None, kappa=None, eps=None,
           background=None, c_rk=0.0):
    """FP64 oracle image of one camera.  Returns dict with A, B, I, nseg (flat, row j=0 first)."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64).copy()
    if background is not None:
        raw = raw.copy()
        raw[17] = background
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields, kappa, eps)
    W, H = int(raw[14]), int(raw[15])
    if pixels is None:
        npo, pix = W * H, None
        nsel = -1
    else:
        pix = _c(pixels, np.int64)
        npo = nsel = pix.shape[0]
    A, B, I = np.zeros(npo), np.zeros(npo), np.zeros(npo)
    nseg = np.zeros(npo, np.int32)
    stats = np.zeros(4, np.int64)
    if _shell(forest):
        nt, tb, gp = _shell_args(forest)
        lib().or_shell_render(forest.nleaves, nt, _p(tb), _p(gp), _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e),
                              METHODS[method], int(substeps), float(c_rk), _p(raw), nsel, _p(pix), _p(A), _p(B), _p(I),
                              _p(nseg),
                              _p(stats))
        return {"A": A, "B": B, "I": I, "nseg": nseg, "segments": int(stats[0]), "overlaps": int(stats[1])}
    lib().or_render(forest.nleaves, _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e), METHODS[method],
                    int(substeps), float(c_rk), _p(raw), nsel, _p(pix), _p(A), _p(B), _p(I), _p(nseg), _p(stats))
    return {"A": A, "B": B, "I": I, "nseg": nseg, "segments": int(stats[0]), "overlaps": int(stats[1])}


def grad(forest, fields, cam, g, method="rk4", substeps=4, pixels=None, kappa=None, eps=None, c_rk=0.0):
    """dL/dkappa, dL/deps ([nc][N]) for per-pixel dL/dI = g."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields, kappa, eps)
    gg = _c(g, np.float64)
    if pixels is None:
        nsel, pix = -1, None
    else:
        pix = _c(pixels, np.int64)
        nsel = pix.shape[0]
    gk, ge = np.zeros_like(k), np.zeros_like(e)
    lib().or_grad(forest.nleaves, _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e), METHODS[method],
                  int(substeps), float(c_rk), _p(_c(raw, np.float64)), nsel, _p(pix), _p(gg), _p(gk), _p(ge))
    return gk, ge


def grad_abs(forest, fields, cam, w, method="rk4", substeps=4, pixels=None, kappa=None, eps=None, c_rk=0.0):
    """sum_p w_p |dI_p/dkappa|, sum_p w_p |dI_p/deps| ([nc][N]) for weights w >= 0: the
    bound on how far a per-pixel perturbation of dL/dI no larger than w moves the gradient."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields, kappa, eps)
    ww = _c(w, np.float64)
    if pixels is None:
        nsel, pix = -1, None
    else:
        pix = _c(pixels, np.int64)
        nsel = pix.shape[0]
    gk, ge = np.zeros_like(k), np.zeros_like(e)
    st = lib().or_grad_abs(forest.nleaves, _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e), METHODS[method],
                           int(substeps), float(c_rk), _p(_c(raw, np.float64)), nsel, _p(pix), _p(ww), _p(gk),
                           _p(ge))
    if st != 0:
        raise ValueError("grad_abs needs non-negative weights")
    return gk, ge


# ---------------------------------------------------------------- one process's share (Sec. 3.3, 3.5, 2.5)


def share_units(forest):
    """Maximal complete subtrees of a share (level u8, x, y, z u32), in curve order."""
    lv, x, y, z = _forest_args(forest)
    n = forest.nleaves
    m = lib().or_share_units(n, _p(lv), _p(x), _p(y), _p(z), None, None, None, None, 0)
    ul = np.zeros(max(m, 1), np.uint8)
    ux, uy, uz = (np.zeros(max(m, 1), np.uint32) for _ in range(3))
    lib().or_share_units(n, _p(lv), _p(x), _p(y), _p(z), _p(ul), _p(ux), _p(uy), _p(uz), m)
    return ul[:m], ux[:m], uy[:m], uz[:m]


def share_lists(forest, fields, cam, method="rk4", substeps=4, c_rk=0.0):
    """Per-pixel entry lists (offsets [P + 1], entries [m, 4] = s_in, s_out, A, B) of a share."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields)
    P_ = int(raw[14]) * int(raw[15])
    off = np.zeros(P_ + 1, np.int64)
    args = (forest.nleaves, _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e), METHODS[method], int(substeps),
            float(c_rk), _p(_c(raw, np.float64)), _p(off))
    m = lib().or_share_lists(*args, None, 0)
    ent = np.zeros((max(m, 1), 4), np.float64)
    lib().or_share_lists(*args, _p(ent), m)
    return off, ent[:m]


def merge_pixel(entries):
    """(A, B) of one pixel's entries sorted by s_in, with cut/average of overlaps; and the overlap count."""
    e = _c(entries, np.float64).reshape(-1, 4)
    ab = np.zeros(2)
    ov = lib().or_merge_pixel(e.shape[0], _p(e), _p(ab))
    return ab, int(ov)


def merge_lists(lists, P_, background=0.0):
    """Merge per-pixel lists of several shares (each (offsets, entries)): A, B, I and overlaps."""
    pix = np.concatenate([np.repeat(np.arange(P_), np.diff(off)) for off, _ in lists])
    ent = np.concatenate([e for _, e in lists]).reshape(-1, 4)
    order = np.lexsort((ent[:, 3], ent[:, 2], ent[:, 1], ent[:, 0], pix))  # by pixel, then (s_in, s_out, A, B)
    ent = _c(ent[order], np.float64)
    off = np.zeros(P_ + 1, np.int64)
    np.add.at(off, pix + 1, 1)
    off = np.cumsum(off)
    ab = np.zeros((P_, 2))
    ov = lib().or_merge_sorted(P_, _p(off), _p(ent), _p(ab))
    A, B = ab[:, 0], ab[:, 1]
    return {"A": A, "B": B, "I": A * background + B, "overlaps": int(ov)}


def surface_render(forest, fields, cam, pixels=None, hits=False):
    """FP64 oracle image of a surface forest (bilinear tree patches, Sec. 2.8 surface
    model).  fields.kappa / fields.eps hold the corner transparency A_s and intensity I_s
    ([4][N]).  hits=True adds hit_leaf / hit_s [npix][2 ntrees] (depth order, leaf -1 after
    the last hit)."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, _ = _forest_args(forest)
    As = _c(fields.kappa, np.float64)
    Is = _c(fields.eps, np.float64)
    assert As.shape == (4, forest.nleaves) and Is.shape == (4, forest.nleaves)
    W, H = int(raw[14]), int(raw[15])
    if pixels is None:
        npo, pix, nsel = W * H, None, -1
    else:
        pix = _c(pixels, np.int64)
        npo = nsel = pix.shape[0]
    A, B, I = np.zeros(npo), np.zeros(npo), np.zeros(npo)
    nh = 2 * forest.ntrees
    hl = np.zeros((npo, nh), np.int32) if hits else None
    hs = np.zeros((npo, nh)) if hits else None
    lib().or_surface_render(forest.nleaves, forest.ntrees, _p(_c(forest.tree_begin, np.int64)),
                            _p(_c(forest.geom_params, np.float64)), _p(lv), _p(x), _p(y), _p(As), _p(Is),
                            _p(_c(raw, np.float64)), nsel, _p(pix), _p(A), _p(B), _p(I), _p(hl), _p(hs))
    out = {"A": A, "B": B, "I": I}
    if hits:
        out["hit_leaf"] = hl
        out["hit_s"] = hs
    return out


def ho_surface_render(forest, fields, cam, pixels=None, hits=False):
    """FP64 oracle image of a degree-R surface forest (geom_params = [R, control points]);
    as surface_render, with up to 2 R^2 hits per tree."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, _ = _forest_args(forest)
    As = _c(fields.kappa, np.float64)
    Is = _c(fields.eps, np.float64)
    geom = _c(forest.geom_params, np.float64)
    R = int(geom[0])
    W, H = int(raw[14]), int(raw[15])
    if pixels is None:
        npo, pix, nsel = W * H, None, -1
    else:
        pix = _c(pixels, np.int64)
        npo = nsel = pix.shape[0]
    A, B, I = np.zeros(npo), np.zeros(npo), np.zeros(npo)
    hcap = min(2 * R * R * forest.ntrees, 64)
    hl = np.zeros((npo, hcap), np.int32) if hits else None
    hs = np.zeros((npo, hcap)) if hits else None
    st = lib().or_ho_surface_render(forest.nleaves, forest.ntrees, _p(_c(forest.tree_begin, np.int64)), _p(geom),
                                    _p(lv), _p(x), _p(y), _p(As), _p(Is), _p(_c(raw, np.float64)), nsel, _p(pix),
                                    _p(A), _p(B), _p(I), _p(hl), _p(hs), hcap)
    assert st == 0, "degree out of range"
    out = {"A": A, "B": B, "I": I}
    if hits:
        out["hit_leaf"] = hl
        out["hit_s"] = hs
    return out


def ho_map(geom, tree, t):
    """Points J(t1, t2) of a degree-R tree map at parameters t [m, 2]."""
    t = _c(np.atleast_2d(t), np.float64)
    out = np.zeros((t.shape[0], 3))
    lib().or_ho_map(_p(_c(geom, np.float64)), int(tree), t.shape[0], _p(t), _p(out))
    return out


def march(forest, fields, cam, M=1024):
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields)
    P_ = int(raw[14]) * int(raw[15])
    A, B, I = np.zeros(P_), np.zeros(P_), np.zeros(P_)
    if _shell(forest):
        nt, tb, gp = _shell_args(forest)
        lib().or_shell_march(forest.nleaves, nt, _p(tb), _p(gp), _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e),
                             _p(_c(raw, np.float64)), int(M), _p(A), _p(B), _p(I))
        return {"A": A, "B": B, "I": I}
    lib().or_march(forest.nleaves, _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e),
                   _p(_c(raw, np.float64)), int(M), _p(A), _p(B), _p(I))
    return {"A": A, "B": B, "I": I}


def shell_map(geom, k, t):
    x = np.zeros(3)
    lib().or_shell_map(_p(_c(geom, np.float64)), int(k), _p(_c(t, np.float64)), _p(x))
    return x


def shell_inverse(geom, k, x):
    t = np.zeros(3)
    lib().or_shell_inverse(_p(_c(geom, np.float64)), int(k), _p(_c(x, np.float64)), _p(t))
    return t


# ---------------------------------------------------------------- degree-R volume trees


def _vol_args(forest):
    return (forest.ntrees, _c(forest.tree_begin, np.int64), _c(forest.geom_params, np.float64))


def vol_render(forest, fields, cam, method="rk4", substeps=4, pixels=None):
    """FP64 image of one camera of a volume forest: dict A, B, I, nseg, segments, overlaps."""
    raw = cam.raw() if hasattr(cam, "raw") else np.asarray(cam, np.float64)
    lv, x, y, z = _forest_args(forest)
    kind, k, e = _field_args(fields)
    W, H = int(raw[14]), int(raw[15])
    if pixels is None:
        npo, pix, nsel = W * H, None, -1
    else:
        pix = _c(pixels, np.int64)
        npo = nsel = pix.shape[0]
    A, B, I = np.zeros(npo), np.zeros(npo), np.zeros(npo)
    nseg = np.zeros(npo, np.int32)
    stats = np.zeros(4, np.int64)
    nt, tb, gp = _vol_args(forest)
    st = lib().or_vol_render(forest.nleaves, nt, _p(tb), _p(gp), _p(lv), _p(x), _p(y), _p(z), kind, _p(k), _p(e),
                             METHODS[method], int(substeps), _p(_c(raw, np.float64)), nsel, _p(pix), _p(A), _p(B),
                             _p(I), _p(nseg), _p(stats))
    assert st == 0
    return {"A": A, "B": B, "I": I, "nseg": nseg, "segments": int(stats[0]), "overlaps": int(stats[1])}


def vol_cands(forest, cam_raw, leaf, pi, pj):
    """Intervals of explicit candidates (leaf, pixel (i, j)): counts and the first two (s_in, s_out)."""
    lv, x, y, z = _forest_args(forest)
    nt, tb, gp = _vol_args(forest)
    leaf = _c(leaf, np.int64)
    m = leaf.shape[0]
    nseg = np.zeros(max(m, 1), np.int32)
    iv = np.zeros((max(m, 1), 4), np.float64)
    st = lib().or_vol_cands(m, _p(leaf), _p(_c(pi, np.int32)), _p(_c(pj, np.int32)), nt, _p(tb), _p(gp), _p(lv),
                            _p(x), _p(y), _p(z), _p(_c(cam_raw, np.float64)), _p(nseg), _p(iv))
    assert st == 0
    return nseg[:m], iv[:m]


def vol_map(geom, tree, xi):
    xi = _c(np.atleast_2d(xi), np.float64)
    out = np.zeros_like(xi)
    lib().or_vol_map(_p(_c(geom, np.float64)), int(tree), xi.shape[0], _p(xi), _p(out))
    return out


def vol_inverse(geom, tree, x):
    x = _c(np.atleast_2d(x), np.float64)
    out = np.zeros_like(x)
    ok = lib().or_vol_inverse(_p(_c(geom, np.float64)), int(tree), x.shape[0], _p(x), _p(out))
    return out, bool(ok)
