"""ctypes view of librc (include/rc.h): structures and the entry points under
their C names.  Argument marshalling only; every step runs in librc's HIP
kernels.  Importing this module never falls back to anything else: if
librc.so is missing, ``lib()`` raises."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librc.so")

c_i32, c_i64, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t

RC_OK = 0
RC_EINVAL = -1
RC_EUNSUPPORTED = -2
RC_EWORKSPACE = -3
RC_ECAPACITY = -4
RC_EFOREST = -5
RC_EHIP = -6
RC_QMAXLEVEL = 19
RC_CAMERA_DOUBLES = 20
RC_GEOM_UNIT_CUBE, RC_GEOM_SHELL6, RC_GEOM_SURFACE, RC_GEOM_SURFACE2, RC_GEOM_SURFACE3 = 0, 1, 2, 3, 4
RC_GEOM_VOLUME2, RC_GEOM_VOLUME3 = 5, 6
RC_MAXTREES = 64
RC_MAXLISTS = 16
RC_MAXCH = 3
RC_MAX_FOLD_RUN = 2
RC_ABSENT = -1
RC_FIELD_CONST, RC_FIELD_TRILINEAR, RC_FIELD_CONST_EQ, RC_FIELD_SURFACE = 0, 1, 2, 3
RC_INT_ANALYTIC, RC_INT_RK4, RC_INT_GAUSS2, RC_INT_SIMPSON = 0, 1, 2, 3
RC_ADAPT_MAXDEPTH = 16
RC_STATIC_SCRATCH_BYTES = 64 << 20


class RcForest(ctypes.Structure):
    _fields_ = [("ntrees", c_i32), ("geom", c_i32), ("nleaves", c_i64), ("tree_begin", c_vp), ("level", c_vp),
                ("x", c_vp), ("y", c_vp), ("z", c_vp), ("geom_table", c_vp)]


class RcFields(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("nch", c_i32), ("kappa", c_vp), ("eps", c_vp)]


class RcIntegrator(ctypes.Structure):
    _fields_ = [("method", c_i32), ("substeps", c_i32), ("c_rk", ctypes.c_double)]


class RcTuning(ctypes.Structure):
    _fields_ = [("seg_blocks", c_i32), ("fold_blocks", c_i32), ("root_blocks", c_i32), ("adj_blocks", c_i32),
                ("fold_skip", ctypes.c_uint32)]


class RcIndex(ctypes.Structure):
    _fields_ = [("maxlevel", c_i32), ("leaf_levels", c_i32), ("ninternal", c_i64), ("cap_internal", c_i64),
                ("level_begin", c_i64 * (RC_QMAXLEVEL + 2)), ("root", c_i32), ("ntrees", c_i32),
                ("roots", c_i32 * RC_MAXTREES), ("child", c_vp), ("level", c_vp), ("x", c_vp), ("y", c_vp),
                ("z", c_vp), ("tree", c_vp)]


class RcVforest(ctypes.Structure):
    _fields_ = [("cap_vis", c_i64), ("cap_cand", c_i64), ("cap_rec", c_i64), ("vis_leaf", c_vp), ("vis_cam", c_vp),
                ("vis_rect", c_vp), ("cand_offset", c_vp), ("leaf_vis", c_vp), ("node_rect", c_vp),
                ("node_offset", c_vp), ("counts", c_vp), ("cand_chunk", c_vp), ("rec_chunk", c_vp),
                ("child_desc", c_vp)]


P = ctypes.POINTER
_SIGS = {
    "rc_strerror": (ctypes.c_char_p, [c_i32]),
    "rc_workspace_bytes": (c_sz, [P(RcForest), P(RcIndex), c_i32, P(RcVforest)]),
    "rc_camera_bytes": (c_sz, [c_i32]),
    "rc_node_slots": (c_i64, [P(RcIndex), c_i32]),
    "rc_camera_prepare": (c_i32, [c_vp, c_i32, c_vp, P(c_i64), c_vp]),
    "rc_forest_index": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_sz, c_vp]),
    "rc_prune_visible": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_i32, P(RcVforest), c_vp, c_sz, c_vp]),
    "rc_prune_visible_static": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_i32, P(RcVforest), c_vp]),
    "rc_segments": (c_i32, [P(RcForest), P(RcFields), c_vp, c_i32, P(RcVforest), P(RcIntegrator), c_vp, c_vp, c_vp,
                            P(RcTuning), c_vp]),
    "rc_composite": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_i32, P(RcVforest), c_vp, c_vp, c_i64, c_vp, c_vp, c_vp,
                             P(RcTuning), c_vp]),
    "rc_render": (c_i32, [P(RcForest), P(RcIndex), P(RcFields), c_vp, c_i32, P(RcVforest), P(RcIntegrator), c_vp,
                          c_vp, c_i64, c_vp, c_vp, c_vp, P(RcTuning), c_vp]),
    "rc_composite_channels": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_i32, P(RcVforest), c_i32, c_vp, c_vp, c_i64,
                                      c_vp, c_vp, c_vp, P(RcTuning), c_vp]),
    "rc_lists_workspace_bytes": (c_sz, [P(RcIndex), c_i32, c_i64]),
    "rc_composite_lists": (c_i32, [P(RcForest), P(RcIndex), c_vp, c_i32, P(RcVforest), c_vp, c_vp, c_i64, c_vp,
                                   c_vp, c_i64, c_vp, c_vp, c_sz, P(RcTuning), c_vp]),
    "rc_merge_lists": (c_i32, [c_vp, c_i32, c_i64, c_i32, P(c_vp), P(c_vp), c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rc_segments_backward": (c_i32, [P(RcForest), P(RcIndex), P(RcFields), c_vp, c_i32, P(RcVforest),
                                     P(RcIntegrator), c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp,
                                     c_sz, P(RcTuning), c_vp]),
}

EXPORTS = tuple(_SIGS)

_lib = None


class RcError(RuntimeError):
    def __init__(self, name, status):
        super().__init__(f"{name} failed: {strerror(status)} ({status})")
        self.status = status


def lib():
    """The loaded librc.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().rc_strerror(int(status)).decode()


def check(name: str, status: int) -> int:
    if status != RC_OK:
        raise RcError(name, status)
    return status


def call(name: str, *args, ok=(RC_OK,)):
    st = getattr(lib(), name)(*args)
    if st not in ok:
        raise RcError(name, st)
    return st
