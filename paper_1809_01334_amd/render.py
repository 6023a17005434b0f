"""Python binding of librc: device buffers (torch) plus calls under the C
names of include/rc.h, and a Renderer that sequences them for one forest and
a set of cameras.  torch supplies device memory and streams only; every step
of the path runs in librc's kernels."""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _empty(n, dtype, device):
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


# ---------------------------------------------------------------------------- device data


class DeviceForest:
    """Leaves of one forest share on the device (SFC order).  Geometry: the
    unit cube (one tree), or with ``geom_table`` the six-tree shell, or with
    geom=RC_GEOM_SURFACE quadtrees on bilinear patches (12 corner doubles per tree)."""

    def __init__(self, level, x, y, z, device, tree_begin=None, geom_table=None, geom=None):
        self.device = torch.device(device)
        self.nleaves = int(len(level))
        self.level = torch.from_numpy(np.ascontiguousarray(level, np.uint8)).to(self.device)
        self.x = torch.from_numpy(np.ascontiguousarray(x, np.uint32).view(np.int32)).to(self.device)
        self.y = torch.from_numpy(np.ascontiguousarray(y, np.uint32).view(np.int32)).to(self.device)
        self.z = torch.from_numpy(np.ascontiguousarray(z, np.uint32).view(np.int32)).to(self.device)
        tb = np.array([0, self.nleaves], np.int64) if tree_begin is None else np.asarray(tree_begin, np.int64)
        self.tree_begin = np.ascontiguousarray(tb)
        if geom is None:
            geom = L.RC_GEOM_UNIT_CUBE if geom_table is None else L.RC_GEOM_SHELL6
        self.geom = int(geom)
        self.geom_table = None
        if geom_table is not None:
            self.geom_table = torch.from_numpy(np.ascontiguousarray(geom_table, np.float64)).to(self.device)
        self.struct = L.RcForest(int(len(tb) - 1), self.geom, self.nleaves,
                                 self.tree_begin.ctypes.data_as(ctypes.c_void_p), _ptr(self.level), _ptr(self.x),
                                 _ptr(self.y), _ptr(self.z), _ptr(self.geom_table))

    @property
    def shell(self) -> bool:
        return self.geom == L.RC_GEOM_SHELL6

    @property
    def curved(self) -> bool:
        """Records hold two depth-tagged intervals (shell intervals, surface hits)."""
        return self.geom in (L.RC_GEOM_SHELL6, L.RC_GEOM_SURFACE, L.RC_GEOM_SURFACE2, L.RC_GEOM_SURFACE3,
                             L.RC_GEOM_VOLUME2, L.RC_GEOM_VOLUME3)

    @classmethod
    def from_synth(cls, forest, device):
        table = forest.geom_params
        if forest.geom in ("surface_ho", "volume"):
            # [R, control points]: the degree picks the geometry code
            codes = ({2: L.RC_GEOM_SURFACE2, 3: L.RC_GEOM_SURFACE3} if forest.geom == "surface_ho"
                     else {2: L.RC_GEOM_VOLUME2, 3: L.RC_GEOM_VOLUME3})
            geom = codes[int(table[0])]
            table = table[1:]
        else:
            geom = {"unit_cube": L.RC_GEOM_UNIT_CUBE, "shell6": L.RC_GEOM_SHELL6,
                    "surface": L.RC_GEOM_SURFACE}[forest.geom]
        if geom == L.RC_GEOM_UNIT_CUBE:
            table = None
        return cls(forest.level, forest.x, forest.y, forest.z, device, forest.tree_begin, table, geom)


class DeviceFields:
    """Coefficients leaf-major: kappa, eps of shape [N, ncorner] (ncorner 1 or 8), or
    [nch, N, ncorner] for several channels.
    equilibrium=True: constant kappa and the equilibrium intensity I in place of eps.
    surface=True: [N, 4] corner transparency A_s (kappa) and intensity I_s (eps)."""

    def __init__(self, kappa: torch.Tensor, eps: torch.Tensor, equilibrium: bool = False, surface: bool = False):
        assert kappa.shape == eps.shape and kappa.dim() in (2, 3)
        self.nch = int(kappa.shape[0]) if kappa.dim() == 3 else 1
        assert 1 <= self.nch <= L.RC_MAXCH
        assert kappa.shape[-1] in ((4,) if surface else (1, 8))
        assert kappa.dtype == torch.float32 and eps.dtype == torch.float32
        assert not (equilibrium and kappa.shape[-1] != 1)
        self.kappa = kappa.contiguous()
        self.eps = eps.contiguous()
        if surface:
            self.kind = L.RC_FIELD_SURFACE
        elif equilibrium:
            self.kind = L.RC_FIELD_CONST_EQ
        else:
            self.kind = L.RC_FIELD_TRILINEAR if kappa.shape[-1] == 8 else L.RC_FIELD_CONST
        self.struct = L.RcFields(self.kind, self.nch, _ptr(self.kappa), _ptr(self.eps))

    @staticmethod
    def leaf_major(a) -> np.ndarray:
        """[ncorner][N] (the generators' layout) to [N][ncorner]; [nch][ncorner][N] to [nch][N][ncorner]."""
        a = np.asarray(a, np.float32)
        return np.ascontiguousarray(a.T if a.ndim == 2 else a.transpose(0, 2, 1))

    @classmethod
    def from_synth(cls, fields, device):
        return cls(torch.from_numpy(cls.leaf_major(fields.kappa)).to(device),
                   torch.from_numpy(cls.leaf_major(fields.eps)).to(device), fields.kind == "const_eq",
                   fields.kind == "surface")


class DeviceCameras:
    def __init__(self, cams_raw: np.ndarray, device):
        self.device = torch.device(device)
        self.raw = np.ascontiguousarray(np.atleast_2d(cams_raw), np.float64)
        self.ncams = int(self.raw.shape[0])
        self.buf = torch.empty(int(L.lib().rc_camera_bytes(self.ncams)), dtype=torch.uint8, device=self.device)
        self.npix = 0
        self.wh = [(int(r[14]), int(r[15])) for r in self.raw]
        off = np.cumsum([0] + [w * h for w, h in self.wh])
        self.img_off = off.astype(np.int64)

    def image(self, t: torch.Tensor, k: int) -> torch.Tensor:
        w, h = self.wh[k]
        return t[self.img_off[k]:self.img_off[k + 1]].view(h, w)


class DeviceIndex:
    def __init__(self, device):
        self.device = torch.device(device)
        self.struct = L.RcIndex()
        self.tensors = []

    def alloc(self, cap):
        d = self.device
        self.child = _empty(cap * 8, torch.int32, d)
        self.level = _empty(cap, torch.uint8, d)
        self.x = _empty(cap, torch.int32, d)
        self.y = _empty(cap, torch.int32, d)
        self.z = _empty(cap, torch.int32, d)
        self.tree = _empty(cap, torch.uint8, d)
        s = self.struct
        s.cap_internal = max(int(cap), 1)
        s.child, s.level, s.x, s.y, s.z, s.tree = (_ptr(self.child), _ptr(self.level), _ptr(self.x), _ptr(self.y),
                                                   _ptr(self.z), _ptr(self.tree))

    @property
    def maxlevel(self):
        return int(self.struct.maxlevel)

    @property
    def ninternal(self):
        return int(self.struct.ninternal)

    def level_begin(self):
        return np.array(list(self.struct.level_begin), np.int64)

    def roots(self):
        return [int(r) for r in self.struct.roots[:int(self.struct.ntrees)]]


class VForest:
    """Buffers of rc_vforest with their capacities."""

    def __init__(self, device, nleaves, ncams, nslots, cap_vis, cap_cand, cap_rec, ninternal=0):
        d = torch.device(device)
        self.device = d
        self.cap_vis, self.cap_cand, self.cap_rec = int(cap_vis), int(cap_cand), int(cap_rec)
        self.vis_leaf = _empty(cap_vis, torch.int32, d)
        self.vis_cam = _empty(cap_vis, torch.int16, d)
        self.vis_rect = _empty(4 * cap_vis, torch.int16, d)
        self.cand_offset = _empty(cap_vis + 1, torch.int64, d)
        self.leaf_vis = _empty(ncams * nleaves, torch.int32, d)
        self.node_rect = _empty(4 * nslots, torch.int16, d)
        self.node_offset = _empty(nslots + 1, torch.int64, d)
        self.counts = torch.zeros(4, dtype=torch.int64, device=d)
        self.cand_chunk = _empty(self.cap_cand // 64 + 2, torch.int32, d)
        self.rec_chunk = _empty(self.cap_rec // 64 + 2, torch.int32, d)
        self.child_desc = _empty(ncams * max(int(ninternal), 1) * 8 * 4, torch.int32, d)  # 16 bytes per child
        self.struct = L.RcVforest(self.cap_vis, self.cap_cand, self.cap_rec, _ptr(self.vis_leaf), _ptr(self.vis_cam),
                                  _ptr(self.vis_rect), _ptr(self.cand_offset), _ptr(self.leaf_vis),
                                  _ptr(self.node_rect), _ptr(self.node_offset), _ptr(self.counts),
                                  _ptr(self.cand_chunk), _ptr(self.rec_chunk), _ptr(self.child_desc))

    def read_counts(self):
        c = self.counts.cpu().numpy()
        return {"nvis": int(c[0]), "ncand": int(c[1]), "nrec": int(c[2]), "status": int(c[3])}


# ---------------------------------------------------------------------------- entry points


def rc_camera_prepare(cams_raw, device) -> DeviceCameras:
    cams = DeviceCameras(cams_raw, device)
    npix = ctypes.c_int64(0)
    L.call("rc_camera_prepare", cams.raw.ctypes.data_as(ctypes.c_void_p), cams.ncams, _ptr(cams.buf),
           ctypes.byref(npix), _stream(cams.device))
    cams.npix = int(npix.value)
    return cams


def workspace_bytes(forest: DeviceForest, index: Optional[DeviceIndex], ncams: int, vf: Optional[VForest]) -> int:
    return int(L.lib().rc_workspace_bytes(ctypes.byref(forest.struct),
                                          ctypes.byref(index.struct) if index is not None else None, int(ncams),
                                          ctypes.byref(vf.struct) if vf is not None else None))


def rc_forest_index(forest: DeviceForest) -> DeviceIndex:
    d = forest.device
    ix = DeviceIndex(d)
    ws = _empty(workspace_bytes(forest, None, 1, None), torch.uint8, d)
    st = L.call("rc_forest_index", ctypes.byref(forest.struct), ctypes.byref(ix.struct), _ptr(ws), ws.numel(),
                _stream(d), ok=(L.RC_OK, L.RC_ECAPACITY))
    if st == L.RC_ECAPACITY or ix.struct.ninternal > 0:
        ix.alloc(max(int(ix.struct.ninternal), 1))
        L.call("rc_forest_index", ctypes.byref(forest.struct), ctypes.byref(ix.struct), _ptr(ws), ws.numel(),
               _stream(d))
    else:
        ix.alloc(1)
        L.call("rc_forest_index", ctypes.byref(forest.struct), ctypes.byref(ix.struct), _ptr(ws), ws.numel(),
               _stream(d))
    return ix


def node_slots(index: DeviceIndex, ncams: int) -> int:
    return int(L.lib().rc_node_slots(ctypes.byref(index.struct), int(ncams)))


def rc_prune_visible(forest: DeviceForest, index: DeviceIndex, cams: DeviceCameras, vf: VForest, ws: torch.Tensor):
    L.call("rc_prune_visible", ctypes.byref(forest.struct), ctypes.byref(index.struct), _ptr(cams.buf), cams.ncams,
           ctypes.byref(vf.struct), _ptr(ws), ws.numel(), _stream(forest.device))


def _tune(t: Optional[L.RcTuning]):
    return ctypes.byref(t) if t is not None else None


def rc_segments(forest: DeviceForest, fields: DeviceFields, cams: DeviceCameras, vf: VForest, method: int,
                substeps: int, rec_leaf: torch.Tensor, hit: Optional[torch.Tensor] = None,
                sio: Optional[torch.Tensor] = None, tuning: Optional[L.RcTuning] = None, c_rk: float = 0.0):
    integ = L.RcIntegrator(int(method), int(substeps), float(c_rk))
    L.call("rc_segments", ctypes.byref(forest.struct), ctypes.byref(fields.struct), _ptr(cams.buf), cams.ncams,
           ctypes.byref(vf.struct), ctypes.byref(integ), _ptr(rec_leaf), _ptr(hit), _ptr(sio), _tune(tuning),
           _stream(forest.device))


def rc_composite(forest: DeviceForest, index: DeviceIndex, cams: DeviceCameras, vf: VForest, rec_leaf, rec_node,
                 A, B, I, tuning: Optional[L.RcTuning] = None):
    L.call("rc_composite", ctypes.byref(forest.struct), ctypes.byref(index.struct), _ptr(cams.buf), cams.ncams,
           ctypes.byref(vf.struct), _ptr(rec_leaf), _ptr(rec_node), cams.npix, _ptr(A), _ptr(B), _ptr(I),
           _tune(tuning), _stream(forest.device))


def rc_render(forest: DeviceForest, index: DeviceIndex, fields: DeviceFields, cams: DeviceCameras, vf: VForest,
              method: int, substeps: int, rec_leaf, rec_node, A, B, I, tuning: Optional[L.RcTuning] = None,
              c_rk: float = 0.0):
    integ = L.RcIntegrator(int(method), int(substeps), float(c_rk))
    L.call("rc_render", ctypes.byref(forest.struct), ctypes.byref(index.struct), ctypes.byref(fields.struct),
           _ptr(cams.buf), cams.ncams, ctypes.byref(vf.struct), ctypes.byref(integ), _ptr(rec_leaf), _ptr(rec_node),
           cams.npix, _ptr(A), _ptr(B), _ptr(I), _tune(tuning), _stream(forest.device))


def rc_composite_channels(forest: DeviceForest, index: DeviceIndex, cams: DeviceCameras, vf: VForest, nch: int,
                          rec_leaf, rec_node, A, B, I, tuning: Optional[L.RcTuning] = None):
    L.call("rc_composite_channels", ctypes.byref(forest.struct), ctypes.byref(index.struct), _ptr(cams.buf),
           cams.ncams, ctypes.byref(vf.struct), int(nch), _ptr(rec_leaf), _ptr(rec_node), cams.npix, _ptr(A),
           _ptr(B), _ptr(I), _tune(tuning), _stream(forest.device))


def lists_workspace_bytes(index: DeviceIndex, ncams: int, npix: int) -> int:
    return int(L.lib().rc_lists_workspace_bytes(ctypes.byref(index.struct), int(ncams), int(npix)))


def rc_composite_lists(forest: DeviceForest, index: DeviceIndex, cams: DeviceCameras, vf: VForest, rec_leaf,
                       rec_node, list_offset, entries, n_entries, ws, tuning: Optional[L.RcTuning] = None):
    cap = entries.numel() // 4 if entries is not None else 0
    L.call("rc_composite_lists", ctypes.byref(forest.struct), ctypes.byref(index.struct), _ptr(cams.buf),
           cams.ncams, ctypes.byref(vf.struct), _ptr(rec_leaf), _ptr(rec_node), cams.npix, _ptr(list_offset),
           _ptr(entries), cap, _ptr(n_entries), _ptr(ws), ws.numel(), _tune(tuning), _stream(forest.device))


def rc_merge_lists(cams: DeviceCameras, lists, A, B, I, overlaps: Optional[torch.Tensor] = None):
    """Merge the per-pixel lists [(offsets, entries), ...] of several shares into A, B, I."""
    n = len(lists)
    if not 1 <= n <= L.RC_MAXLISTS:
        raise ValueError(f"between 1 and {L.RC_MAXLISTS} lists, got {n}")
    offs = (ctypes.c_void_p * n)(*[off.data_ptr() for off, _ in lists])
    ents = (ctypes.c_void_p * n)(*[e.data_ptr() for _, e in lists])
    L.call("rc_merge_lists", _ptr(cams.buf), cams.ncams, cams.npix, n, offs, ents, _ptr(A), _ptr(B), _ptr(I),
           _ptr(overlaps), _stream(A.device))


def merge_lists(cams: DeviceCameras, lists):
    """Images (A, B, I) and the overlap count of the merged lists of several shares."""
    dev = cams.buf.device
    A, B, I = (_empty(cams.npix, torch.float32, dev) for _ in range(3))
    ov = torch.zeros(1, dtype=torch.int64, device=dev)
    rc_merge_lists(cams, lists, A, B, I, ov)
    return A, B, I, int(ov.item())


def rc_segments_backward(forest: DeviceForest, index: DeviceIndex, fields: DeviceFields, cams: DeviceCameras,
                         vf: VForest, method: int, substeps: int, rec_leaf, rec_node, dLdI, adj_leaf, adj_node, dk,
                         de, accumulate: bool, ws, tuning: Optional[L.RcTuning] = None, c_rk: float = 0.0):
    integ = L.RcIntegrator(int(method), int(substeps), float(c_rk))
    L.call("rc_segments_backward", ctypes.byref(forest.struct), ctypes.byref(index.struct),
           ctypes.byref(fields.struct), _ptr(cams.buf), cams.ncams, ctypes.byref(vf.struct), ctypes.byref(integ),
           _ptr(rec_leaf), _ptr(rec_node), cams.npix, _ptr(dLdI), _ptr(adj_leaf), _ptr(adj_node), _ptr(dk), _ptr(de),
           1 if accumulate else 0, _ptr(ws), ws.numel(), _tune(tuning), _stream(forest.device))


# ---------------------------------------------------------------------------- renderer

METHODS = {"analytic": L.RC_INT_ANALYTIC, "rk4": L.RC_INT_RK4, "gauss2": L.RC_INT_GAUSS2,
           "simpson": L.RC_INT_SIMPSON}


class Renderer:
    """Prune, segments and composite for one forest share and a set of cameras.

    ``plan()`` sizes every buffer once (one host read-back of the device
    counts); after that ``forward()`` and ``backward()`` only enqueue work.
    """

    def __init__(self, forest, fields, cameras, method="rk4", substeps=4, device="cuda:0", index=None,
                 tuning: Optional[dict] = None, c_rk: float = 0.0, use_render: bool = False):
        self.device = torch.device(device)
        if not torch.cuda.is_available():
            raise RuntimeError("the rc renderer needs a GPU")
        L.lib()
        self.forest = forest if isinstance(forest, DeviceForest) else DeviceForest.from_synth(forest, self.device)
        self.fields = fields if isinstance(fields, DeviceFields) else DeviceFields.from_synth(fields, self.device)
        raw = cameras if isinstance(cameras, np.ndarray) else np.stack([c.raw() for c in cameras])
        self.cams = rc_camera_prepare(raw, self.device)
        # floats per record: (A, B), or two (s_in, s_out, A, B) intervals on the shell
        self.rec_floats = 8 if self.forest.curved else 2
        self.method = METHODS[method] if isinstance(method, str) else int(method)
        self.substeps = int(substeps)
        self.c_rk = float(c_rk)  # > 0: the adaptive recursion with this stability parameter
        self.index = index if index is not None else rc_forest_index(self.forest)
        self.tuning = L.RcTuning(**(tuning or {}))
        self.nslots = node_slots(self.index, self.cams.ncams)
        self.vf = None
        self.counts = None
        self.bwd_ready = False
        self.leaf_records = False  # rec_leaf holds the current fields' leaf records
        self.node_records = False  # rec_node holds every level's node records (no fold_skip)
        # forward() through rc_render (the intra-tile fold) instead of rc_segments + rc_composite
        self.use_render = bool(use_render)
        # bumped by every call that changes the fields or rewrites the records, so
        # that an autograd backward can tell whether they still belong to its forward
        self.generation = 0
        self.plan()

    # -- sizing -----------------------------------------------------------
    def plan(self, slack: float = 1.0):
        N, nc = self.forest.nleaves, self.cams.ncams
        ws = _empty(workspace_bytes(self.forest, self.index, nc, None), torch.uint8, self.device)
        caps = (0, 0, 0)
        # a pass with too little room still counts; on the curved shell the
        # node record count needs the leaf rectangles, so it settles one pass later
        for _ in range(3):
            vf = VForest(self.device, N, nc, self.nslots, *caps, self.index.ninternal)
            rc_prune_visible(self.forest, self.index, self.cams, vf, ws)
            c = vf.read_counts()
            if c["status"] == 0 and caps[0] > 0:
                break
            caps = tuple(int(c[k] * slack) + 1 for k in ("nvis", "ncand", "nrec"))
        cap_vis, cap_cand, cap_rec = caps
        self.vf = VForest(self.device, N, nc, self.nslots, cap_vis, cap_cand, cap_rec, self.index.ninternal)
        self.ws = _empty(workspace_bytes(self.forest, self.index, nc, self.vf), torch.uint8, self.device)
        nch = self.fields.nch
        self.rec_leaf = _empty(nch * self.rec_floats * cap_cand, torch.float32, self.device)
        self.rec_node = _empty(nch * self.rec_floats * max(cap_rec, 1), torch.float32, self.device)
        P = self.cams.npix
        self.A = _empty(nch * P, torch.float32, self.device)
        self.B = _empty(nch * P, torch.float32, self.device)
        self.I = _empty(nch * P, torch.float32, self.device)
        self.bwd_ready = False
        self.prune()
        self.counts = self.vf.read_counts()
        if self.counts["status"] != 0:
            raise RuntimeError(f"capacity plan failed: {self.counts}")
        return self.counts

    def _bwd_alloc(self):
        if not self.bwd_ready:
            self.adj_leaf = _empty(2 * self.vf.cap_cand, torch.float32, self.device)
            self.adj_node = _empty(2 * self.vf.cap_rec, torch.float32, self.device)
            self.bwd_ready = True

    # -- steps -------------------------------------------------------------
    def prune(self):
        rc_prune_visible(self.forest, self.index, self.cams, self.vf, self.ws)

    def segments(self, hit=None, sio=None):
        self.generation += 1
        self.leaf_records = True
        rc_segments(self.forest, self.fields, self.cams, self.vf, self.method, self.substeps, self.rec_leaf, hit, sio,
                    self.tuning, self.c_rk)

    def _tuning(self, full_records: bool):
        """The tuning for a call; full_records: with every node record (fold_skip 0)."""
        if not full_records or self.tuning.fold_skip == 0:
            return self.tuning
        t = L.RcTuning()
        ctypes.pointer(t)[0] = self.tuning
        t.fold_skip = 0
        return t

    def composite(self, full_records: bool = False):
        """rc_composite (every channel in one call); full_records: write every
        level's node records, as the adjoint needs, whatever the tuning skips."""
        self.generation += 1
        tuning = self._tuning(full_records)
        if self.fields.nch > 1:
            # every channel in one call, on the channel-major blocks
            rc_composite_channels(self.forest, self.index, self.cams, self.vf, self.fields.nch, self.rec_leaf,
                                  self.rec_node, self.A, self.B, self.I, tuning)
        else:
            rc_composite(self.forest, self.index, self.cams, self.vf, self.rec_leaf, self.rec_node, self.A, self.B,
                         self.I, tuning)
        self.node_records = tuning.fold_skip == 0 or self.fields.nch > 1

    def composite_per_channel(self):
        """rc_composite once per channel, on that channel's blocks of the records and images."""
        nl, nn, P = self.rec_floats * self.vf.cap_cand, self.rec_floats * self.vf.cap_rec, self.cams.npix
        self.generation += 1
        for ch in range(self.fields.nch):
            rc_composite(self.forest, self.index, self.cams, self.vf, self.rec_leaf[ch * nl:(ch + 1) * nl],
                         self.rec_node[ch * nn:(ch + 1) * nn], self.A[ch * P:(ch + 1) * P],
                         self.B[ch * P:(ch + 1) * P], self.I[ch * P:(ch + 1) * P], self.tuning)

    def composite_lists(self):
        """This share's per-pixel lists after prune and segments: offsets [P + 1]
        (int64) and entries [m, 4] (s_in, s_out, A, B; float32).  The entry buffer
        grows to the count on first use (one host read-back)."""
        P = self.cams.npix
        if getattr(self, "list_offset", None) is None:
            self.lists_ws = _empty(lists_workspace_bytes(self.index, self.cams.ncams, P), torch.uint8, self.device)
            self.list_offset = _empty(P + 1, torch.int64, self.device)
            self.n_entries = _empty(1, torch.int64, self.device)
            self.entries = None
        for _ in range(2):
            self.generation += 1
            rc_composite_lists(self.forest, self.index, self.cams, self.vf, self.rec_leaf, self.rec_node,
                               self.list_offset, self.entries, self.n_entries, self.lists_ws, self.tuning)
            n = int(self.n_entries.item())
            if self.entries is not None and n <= self.entries.numel() // 4:
                return self.list_offset, self.entries[:4 * n].view(n, 4)
            self.entries = _empty(4 * max(n, 1), torch.float32, self.device)
        raise RuntimeError("list entry count changed between two identical passes")

    def lists_step(self):
        """Enqueue rc_composite_lists into the buffers sized by composite_lists()."""
        self.generation += 1
        rc_composite_lists(self.forest, self.index, self.cams, self.vf, self.rec_leaf, self.rec_node,
                           self.list_offset, self.entries, self.n_entries, self.lists_ws, self.tuning)

    def forward_lists(self):
        self.prune()
        self.segments()
        return self.composite_lists()

    def forward_lists_enqueue(self):
        """prune, segments and lists into the buffers sized by composite_lists(), with no host read."""
        self.prune()
        self.segments()
        self.lists_step()

    @property
    def fused(self) -> bool:
        """rc_render folds the leaf segments in registers and LDS (no leaf records)
        for this forest, field kind, channel count and integrator."""
        return (not self.forest.curved and self.fields.nch == 1 and self.index.maxlevel >= 1
                and int(self.index.struct.root) >= 0
                and (self.method == L.RC_INT_ANALYTIC or (self.method == L.RC_INT_RK4 and self.c_rk == 0.0)))

    def render_step(self):
        """rc_render after prune: segments and compositing, fused where they can be."""
        self.generation += 1
        rc_render(self.forest, self.index, self.fields, self.cams, self.vf, self.method, self.substeps,
                  self.rec_leaf, self.rec_node, self.A, self.B, self.I, self.tuning, self.c_rk)
        self.leaf_records = not self.fused
        self.node_records = self.tuning.fold_skip == 0

    def forward(self, leaf_records: Optional[bool] = None, for_adjoint: bool = False):
        """Prune, segments and composite: rc_segments and rc_composite, which keep
        the leaf records the adjoint reads, or with leaf_records=False (default:
        not self.use_render) rc_render, which keeps them only where it cannot fuse.
        for_adjoint: keep every record the adjoint reads (leaf records, and node
        records of the levels the tuning's fold_skip would leave out)."""
        if leaf_records is None:
            leaf_records = not self.use_render
        self.prune()
        if leaf_records or for_adjoint:
            self.segments()
            self.composite(full_records=for_adjoint)
            self.leaf_records = True
        else:
            self.render_step()
        return self.A, self.B, self.I

    def backward(self, dLdI: torch.Tensor, dk: Optional[torch.Tensor] = None, de: Optional[torch.Tensor] = None,
                 accumulate=False):
        self._bwd_alloc()
        if not self.leaf_records:
            # the adjoint reads the leaf records, which rc_render's fused path does not write
            self.segments()
            self.leaf_records = True
            self.node_records = False
        if not self.node_records:
            # and every level's node records, which a fold_skip forward leaves out
            self.composite(full_records=True)
        if dk is None:
            dk = torch.empty_like(self.fields.kappa)
        if de is None:
            de = torch.empty_like(self.fields.eps)
        rc_segments_backward(self.forest, self.index, self.fields, self.cams, self.vf, self.method, self.substeps,
                             self.rec_leaf, self.rec_node, dLdI.contiguous(), self.adj_leaf, self.adj_node, dk, de,
                             accumulate, self.ws, self.tuning, self.c_rk)
        return dk, de

    # -- graph capture -----------------------------------------------------
    def capture(self, backward: bool = False, dLdI: Optional[torch.Tensor] = None):
        """Capture forward (and optionally backward with the gradient buffer dLdI)
        into a HIP graph; ``replay()`` then re-runs it with one launch."""
        if backward:
            self._bwd_alloc()
            self.g_dk = torch.empty_like(self.fields.kappa)
            self.g_de = torch.empty_like(self.fields.eps)
            self.g_dLdI = dLdI
        s = torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            for _ in range(2):
                self._graph_body(backward)
        torch.cuda.current_stream(self.device).wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._graph_body(backward)
        return self.graph

    def _graph_body(self, backward):
        self.forward(leaf_records=True if backward else None, for_adjoint=backward)
        if backward:
            self.backward(self.g_dLdI, self.g_dk, self.g_de)

    def replay(self):
        self.generation += 1
        self.graph.replay()
        return self.A, self.B, self.I

    def set_fields(self, kappa: torch.Tensor, eps: torch.Tensor):
        self.generation += 1
        self.leaf_records = False
        self.fields = DeviceFields(kappa, eps, self.fields.kind == L.RC_FIELD_CONST_EQ,
                                   self.fields.kind == L.RC_FIELD_SURFACE)

    def debug_segments(self, intervals: bool = True):
        """Run rc_segments with the pairing outputs per candidate: hits (u8; 0/1, or
        0..2 intervals on the shell) and the intervals in FP64 (2 or 4 doubles) or None."""
        n = self.vf.cap_cand
        hit = _empty(n, torch.uint8, self.device)
        sio = _empty((4 if self.forest.curved else 2) * n, torch.float64, self.device) if intervals else None
        self.segments(hit, sio)
        return hit, sio

    def count_segments(self) -> int:
        """Number of hit segments (one rc_segments pass with the hit flags)."""
        hit, _ = self.debug_segments(intervals=False)
        return int(hit[:self.counts["ncand"]].to(torch.int64).sum().item())

    def image(self, t: torch.Tensor, k: int = 0, ch: int = 0) -> torch.Tensor:
        P = self.cams.npix
        return self.cams.image(t[ch * P:(ch + 1) * P], k)


class RenderFn(torch.autograd.Function):
    """I = render(kappa, eps) with the hand-written adjoint of librc.

    The adjoint reads the renderer's records of the forward.  If the same
    renderer has changed fields or rendered again between this forward and its
    backward (two render() calls in one loss, a target rendered with other
    fields), the backward first restores this call's fields and recomputes its
    forward, so the gradient is always taken at this call's inputs."""

    @staticmethod
    def forward(ctx, kappa, eps, renderer: Renderer):
        kd, ed = kappa.detach(), eps.detach()
        renderer.set_fields(kd, ed)
        # the leaf records stay for the adjoint when a gradient is wanted
        grad = any(ctx.needs_input_grad[:2])
        _, _, I = renderer.forward(leaf_records=True if grad else None, for_adjoint=grad)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.save_for_backward(kd, ed)
        return I.clone()

    @staticmethod
    def backward(ctx, gI):
        r = ctx.renderer
        kd, ed = ctx.saved_tensors
        if r.generation != ctx.generation:
            r.set_fields(kd, ed)
            r.forward(leaf_records=True, for_adjoint=True)
        dk, de = r.backward(gI.contiguous().float())
        return dk, de, None


def render(kappa: torch.Tensor, eps: torch.Tensor, renderer: Renderer) -> torch.Tensor:
    return RenderFn.apply(kappa, eps, renderer)
