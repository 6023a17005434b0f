// rc_prune.hip -- visibility and work partition (Sec. 3.1 culling, Sec. 2.2
// bounding rectangles).  One scan over (camera, leaf) compacts the visible
// leaves in SFC order and prefixes their rectangle areas (the candidate
// offsets, i.e. the paper's visible-pixel weights); one scan over
// (level >= 1, camera, internal node) prefixes the record space of the
// coarsening hierarchy used by compositing.
#include "rc_host.h"
#include "rc_internal.h"

namespace rc {
namespace {

struct LeafItem {
    I64x2 val;  // (visible, rectangle area)
    Rect r;
};

struct LeafSrc {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    __device__ LeafItem operator()(int64_t i) const {
        int64_t cam = i / N, l = i - cam * N;
        double lo[3], hi[3];
        node_box(level[l], x[l], y[l], z[l], lo, hi);
        LeafItem it;
        it.r = box_rect(cams[cam], lo, hi);
        it.val = it.r.empty() ? I64x2{0, 0} : I64x2{1, it.r.area()};
        return it;
    }
};

struct LeafDst {
    int64_t N, cap_vis, cap_cand;
    int32_t* vis_leaf;
    int16_t* vis_cam;
    int16_t* vis_rect;
    int64_t* cand_offset;
    int32_t* leaf_vis;
    int64_t* counts;
    __device__ void operator()(int64_t i, I64x2 pre, const LeafItem& it) const {
        int32_t v = -1;
        if (it.val.a && pre.a < cap_vis && pre.b + it.val.b <= cap_cand) {
            int64_t cam = i / N;
            v = (int32_t)pre.a;
            vis_leaf[v] = (int32_t)(i - cam * N);
            vis_cam[v] = (int16_t)cam;
            store_rect(vis_rect + 4 * (int64_t)v, it.r);
            cand_offset[v] = pre.b;
        }
        leaf_vis[i] = v;
    }
    __device__ void total(I64x2 t) const {
        counts[0] = t.a;
        counts[1] = t.b;
        if (t.a <= cap_vis) cand_offset[t.a] = t.b;
        counts[3] = (t.a > cap_vis || t.b > cap_cand) ? 1 : 0;
    }
};

struct NodeItem {
    int64_t val;  // rectangle area
    Rect r;
};

struct NodeSrc {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    SlotLayout L;
    __device__ NodeItem operator()(int64_t s) const {
        int l = 1;
        while (l < L.maxlevel && s >= L.slot_begin[l + 1]) l++;
        int64_t M = L.level_begin[l + 1] - L.level_begin[l];
        int64_t loc = s - L.slot_begin[l];
        int64_t cam = loc / M;
        int64_t m = L.level_begin[l] + (loc - cam * M);
        double lo[3], hi[3];
        node_box(level[m], x[m], y[m], z[m], lo, hi);
        NodeItem it;
        it.r = box_rect(cams[cam], lo, hi);
        it.val = it.r.area();
        return it;
    }
};

struct NodeDst {
    int64_t nslots, cap_rec;
    int16_t* node_rect;
    int64_t* node_offset;
    int64_t* counts;
    __device__ void operator()(int64_t s, int64_t pre, const NodeItem& it) const {
        store_rect(node_rect + 4 * s, it.r);
        node_offset[s] = pre;
    }
    __device__ void total(int64_t t) const {
        node_offset[nslots] = t;
        counts[2] = t;
        if (t > cap_rec) counts[3] |= 2;
    }
};

__global__ void k_empty_nodes(int64_t* node_offset, int64_t* counts) {
    if (node_offset) node_offset[0] = 0;
    counts[2] = 0;
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_prune_visible(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                                      rc_vforest* vf, void* ws, size_t ws_bytes, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || ncams > 32767) return RC_EINVAL;
    if (!ws || ws_bytes < rc_workspace_bytes(f, ix, ncams, nullptr)) return RC_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const Cam* cams = (const Cam*)dcams;
    int64_t N = f->nleaves;

    LeafSrc ls{cams, f->level, f->x, f->y, f->z, N};
    LeafDst ld{N, vf->cap_vis, vf->cap_cand, vf->vis_leaf, vf->vis_cam, vf->vis_rect, vf->cand_offset, vf->leaf_vis,
               vf->counts};
    RC_HIP(launch_scan<I64x2>(N * (int64_t)ncams, ls, ld, (I64x2*)ws, st));

    SlotLayout L = make_layout(ix, ncams);
    int64_t nslots = rc_node_slots(ix, ncams);
    NodeSrc ns{cams, ix->level, ix->x, ix->y, ix->z, L};
    NodeDst nd{nslots, vf->cap_rec, vf->node_rect, vf->node_offset, vf->counts};
    if (nslots > 0) {
        RC_HIP(launch_scan<int64_t>(nslots, ns, nd, (int64_t*)ws, st));
    } else {
        // no internal node below the roots: the record space is empty
        hipLaunchKernelGGL(k_empty_nodes, dim3(1), dim3(1), 0, st, vf->node_offset, vf->counts);
        RC_HIP(hipGetLastError());
    }
    return RC_OK;
}
