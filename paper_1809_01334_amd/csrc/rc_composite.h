// rc_composite.h -- the coarsening hierarchy as seen by compositing and its
// adjoint: where a child's record of a pixel lives, and the ordered fold of
// a node's children.
#pragma once

#include "rc_host.h"
#include "rc_internal.h"

namespace rc {

struct FoldCtx {
    const Cam* cams;
    int ncams;
    int64_t N;
    const int32_t* child;
    const uint8_t* nlevel;
    const uint32_t *nx, *ny, *nz;
    const int32_t* leaf_vis;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const float2* rec_leaf;
    const int16_t* node_rect;
    const int64_t* node_offset;
    const float2* rec_node;
    const int64_t* counts;
    SlotLayout L;
};

inline FoldCtx make_fold_ctx(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                             const rc_vforest* vf, const float* rec_leaf, const float* rec_node) {
    FoldCtx C;
    C.cams = (const Cam*)dcams;
    C.ncams = ncams;
    C.N = f->nleaves;
    C.child = ix->child;
    C.nlevel = ix->level;
    C.nx = ix->x;
    C.ny = ix->y;
    C.nz = ix->z;
    C.leaf_vis = vf->leaf_vis;
    C.vis_rect = vf->vis_rect;
    C.cand_offset = vf->cand_offset;
    C.rec_leaf = (const float2*)rec_leaf;
    C.node_rect = vf->node_rect;
    C.node_offset = vf->node_offset;
    C.rec_node = (const float2*)rec_node;
    C.counts = vf->counts;
    C.L = make_layout(ix, ncams);
    return C;
}

// Location of the record of child `ref` (a slot value of a level-l node) for
// pixel (i, j) of camera `cam`: index into rec_leaf (leaf, returns 1) or
// rec_node (internal, returns 2); 0 when the child contributes nothing.
__device__ inline int child_slot(const FoldCtx& C, int cam, int32_t ref, int l, int i, int j, int64_t& idx) {
    if (ref == RC_ABSENT) return 0;
    if (ref >= 0) {
        int lc = l + 1;
        int64_t M = C.L.level_begin[lc + 1] - C.L.level_begin[lc];
        int64_t slot = C.L.slot_begin[lc] + (int64_t)cam * M + (ref - C.L.level_begin[lc]);
        Rect r = load_rect(C.node_rect + 4 * slot);
        if (!r.contains(i, j)) return 0;
        idx = C.node_offset[slot] + (int64_t)(j - r.j0) * r.width() + (i - r.i0);
        return 2;
    }
    int64_t leaf = -2 - (int64_t)ref;
    int32_t v = C.leaf_vis[(int64_t)cam * C.N + leaf];
    if (v < 0) return 0;
    Rect r = load_rect(C.vis_rect + 4 * (int64_t)v);
    if (!r.contains(i, j)) return 0;
    idx = C.cand_offset[v] + (int64_t)(j - r.j0) * r.width() + (i - r.i0);
    return 1;
}

__device__ inline float2 child_record(const FoldCtx& C, int cam, int32_t ref, int l, int i, int j) {
    int64_t idx = 0;
    int kind = child_slot(C, cam, ref, l, i, j, idx);
    if (kind == 1) return C.rec_leaf[idx];
    if (kind == 2) return C.rec_node[idx];
    return make_float2(1.0f, 0.0f);
}

// Group product of the children of internal node m (level l) at pixel (i, j),
// nearest child first.
__device__ inline float2 fold_children(const FoldCtx& C, int cam, int64_t m, int l, int i, int j) {
    int sb = view_bits(C.cams[cam], l, C.nx[m], C.ny[m], C.nz[m]);
    float2 acc = make_float2(1.0f, 0.0f);
    const int32_t* ch = C.child + m * 8;
    for (int q = 0; q < 8; q++) {
        int32_t ref = ch[q ^ sb];
        int64_t idx = 0;
        int kind = child_slot(C, cam, ref, l, i, j, idx);
        if (kind == 0) continue;
        float2 rv = (kind == 1) ? C.rec_leaf[idx] : C.rec_node[idx];
        acc = seg_combine(acc, rv);
    }
    return acc;
}

}  // namespace rc
