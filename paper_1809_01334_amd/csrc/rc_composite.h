// rc_composite.h -- the coarsening hierarchy as seen by compositing and its
// adjoint: the ordered fold of a node's children through the per-node child
// descriptors written by rc_prune_visible.
#pragma once

#include <stddef.h>

#include "rc_host.h"
#include "rc_internal.h"

namespace rc {

struct FoldCtx {
    const Cam* cams;
    int ncams;
    int64_t N, ninternal;
    const ChildDesc* desc;
    const int16_t* node_rect;
    const int64_t* node_offset;
    const int32_t* rec_chunk;
    const float2* rec_leaf;
    const float2* rec_node;
    const int64_t* counts;
    int64_t nslots;
    SlotLayout L;
    const int32_t* child;        // static node table: children and anchors of internal nodes
    const uint32_t *nx, *ny, *nz;
};

inline FoldCtx make_fold_ctx(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                             const rc_vforest* vf, const float* rec_leaf, const float* rec_node) {
    FoldCtx C;
    C.cams = (const Cam*)dcams;
    C.ncams = ncams;
    C.N = f->nleaves;
    C.ninternal = ix->ninternal;
    C.desc = (const ChildDesc*)vf->child_desc;
    C.node_rect = vf->node_rect;
    C.node_offset = vf->node_offset;
    C.rec_chunk = vf->rec_chunk;
    C.rec_leaf = (const float2*)rec_leaf;
    C.rec_node = (const float2*)rec_node;
    C.counts = vf->counts;
    C.L = make_layout(ix, ncams);
    C.nslots = C.L.slot_begin[ix->maxlevel > 0 ? ix->maxlevel : 0];
    C.child = ix->child;
    C.nx = ix->x;
    C.ny = ix->y;
    C.nz = ix->z;
    return C;
}

// First pixel of camera idx through the scalar cache: `idx` must be wave-uniform.
static_assert(offsetof(Cam, img_off) % 8 == 0, "img_off is read as a 64-bit word");
__device__ inline int64_t cam_img_off_scalar(const Cam* cams, int idx) {
    return (int64_t)((const_u64_ptr)(cams + idx))[offsetof(Cam, img_off) / 8];
}

// camera_of_pixel for every active lane of a wave: one search for the first
// active lane's pixel through the scalar cache; the lanes whose pixel lies in
// another image (a wave that straddles images) search on their own.
__device__ inline int camera_of_pixel_wave(const Cam* cams, int ncams, int64_t p) {
    const int64_t p0 = uniform64(p);
    int lo = 0, hi = ncams;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cam_img_off_scalar(cams, mid) <= p0)
            lo = mid;
        else
            hi = mid;
    }
    const int64_t b0 = cam_img_off_scalar(cams, lo);
    const int64_t b1 = lo + 1 < ncams ? cam_img_off_scalar(cams, lo + 1) : INT64_MAX;
    const bool in = p >= b0 && p < b1;
    if (__all(in)) return lo;
    return in ? lo : camera_of_pixel(cams, ncams, p);
}

__device__ inline bool desc_has(const ChildDesc& d, int i, int j) {
    return i >= d.i0 && i <= d.i1 && j >= d.j0 && j <= d.j1;
}

__device__ inline int64_t desc_index(const ChildDesc& d, int i, int j) {
    return (int64_t)(j - d.j0) * (d.i1 - d.i0 + 1) + (i - d.i0);
}

// Address of the record of child d at (i, j), or of the first leaf record
// (always present) when the child does not hold the pixel: every lane can
// issue all eight loads at once and select afterwards.
__device__ inline const float2* desc_ptr(const FoldCtx& C, const ChildDesc& d, bool has, int i, int j) {
    if (!has) return C.rec_leaf;
    int64_t k = desc_index(d, i, j);
    return d.off >= 0 ? C.rec_node + (d.off + k) : C.rec_leaf + (-1 - d.off + k);
}

// Group product of the children of descriptor slot `dslot` at pixel (i, j),
// nearest child first (descriptors are stored in view order).  UNIFORM: dslot
// is the same in every lane, so the descriptors come through the scalar cache.
template <bool UNIFORM>
__device__ inline float2 fold_desc(const FoldCtx& C, int64_t dslot, int i, int j) {
    ChildDesc d[8];
    if (UNIFORM) {
#pragma unroll
        for (int q = 0; q < 8; q++) d[q] = load_desc_scalar(C.desc, dslot * 8 + q);
    } else {
        const ChildDesc* dp = C.desc + dslot * 8;
#pragma unroll
        for (int q = 0; q < 8; q++) d[q] = load_desc(dp + q);
    }
    bool has[8];
    float2 rv[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        has[q] = desc_has(d[q], i, j);
        rv[q] = *desc_ptr(C, d[q], has[q], i, j);
    }
    float2 acc = make_float2(1.0f, 0.0f);
#pragma unroll
    for (int q = 0; q < 8; q++)
        if (has[q]) acc = seg_combine(acc, rv[q]);
    return acc;
}

// fold_desc, switching to scalar descriptor loads when the wave agrees on dslot
// (inactive lanes pass active = false and take part in the vote only).
__device__ inline float2 fold_desc_auto(const FoldCtx& C, int64_t dslot, bool active, int i, int j) {
    int64_t d0 = uniform64(dslot);
    if (__all(!active || dslot == d0)) return fold_desc<true>(C, d0, i, j);
    return fold_desc<false>(C, dslot, i, j);
}

// Slot of internal-node record g of level l, searched between the slots of
// its wave chunk's first and next records.
__device__ inline int64_t record_slot(const FoldCtx& C, int64_t g, int64_t w, int64_t s0, int64_t s1, int64_t Rtot) {
    int64_t lo = C.rec_chunk[w];
    if (lo < s0) lo = s0;
    int64_t hi = ((w + 1) * WAVE < Rtot) ? (int64_t)C.rec_chunk[w + 1] + 1 : s1;
    if (hi > s1) hi = s1;
    return upper_index(C.node_offset, lo, hi, g);
}

// One level pass of the coarsening (records of level l from their
// children's, folding the `run` skipped levels below l on the way) and the
// root pass into the images (walking `run` skipped levels below the root),
// as rc_composite launches them.
rc_status launch_fold_level(const FoldCtx& C, int l, int run, float* rec_node, unsigned grid, hipStream_t st);
rc_status launch_fold_root(const FoldCtx& C, int32_t root, int run, int64_t npix, float* A, float* B, float* I,
                           const rc_vforest* vf, unsigned grid, hipStream_t st);

// Node records of levels maxlevel-1 .. 1 (rc_composite.hip).
rc_status fold_levels(const FoldCtx& C, const rc_index* ix, const rc_vforest* vf, float* rec_node,
                      const rc_tuning* tune, hipStream_t st);

// The levels whose node records a unit-cube forward leaves unwritten (bits 1
// .. maxlevel - 1 of the tuning's fold_skip; none when the root is not an
// internal node), and whether no run of them exceeds RC_MAX_FOLD_RUN.
inline uint32_t fold_skip_mask(const rc_index* ix, const rc_tuning* t) {
    if (!t || ix->root < 0 || ix->maxlevel < 2) return 0;
    uint32_t levels = ((1u << ix->maxlevel) - 1u) & ~1u;
    return t->fold_skip & levels;
}
inline int skip_run(uint32_t mask, int l) {
    int d = 0;
    while (l + 1 + d < 32 && (mask & (1u << (l + 1 + d)))) d++;
    return d;
}
inline bool fold_skip_ok(uint32_t mask) {
    for (int l = 0; l < 31; l++)
        if (skip_run(mask, l) > RC_MAX_FOLD_RUN) return false;
    return true;
}

}  // namespace rc
