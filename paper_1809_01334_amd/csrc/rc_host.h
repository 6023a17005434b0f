// rc_host.h -- host-side helpers shared by the entry points of librc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc.h"
#include "rc_internal.h"

namespace rc {

constexpr int WAVE = 64;
constexpr int GRAD_MAX = 16;  // 8 kappa + 8 eps corners per leaf

inline size_t align_up(size_t b, size_t a = 256) { return (b + a - 1) / a * a; }

// Workspace of rc_segments_backward: per-(wave chunk, visible pair) gradient
// partials.
inline size_t backward_ws_bytes(int64_t cap_cand, int64_t cap_vis, int64_t ncams, int64_t N) {
    (void)ncams;
    (void)N;
    int64_t nchunks = (cap_cand + WAVE - 1) / WAVE;
    return align_up((size_t)(nchunks + cap_vis + 1) * GRAD_MAX * sizeof(float));
}

// Workspace of rc_prune_visible: partials of the joint scan over (camera,
// leaf) items and node slots, then every item's rectangle (8 bytes).
inline size_t prune_ws_bytes(const rc_forest* f, const rc_index* ix, int32_t ncams) {
    int64_t nc = ncams > 0 ? ncams : 1;
    int64_t items = f->nleaves * nc + (ix ? rc_node_slots(ix, ncams) : 0);
    return align_up(scan_partial_bytes(items, sizeof(I64x3))) + align_up((size_t)items * 8);
}

#define RC_HIP(call)                                 \
    do {                                             \
        if ((call) != hipSuccess) return RC_EHIP;    \
    } while (0)

inline rc_status check_forest(const rc_forest* f) {
    if (!f || f->nleaves < 1 || !f->level || !f->x || !f->y || !f->z) return RC_EINVAL;
    if (f->geom == RC_GEOM_UNIT_CUBE) {
        if (f->ntrees != 1) return RC_EUNSUPPORTED;
    } else if (f->geom == RC_GEOM_SHELL6) {
        if (f->ntrees != 6 || !f->geom_table || !f->tree_begin) return RC_EINVAL;
    } else if (f->geom == RC_GEOM_SURFACE || f->geom == RC_GEOM_SURFACE2 || f->geom == RC_GEOM_SURFACE3 ||
               f->geom == RC_GEOM_VOLUME2 || f->geom == RC_GEOM_VOLUME3) {
        if (f->ntrees < 1 || f->ntrees > 6 || !f->geom_table || !f->tree_begin) return RC_EINVAL;
    } else {
        return RC_EUNSUPPORTED;
    }
    if (f->tree_begin) {
        if (f->tree_begin[0] != 0 || f->tree_begin[f->ntrees] != f->nleaves) return RC_EINVAL;
        for (int k = 0; k < f->ntrees; k++)
            if (f->tree_begin[k + 1] < f->tree_begin[k]) return RC_EINVAL;
    }
    if (f->nleaves > (int64_t)0x7ffffffe) return RC_EUNSUPPORTED;
    return RC_OK;
}

inline bool is_shell(const rc_forest* f) { return f->geom == RC_GEOM_SHELL6; }
inline bool is_surface(const rc_forest* f) {
    return f->geom == RC_GEOM_SURFACE || f->geom == RC_GEOM_SURFACE2 || f->geom == RC_GEOM_SURFACE3;
}
// Degree of a surface forest's tree maps (1: bilinear).
inline int surface_degree(const rc_forest* f) {
    return f->geom == RC_GEOM_SURFACE2 ? 2 : f->geom == RC_GEOM_SURFACE3 ? 3 : 1;
}
inline bool is_volume(const rc_forest* f) { return f->geom == RC_GEOM_VOLUME2 || f->geom == RC_GEOM_VOLUME3; }
// Degree of a volume forest's tree maps.
inline int volume_degree(const rc_forest* f) { return f->geom == RC_GEOM_VOLUME3 ? 3 : 2; }
// Geometries whose records hold two depth-tagged intervals and whose node
// rectangles are unions of the children's.
inline bool is_curved(const rc_forest* f) { return is_shell(f) || is_surface(f) || is_volume(f); }

// Curved six-tree shell variants of rc_segments and rc_composite (arguments
// already validated by the entry points).
rc_status rc_shell_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                            const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                            const rc_tuning* tune, hipStream_t st);
rc_status rc_shell_composite(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                             const rc_vforest* vf, const float* rec_leaf, float* rec_node, int64_t npix, float* A,
                             float* B, float* I, const rc_tuning* tune, hipStream_t st);
// Surface forests: segments (rc_surface.hip); compositing is the shell's with
// zero-length intervals.
rc_status rc_surface_ho_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                 const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                                 const rc_tuning* tune, hipStream_t st);
rc_status rc_volume_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                             const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                             const rc_tuning* tune, hipStream_t st);
rc_status rc_surface_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                              const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                              const rc_tuning* tune, hipStream_t st);

// Workspace layout of rc_forest_index.
constexpr size_t IX_STATUS = 0, IX_COUNT = 64, IX_TREES = 256, IX_ROOTS = 1280, IX_CUR = 1536;

inline rc_status check_index(const rc_index* ix) {
    if (!ix || !ix->child || !ix->level || !ix->x || !ix->y || !ix->z) return RC_EINVAL;
    if (ix->maxlevel < 0 || ix->maxlevel > RC_QMAXLEVEL) return RC_EINVAL;
    if (ix->ninternal > ix->cap_internal) return RC_ECAPACITY;
    return RC_OK;
}

inline rc_status check_vforest(const rc_vforest* vf, bool need_nodes) {
    if (!vf || !vf->vis_leaf || !vf->vis_cam || !vf->vis_rect || !vf->cand_offset || !vf->leaf_vis || !vf->counts)
        return RC_EINVAL;
    if (need_nodes && (!vf->node_rect || !vf->node_offset)) return RC_EINVAL;
    if (vf->cap_vis < 0 || vf->cap_cand < 0 || vf->cap_rec < 0) return RC_EINVAL;
    // the chunk table holds pair indices as int32
    if (vf->cap_vis > (int64_t)0x7ffffffe) return RC_EUNSUPPORTED;
    return RC_OK;
}

inline rc_status check_fields(const rc_fields* fl, const rc_integrator* in) {
    if (!fl || !fl->kappa || !fl->eps || !in) return RC_EINVAL;
    if (fl->nch < 1 || fl->nch > RC_MAXCH) return RC_EINVAL;
    if (fl->kind != RC_FIELD_CONST && fl->kind != RC_FIELD_TRILINEAR && fl->kind != RC_FIELD_CONST_EQ &&
        fl->kind != RC_FIELD_SURFACE)
        return RC_EUNSUPPORTED;
    if (fl->kind == RC_FIELD_SURFACE) return in->method == RC_INT_ANALYTIC ? RC_OK : RC_EUNSUPPORTED;
    if (in->method == RC_INT_ANALYTIC) {
        if (fl->kind == RC_FIELD_TRILINEAR) return RC_EUNSUPPORTED;
        return RC_OK;
    }
    if (in->method != RC_INT_RK4 && in->method != RC_INT_GAUSS2 && in->method != RC_INT_SIMPSON)
        return RC_EUNSUPPORTED;
    if (fl->kind == RC_FIELD_CONST_EQ) return RC_EUNSUPPORTED;
    if (in->substeps < 1 || in->substeps > 64) return RC_EINVAL;
    if (!(in->c_rk >= 0.0)) return RC_EINVAL;  // also rejects NaN
    bool dyadic = in->method != RC_INT_RK4 || in->c_rk > 0.0;
    if (dyadic && (in->substeps & (in->substeps - 1))) return RC_EINVAL;
    return RC_OK;
}

// The hand-written adjoint covers (kappa, eps) fields with the closed form,
// with RK4, Gauss or Simpson over equal pieces (1, 2, 4 or 8, checked by the
// entry point) and with the recursion of any of the three, and (kappa, I)
// equilibrium fields with the closed form.
inline bool adjoint_supported(const rc_fields* fl, const rc_integrator* in) {
    (void)in;
    return fl->kind != RC_FIELD_SURFACE;
}

// Integrators beyond the closed form and fixed-step RK4: rc_integrators.hip.
rc_status rc_segments_general(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                              const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                              const rc_tuning* tune, hipStream_t st);
// Leaf adjoint of the recursion (c_rk > 0): per (chunk, pair) partials as the
// fixed-piece leaf adjoint writes them (rc_integrators.hip).
rc_status rc_adjoint_pieces(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                            const rc_integrator* in, const float* adj_leaf, float* partial, const rc_tuning* tune,
                            hipStream_t st);

// The per-call tables written by rc_prune_visible and read by later calls.
inline rc_status check_tables(const rc_vforest* vf, const rc_index* ix, int32_t ncams) {
    if (!vf->cand_chunk) return RC_EINVAL;
    // the record chunk table stores (level, camera, node) slot indices as int32
    if (rc_node_slots(ix, ncams) > (int64_t)0x7ffffffe) return RC_EUNSUPPORTED;
    if (ix->maxlevel >= 1 && ncams > 0 && (int64_t)ncams * (ix->level_begin[ix->maxlevel] - ix->level_begin[1]) > 0 &&
        !vf->rec_chunk)
        return RC_EINVAL;
    if (ix->ninternal > 0 && !vf->child_desc) return RC_EINVAL;
    return RC_OK;
}

inline unsigned tuned(const rc_tuning* t, int which, unsigned dflt) {
    if (!t) return dflt;
    int32_t v = which == 0 ? t->seg_blocks : which == 1 ? t->fold_blocks : which == 2 ? t->root_blocks : t->adj_blocks;
    return v > 0 ? (unsigned)v : dflt;
}

// Slot layout of internal nodes of level >= 1: (level, camera, node).
struct SlotLayout {
    int64_t level_begin[RC_QMAXLEVEL + 2];
    int64_t slot_begin[RC_QMAXLEVEL + 2];
    int32_t maxlevel;
    int32_t ncams;
};

inline SlotLayout make_layout(const rc_index* ix, int32_t ncams) {
    SlotLayout L;
    L.maxlevel = ix->maxlevel;
    L.ncams = ncams;
    for (int l = 0; l < RC_QMAXLEVEL + 2; l++) {
        int ll = l <= ix->maxlevel ? l : ix->maxlevel;
        L.level_begin[l] = ix->level_begin[ll];
    }
    for (int l = 0; l < RC_QMAXLEVEL + 2; l++) {
        int ll = l < 1 ? 1 : l;
        L.slot_begin[l] = (int64_t)ncams * (L.level_begin[ll] - L.level_begin[1]);
    }
    return L;
}

}  // namespace rc
