// rc_composite.hip -- sort-free compositing by octree coarsening (Sec. 3.3,
// Sec. 2.4).  Level by level from the deepest, the record of an internal
// node at a pixel is the group product of its children's records taken in
// the camera's view order; children that are absent, invisible or whose
// rectangle misses the pixel act as the identity (segments separated by
// empty space may be combined, Sec. 2.4).  The tree roots are folded straight
// into the images, where I = A I_b + B (Sec. 2.4, final intensity).
#include "rc_composite.h"

using namespace rc;

namespace rc {
namespace {

__global__ __launch_bounds__(256) void k_fold_level(FoldCtx C, int l, float2* out) {
    if (C.counts[3]) return;
    int64_t s0 = C.L.slot_begin[l], s1 = C.L.slot_begin[l + 1];
    int64_t R0 = C.node_offset[s0], R1 = C.node_offset[s1], Rtot = C.node_offset[C.nslots];
    int64_t M = C.L.level_begin[l + 1] - C.L.level_begin[l];
    int lane = threadIdx.x & (WAVE - 1);
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t w = R0 / WAVE + wave; w * WAVE < R1; w += nw) {
        int64_t g = w * WAVE + lane;
        bool act = g >= R0 && g < R1;
        int64_t gg = act ? g : (g < R0 ? R0 : R1 - 1);
        int64_t slot = record_slot(C, gg, w, s0, s1, Rtot);
        int64_t loc = slot - s0;
        int64_t cam = divu(loc, M);
        int64_t m = C.L.level_begin[l] + (loc - cam * M);
        Rect r = load_rect(C.node_rect + 4 * slot);
        int k = (int)(gg - C.node_offset[slot]);
        int i, j;
        rect_pixel(r, k, i, j);
        float2 v = fold_desc_auto(C, cam * C.ninternal + m, act, i, j);
        if (act) out[g] = v;
    }
}

__global__ __launch_bounds__(256) void k_fold_root(FoldCtx C, int32_t root, int64_t npix, float* A, float* B,
                                                   float* I, const int32_t* leaf_vis, const int16_t* vis_rect,
                                                   const int64_t* cand_offset) {
    if (C.counts[3]) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int cam = camera_of_pixel(C.cams, C.ncams, p);
        const Cam& c = C.cams[cam];
        int64_t loc = p - c.img_off;
        int j = (int)(loc / c.w);
        int i = (int)(loc - (int64_t)j * c.w);
        float2 acc = make_float2(1.0f, 0.0f);
        if (root >= 0) {
            acc = fold_desc_auto(C, (int64_t)cam * C.ninternal + root, true, i, j);
        } else if (root <= -2) {
            // a forest of one leaf
            int32_t v = leaf_vis[(int64_t)cam * C.N + (-2 - (int64_t)root)];
            if (v >= 0) {
                Rect r = load_rect(vis_rect + 4 * (int64_t)v);
                if (r.contains(i, j)) acc = C.rec_leaf[cand_offset[v] + (int64_t)(j - r.j0) * r.width() + (i - r.i0)];
            }
        }
        A[p] = acc.x;
        B[p] = acc.y;
        I[p] = fmaf(acc.x, (float)c.bg, acc.y);
    }
}

}  // namespace

rc_status launch_fold_level(const FoldCtx& C, int l, float* rec_node, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_level, dim3(grid), dim3(256), 0, st, C, l, (float2*)rec_node);
    return hipGetLastError() == hipSuccess ? RC_OK : RC_EHIP;
}

rc_status launch_fold_root(const FoldCtx& C, int32_t root, int64_t npix, float* A, float* B, float* I,
                           const rc_vforest* vf, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_fold_root, dim3(grid), dim3(256), 0, st, C, root, npix, A, B, I, vf->leaf_vis,
                       vf->vis_rect, vf->cand_offset);
    return hipGetLastError() == hipSuccess ? RC_OK : RC_EHIP;
}

// Node records of levels maxlevel-1 .. 1, deepest first.
rc_status fold_levels(const FoldCtx& C, const rc_index* ix, const rc_vforest* vf, float* rec_node,
                      const rc_tuning* tune, hipStream_t st) {
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 32));
    for (int l = ix->maxlevel - 1; l >= 1; l--) {
        if (ix->level_begin[l + 1] == ix->level_begin[l]) continue;
        hipLaunchKernelGGL(k_fold_level, dim3(grid), dim3(256), 0, st, C, l, (float2*)rec_node);
        RC_HIP(hipGetLastError());
    }
    return RC_OK;
}

}  // namespace rc

extern "C" rc_status rc_composite(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                                  const rc_vforest* vf, const float* rec_leaf, float* rec_node, int64_t npix,
                                  float* A, float* B, float* I, const rc_tuning* tune, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || npix <= 0 || !rec_leaf || !A || !B || !I || vf->cap_cand < 1) return RC_EINVAL;
    if (rc_node_slots(ix, ncams) > 0 && !rec_node) return RC_EINVAL;
    if ((s = check_tables(vf, ix, ncams)) != RC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (is_curved(f)) return rc_shell_composite(f, ix, dcams, ncams, vf, rec_leaf, rec_node, npix, A, B, I, tune, st);
    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    if ((s = fold_levels(C, ix, vf, rec_node, tune, st)) != RC_OK) return s;
    hipLaunchKernelGGL(k_fold_root, dim3(stride_grid(npix, 256, tuned(tune, 2, 256 * 16))), dim3(256), 0, st, C,
                       ix->root, npix, A,
                       B, I, vf->leaf_vis, vf->vis_rect, vf->cand_offset);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
