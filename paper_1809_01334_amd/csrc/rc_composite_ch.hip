// rc_composite_ch.hip -- sort-free compositing of several channels in one
// pass (Sec. 3.3, Sec. 2.4; each RGB channel is its own (A, B), Sec. 4.1).
// The level and root folds locate a record's node and pixel once and fold
// every channel there: one slot search, one rectangle, one set of child
// descriptors and pixel tests, and 8 x nch child records in flight.  Each
// channel's records are the group products rc_composite computes for that
// channel alone, in the same order, so they agree bit for bit.
#include "rc_composite.h"

using namespace rc;

namespace rc {
namespace {

// Record blocks of channel ch start ch * leaf_cs (leaf records) and
// ch * node_cs (node records) records in.
struct ChStrides {
    int64_t leaf_cs, node_cs;
};

// fold_desc for NCH channels at once.
template <bool UNIFORM, int NCH>
__device__ inline void fold_desc_ch(const FoldCtx& C, const ChStrides& S, int64_t dslot, int i, int j,
                                    float2 (&acc)[NCH]) {
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
    float2 rv[NCH][8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        has[q] = desc_has(d[q], i, j);
        // channel 0's record, or leaf record 0 where the child misses the pixel
        const float2* p = desc_ptr(C, d[q], has[q], i, j);
        int64_t cs = (has[q] && d[q].off >= 0) ? S.node_cs : S.leaf_cs;
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) rv[ch][q] = p[ch * cs];
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
        acc[ch] = make_float2(1.0f, 0.0f);
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (has[q]) acc[ch] = seg_combine(acc[ch], rv[ch][q]);
    }
}

template <int NCH>
__device__ inline void fold_desc_auto_ch(const FoldCtx& C, const ChStrides& S, int64_t dslot, bool active, int i,
                                         int j, float2 (&acc)[NCH]) {
    int64_t d0 = uniform64(dslot);
    if (__all(!active || dslot == d0))
        fold_desc_ch<true, NCH>(C, S, d0, i, j, acc);
    else
        fold_desc_ch<false, NCH>(C, S, dslot, i, j, acc);
}

template <int NCH>
__global__ __launch_bounds__(256) void k_fold_level_ch(FoldCtx C, ChStrides S, int l, float2* out) {
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
        float2 v[NCH];
        fold_desc_auto_ch<NCH>(C, S, cam * C.ninternal + m, act, i, j, v);
        if (act) {
#pragma unroll
            for (int ch = 0; ch < NCH; ch++) out[ch * S.node_cs + g] = v[ch];
        }
    }
}

template <int NCH>
__global__ __launch_bounds__(256) void k_fold_root_ch(FoldCtx C, ChStrides S, int32_t root, int64_t npix, float* A,
                                                      float* B, float* I, const int32_t* leaf_vis,
                                                      const int16_t* vis_rect, const int64_t* cand_offset) {
    if (C.counts[3]) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int cam = camera_of_pixel_wave(C.cams, C.ncams, p);
        const Cam& c = C.cams[cam];
        int64_t loc = p - c.img_off;
        int j = (int)(loc / c.w);
        int i = (int)(loc - (int64_t)j * c.w);
        float2 acc[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) acc[ch] = make_float2(1.0f, 0.0f);
        if (root >= 0) {
            fold_desc_auto_ch<NCH>(C, S, (int64_t)cam * C.ninternal + root, true, i, j, acc);
        } else if (root <= -2) {
            // a forest of one leaf
            int32_t v = leaf_vis[(int64_t)cam * C.N + (-2 - (int64_t)root)];
            if (v >= 0) {
                Rect r = load_rect(vis_rect + 4 * (int64_t)v);
                if (r.contains(i, j)) {
                    int64_t e = cand_offset[v] + (int64_t)(j - r.j0) * r.width() + (i - r.i0);
#pragma unroll
                    for (int ch = 0; ch < NCH; ch++) acc[ch] = C.rec_leaf[ch * S.leaf_cs + e];
                }
            }
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) {
            A[ch * npix + p] = acc[ch].x;
            B[ch * npix + p] = acc[ch].y;
            I[ch * npix + p] = fmaf(acc[ch].x, (float)c.bg, acc[ch].y);
        }
    }
}

template <int NCH>
rc_status composite_ch(const FoldCtx& C, const ChStrides& S, const rc_index* ix, const rc_vforest* vf,
                       float* rec_node, int64_t npix, float* A, float* B, float* I, const rc_tuning* tune,
                       hipStream_t st) {
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 16));
    for (int l = ix->maxlevel - 1; l >= 1; l--) {
        if (ix->level_begin[l + 1] == ix->level_begin[l]) continue;
        hipLaunchKernelGGL(k_fold_level_ch<NCH>, dim3(grid), dim3(256), 0, st, C, S, l, (float2*)rec_node);
        RC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fold_root_ch<NCH>, dim3(stride_grid(npix, 256, tuned(tune, 2, 256 * 16))), dim3(256), 0,
                       st, C, S, ix->root, npix, A, B, I, vf->leaf_vis, vf->vis_rect, vf->cand_offset);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

}  // namespace
}  // namespace rc

extern "C" rc_status rc_composite_channels(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                                           const rc_vforest* vf, int32_t nch, const float* rec_leaf,
                                           float* rec_node, int64_t npix, float* A, float* B, float* I,
                                           const rc_tuning* tune, void* stream) {
    if (nch < 1 || nch > RC_MAXCH) return RC_EINVAL;
    if (nch == 1) return rc_composite(f, ix, dcams, ncams, vf, rec_leaf, rec_node, npix, A, B, I, tune, stream);
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || npix <= 0 || !rec_leaf || !A || !B || !I || vf->cap_cand < 1) return RC_EINVAL;
    if (rc_node_slots(ix, ncams) > 0 && !rec_node) return RC_EINVAL;
    if ((s = check_tables(vf, ix, ncams)) != RC_OK) return s;
    if (is_curved(f)) {
        // interval records: one channel at a time
        int64_t lf = 8 * vf->cap_cand, nf = 8 * vf->cap_rec;
        for (int ch = 0; ch < nch; ch++) {
            s = rc_composite(f, ix, dcams, ncams, vf, rec_leaf + ch * lf, rec_node ? rec_node + ch * nf : nullptr,
                             npix, A + ch * npix, B + ch * npix, I + ch * npix, tune, stream);
            if (s != RC_OK) return s;
        }
        return RC_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    ChStrides S{vf->cap_cand, vf->cap_rec};
    if (nch == 2) return composite_ch<2>(C, S, ix, vf, rec_node, npix, A, B, I, tune, st);
    return composite_ch<3>(C, S, ix, vf, rec_node, npix, A, B, I, tune, st);
}
