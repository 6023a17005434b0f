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
        int cam = camera_of_pixel_wave(C.cams, C.ncams, p);
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

// Per-wave LDS of the walk.  top: the walked node's descriptors (view order)
// and children (natural order).  At depth d (a node with d more skipped levels
// below it) the descriptors of all eight children come in one batch, one per
// lane: bdesc[d - 1][q] holds child q's (natural order), and for d >= 2 also
// bchild[d - 1][q] its children and bbits[d - 1][q] its view bits.  A child
// is then walked from LDS, and a covered grandchild costs one round trip to
// memory (its records), not two.
struct WalkLDS {
    uint4 top[8];
    int32_t topchild[8];
    uint4 bdesc[RC_MAX_FOLD_RUN][8][8];
    int32_t bchild[RC_MAX_FOLD_RUN][8][8];
    int32_t bbits[RC_MAX_FOLD_RUN][8];
};

// The camera's view-order inputs, read once per walk.
struct WalkCam {
    double o[3], vh[3];
    int ortho;
};

__device__ inline WalkCam walk_cam(const FoldCtx& C, int cam) {
    WalkCam wc;
    const Cam& cc = C.cams[cam];
    wc.ortho = cc.ortho;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        wc.o[k] = cc.o[k];
        wc.vh[k] = cc.vh[k];
    }
    return wc;
}

__device__ inline int walk_view_bits(const WalkCam& c, int level, uint32_t x, uint32_t y, uint32_t z) {
    if (c.ortho) return (c.vh[0] < 0.0 ? 1 : 0) | (c.vh[1] < 0.0 ? 2 : 0) | (c.vh[2] < 0.0 ? 4 : 0);
    uint32_t half = 1u << (QMAX - level - 1);
    double m0 = (double)(x + half) * QSCALE;
    double m1 = (double)(y + half) * QSCALE;
    double m2 = (double)(z + half) * QSCALE;
    return (c.o[0] >= m0 ? 1 : 0) | (c.o[1] >= m1 ? 2 : 0) | (c.o[2] >= m2 ? 4 : 0);
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline ChildDesc unpack_desc(const uint4& u) {
    ChildDesc d;
    d.i0 = (int16_t)(u.x & 0xffff);
    d.i1 = (int16_t)(u.x >> 16);
    d.j0 = (int16_t)(u.y & 0xffff);
    d.j1 = (int16_t)(u.y >> 16);
    d.off = (int64_t)(((uint64_t)u.w << 32) | (uint64_t)u.z);
    return d;
}

// Value at pixel (i, j) of an internal node of level l for camera cam: the
// fold of its children's values, nearest first, from the identity -- the
// record a level pass would write there.  desc: the node's eight descriptors
// (view order), child: its children (natural order), sb: its view bits, all in
// LDS.  Children that are internal nodes within D more levels are folded here
// in turn; the others' records are read.  Every lane of the wave calls it with
// the same node; lanes with act = false load no records and take part in the
// votes only.
template <int D>
__device__ float2 walk_from(const FoldCtx& C, const WalkCam& wc, WalkLDS& S, int cam, int l, bool act, int i, int j,
                            const uint4* desc, const int32_t* child, int sb) {
    float2 acc = make_float2(1.0f, 0.0f);
    if constexpr (D == 0) {
        ChildDesc d[8];
        bool has[8];
        float2 rv[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            d[q] = unpack_desc(desc[q]);
            has[q] = act && desc_has(d[q], i, j);
            rv[q] = has[q] ? *desc_ptr(C, d[q], true, i, j) : make_float2(1.0f, 0.0f);
        }
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (has[q]) acc = seg_combine(acc, rv[q]);
    } else {
        const int lane = threadIdx.x & (WAVE - 1);
        wave_sync();  // the previous node of this depth is done with its batch
        {
            const int q = lane >> 3, qq = lane & 7;
            const int32_t cq = child[q];
            if (cq >= 0) {
                S.bdesc[D - 1][q][qq] =
                    reinterpret_cast<const uint4*>(C.desc)[((int64_t)cam * C.ninternal + cq) * 8 + qq];
                if constexpr (D >= 2) S.bchild[D - 1][q][qq] = C.child[(int64_t)cq * 8 + qq];
            }
            if constexpr (D >= 2) {
                const int32_t cl = child[lane & 7];
                if (lane < 8 && cl >= 0) S.bbits[D - 1][lane] = walk_view_bits(wc, l + 1, C.nx[cl], C.ny[cl], C.nz[cl]);
            }
        }
        wave_sync();
#pragma unroll 1
        for (int qv = 0; qv < 8; qv++) {
            ChildDesc d = unpack_desc(desc[qv]);
            bool has = act && desc_has(d, i, j);
            if (!__any(has)) continue;
            if (d.off >= 0) {
                const int q = qv ^ sb;
                float2 v;
                if constexpr (D >= 2)
                    v = walk_from<D - 1>(C, wc, S, cam, l + 1, has, i, j, S.bdesc[D - 1][q], S.bchild[D - 1][q],
                                         S.bbits[D - 1][q]);
                else
                    v = walk_from<0>(C, wc, S, cam, l + 1, has, i, j, S.bdesc[0][q], nullptr, 0);
                if (has) acc = seg_combine(acc, v);
            } else if (has) {
                acc = seg_combine(acc, C.rec_leaf[-1 - d.off + desc_index(d, i, j)]);
            }
        }
    }
    return acc;
}

// walk_from for internal node m, its descriptors, children and view bits
// loaded first (cam and m the same in every lane).
template <int D>
__device__ float2 walk_node(const FoldCtx& C, const WalkCam& wc, WalkLDS& S, int cam, int64_t m, int l, bool act,
                            int i, int j) {
    const int lane = threadIdx.x & (WAVE - 1);
    wave_sync();  // the previous walk is done with the node's slots
    if (lane < 8) {
        S.top[lane] = reinterpret_cast<const uint4*>(C.desc)[((int64_t)cam * C.ninternal + m) * 8 + lane];
        S.topchild[lane] = C.child[m * 8 + lane];
    }
    int sb = walk_view_bits(wc, l, C.nx[m], C.ny[m], C.nz[m]);
    wave_sync();
    return walk_from<D>(C, wc, S, cam, l, act, i, j, S.top, S.topchild, sb);
}

// Root pass that walks W levels below the root: node records are read from
// level W + 1 down.  A wave takes 64 consecutive pixels and walks once per
// camera among them.
template <int W>
__global__ __launch_bounds__(256) void k_fold_walk(FoldCtx C, int32_t root, int64_t npix, float* A, float* B,
                                                   float* I) {
    __shared__ WalkLDS SL[256 / WAVE];
    if (C.counts[3]) return;
    WalkLDS& S = SL[threadIdx.x / WAVE];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & (WAVE - 1);
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < npix; base += stride) {
        int64_t p = base + lane;
        bool valid = p < npix;
        int cam = 0, i = 0, j = 0;
        if (valid) {
            cam = camera_of_pixel_wave(C.cams, C.ncams, p);
            int64_t loc = p - C.cams[cam].img_off;
            int w = C.cams[cam].w;
            j = (int)(loc / w);
            i = (int)(loc - (int64_t)j * w);
        }
        bool pending = valid;
        float2 acc = make_float2(1.0f, 0.0f);
        for (;;) {
            uint64_t pm = __ballot(pending);
            if (pm == 0) break;
            int c0 = __builtin_amdgcn_readfirstlane(__shfl(cam, __ffsll((unsigned long long)pm) - 1));
            bool mine = pending && cam == c0;
            WalkCam wc = walk_cam(C, c0);
            float2 v = walk_node<W>(C, wc, S, c0, root, 0, mine, i, j);
            if (mine) {
                acc = v;
                pending = false;
            }
        }
        if (valid) {
            A[p] = acc.x;
            B[p] = acc.y;
            I[p] = fmaf(acc.x, (float)C.cams[cam].bg, acc.y);
        }
    }
}

// Level pass whose children's level is skipped: each record folds the RUN
// skipped levels below its node on the fly.  A wave walks once per node among
// its records (one or two for the large rectangles of the upper levels).
template <int RUN>
__global__ __launch_bounds__(256) void k_fold_level_walk(FoldCtx C, int l, float2* out) {
    __shared__ WalkLDS SL[256 / WAVE];
    if (C.counts[3]) return;
    WalkLDS& S = SL[threadIdx.x / WAVE];
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
        Rect r = load_rect(C.node_rect + 4 * slot);
        int k = (int)(gg - C.node_offset[slot]);
        int i, j;
        rect_pixel(r, k, i, j);
        bool pending = act;
        float2 res = make_float2(1.0f, 0.0f);
        for (;;) {
            uint64_t pm = __ballot(pending);
            if (pm == 0) break;
            int src = __ffsll((unsigned long long)pm) - 1;
            int64_t sl = uniform64(__shfl(slot, src));
            bool mine = pending && slot == sl;
            int64_t loc = sl - s0;
            int64_t cam = divu(loc, M);
            int64_t m = C.L.level_begin[l] + (loc - cam * M);
            WalkCam wc = walk_cam(C, (int)cam);
            float2 v = walk_node<RUN>(C, wc, S, (int)cam, m, l, mine, i, j);
            if (mine) {
                res = v;
                pending = false;
            }
        }
        if (act) out[g] = res;
    }
}

}  // namespace

rc_status launch_fold_level(const FoldCtx& C, int l, int run, float* rec_node, unsigned grid, hipStream_t st) {
    float2* out = (float2*)rec_node;
    switch (run) {
        case 0: hipLaunchKernelGGL(k_fold_level, dim3(grid), dim3(256), 0, st, C, l, out); break;
        case 1: hipLaunchKernelGGL(k_fold_level_walk<1>, dim3(grid), dim3(256), 0, st, C, l, out); break;
        case 2: hipLaunchKernelGGL(k_fold_level_walk<2>, dim3(grid), dim3(256), 0, st, C, l, out); break;
        default: return RC_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? RC_OK : RC_EHIP;
}

rc_status launch_fold_root(const FoldCtx& C, int32_t root, int run, int64_t npix, float* A, float* B, float* I,
                           const rc_vforest* vf, unsigned grid, hipStream_t st) {
    switch (run) {
        case 0:
            hipLaunchKernelGGL(k_fold_root, dim3(grid), dim3(256), 0, st, C, root, npix, A, B, I, vf->leaf_vis,
                               vf->vis_rect, vf->cand_offset);
            break;
        case 1: hipLaunchKernelGGL(k_fold_walk<1>, dim3(grid), dim3(256), 0, st, C, root, npix, A, B, I); break;
        case 2: hipLaunchKernelGGL(k_fold_walk<2>, dim3(grid), dim3(256), 0, st, C, root, npix, A, B, I); break;
        default: return RC_EINVAL;
    }
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
    uint32_t skip = fold_skip_mask(ix, tune);
    if (!fold_skip_ok(skip)) return RC_EINVAL;
    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 32));
    for (int l = ix->maxlevel - 1; l >= 1; l--) {
        if (ix->level_begin[l + 1] == ix->level_begin[l] || (skip & (1u << l))) continue;
        if ((s = launch_fold_level(C, l, skip_run(skip, l), rec_node, grid, st)) != RC_OK) return s;
    }
    unsigned rg = stride_grid(npix, 256, tuned(tune, 2, 256 * 16));
    return launch_fold_root(C, ix->root, skip_run(skip, 0), npix, A, B, I, vf, rg, st);
}
