// rc_lists.hip -- one process's share composited to per-pixel lists, and the
// merge of several shares' lists.
//
// A share is a contiguous curve-order range of a forest's leaves.  Its maximal
// complete subtrees are the coarsest nodes all of whose leaves it holds
// (Sec. 3.3: coarsening stops where the share ends); each meets a ray in one
// interval, so a pixel's part of the share is a short depth-ordered list of
// (s_in, s_out, A, B) entries, one per subtree the ray crosses (Sec. 3.5
// per-pixel segment lists, here in a compressed-row layout).  Merging the
// shares' lists by depth and folding them nearest first gives the image of
// the whole forest; where rounding makes two entries overlap, they are cut
// (eq. segsplit) and the overlap averaged (eq. segaverage).
#include "rc_composite.h"

namespace rc {
namespace {

// complete[m]: the curve interval of node m lies inside the share's, from its
// first leaf's anchor to the end of its last leaf; the share's leaves tile that
// interval, so m's leaves are all in the share.
__global__ __launch_bounds__(256) void k_complete(const uint8_t* nlevel, const uint32_t* nx, const uint32_t* ny,
                                                  const uint32_t* nz, int64_t nint, const uint8_t* level,
                                                  const uint32_t* x, const uint32_t* y, const uint32_t* z, int64_t N,
                                                  uint8_t* complete) {
    uint64_t S = morton(x[0], y[0], z[0]);
    uint64_t E = morton(x[N - 1], y[N - 1], z[N - 1]) + curve_span(level[N - 1]);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < nint; m += stride) {
        uint64_t k0 = morton(nx[m], ny[m], nz[m]);
        complete[m] = (k0 >= S && k0 + curve_span(nlevel[m]) <= E) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_zero_i32(int64_t n, int32_t* p) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// Unit items: (camera, internal node m, child slot c) for m not complete, and
// one root item per camera.  A unit is a leaf or a complete node under an
// incomplete parent, or the root when it is complete (or a leaf).
enum { U_NONE = 0, U_LEAF = 1, U_NODE = 2, U_ROOT = 3 };

struct UnitArgs {
    const Cam* cams;
    int ncams;
    int64_t N, ninternal;
    int32_t root;
    const int32_t* child;
    const uint8_t* complete;
    const uint8_t* nlevel;
    const uint32_t *nx, *ny, *nz;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    const int32_t* leaf_vis;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int16_t* node_rect;
    const int64_t* node_offset;
    SlotLayout L;
};

struct Unit {
    int kind;
    int cam;
    int64_t id;    // leaf or node index
    int64_t rec0;  // first record of the unit's rectangle (leaf or node records)
};

__device__ inline Unit unit_of(const UnitArgs& a, int64_t t) {
    Unit u{U_NONE, 0, 0, 0};
    int64_t per = a.ninternal * 8;
    int64_t base = per * a.ncams;
    int32_t ref;
    if (t < base) {
        int64_t cam = divu(t, per);
        int64_t rem = t - cam * per;
        int64_t m = rem >> 3;
        u.cam = (int)cam;
        if (a.complete[m]) return u;
        ref = a.child[m * 8 + (rem & 7)];
        if (ref >= 0 && !a.complete[ref]) return u;
    } else {
        u.cam = (int)(t - base);
        ref = a.root;
        if (ref >= 0 && !a.complete[ref]) return u;
        if (ref >= 0) {
            u.kind = U_ROOT;
            u.id = ref;
            return u;
        }
    }
    if (ref == RC_ABSENT) return u;
    if (ref <= -2) {
        int64_t leaf = -2 - (int64_t)ref;
        int32_t v = a.leaf_vis[(int64_t)u.cam * a.N + leaf];
        if (v < 0) return u;
        u.kind = U_LEAF;
        u.id = leaf;
        u.rec0 = a.cand_offset[v];
        return u;
    }
    int lv = a.nlevel[ref];
    int64_t M = a.L.level_begin[lv + 1] - a.L.level_begin[lv];
    int64_t slot = a.L.slot_begin[lv] + (int64_t)u.cam * M + (ref - a.L.level_begin[lv]);
    u.kind = U_NODE;
    u.id = ref;
    u.rec0 = a.node_offset[slot];
    return u;
}

__device__ inline Rect unit_rect(const UnitArgs& a, const Unit& u) {
    Rect r{1, 0, 1, 0};
    if (u.kind == U_LEAF) {
        int32_t v = a.leaf_vis[(int64_t)u.cam * a.N + u.id];
        r = load_rect(a.vis_rect + 4 * (int64_t)v);
    } else if (u.kind == U_NODE) {
        int lv = a.nlevel[u.id];
        int64_t M = a.L.level_begin[lv + 1] - a.L.level_begin[lv];
        int64_t slot = a.L.slot_begin[lv] + (int64_t)u.cam * M + (u.id - a.L.level_begin[lv]);
        r = load_rect(a.node_rect + 4 * slot);
    } else if (u.kind == U_ROOT) {
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {1.0, 1.0, 1.0};
        r = box_rect(a.cams[u.cam], lo, hi);
    }
    return r;
}

__device__ inline void unit_box(const UnitArgs& a, const Unit& u, double lo[3], double hi[3]) {
    if (u.kind == U_LEAF)
        node_box(a.level[u.id], a.x[u.id], a.y[u.id], a.z[u.id], lo, hi);
    else
        node_box(a.nlevel[u.id], a.nx[u.id], a.ny[u.id], a.nz[u.id], lo, hi);
}

struct UItem {
    int64_t val;
};

// Scan source: the unit's rectangle area, the rectangle stashed for the passes.
// Nothing is read past the visibility tables when they overflowed.
struct UnitSrc {
    UnitArgs a;
    const int64_t* counts;
    int16_t* stash;
    __device__ UItem operator()(int64_t t) const {
        Unit u = counts[3] ? Unit{U_NONE, 0, 0, 0} : unit_of(a, t);
        Rect r = u.kind == U_NONE ? Rect{1, 0, 1, 0} : unit_rect(a, u);
        store_rect(stash + 4 * t, r);
        return UItem{r.area()};
    }
};

struct UnitStashSrc {
    const int16_t* stash;
    __device__ UItem operator()(int64_t t) const { return UItem{load_rect(stash + 4 * t).area()}; }
};

struct UnitDst {
    int64_t nitems;
    int64_t* off;  // nitems + 1
    __device__ void operator()(int64_t t, int64_t pre, const UItem&) const { off[t] = pre; }
    __device__ void total(int64_t tot) const { off[nitems] = tot; }
};

// Per-pixel counts to list offsets.
struct CountSrc {
    const int32_t* cnt;
    __device__ UItem operator()(int64_t p) const { return UItem{cnt[p]}; }
};

struct CountDst {
    int64_t npix;
    int64_t* off;
    int64_t* n_entries;
    __device__ void operator()(int64_t p, int64_t pre, const UItem&) const { off[p] = pre; }
    __device__ void total(int64_t tot) const {
        off[npix] = tot;
        *n_entries = tot;
    }
};

struct PassArgs {
    UnitArgs a;
    FoldCtx C;
    int64_t nitems;
    const int64_t* uoff;
    const int16_t* stash;
    int32_t* cnt;
    const int64_t* loff;
    float4* entries;
    int64_t cap;
};

// FILL = false: count each pixel's entries; true: write them.
template <bool FILL>
__global__ __launch_bounds__(256) void k_unit_pixels(PassArgs P) {
    if (P.C.counts[3]) return;
    int64_t total = P.uoff[P.nitems];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
        int64_t t = upper_index_wide(P.uoff, 0, P.nitems, q);
        Unit u = unit_of(P.a, t);
        Rect r = load_rect(P.stash + 4 * t);
        int k = (int)(q - P.uoff[t]);
        int i, j;
        rect_pixel(r, k, i, j);
        const Cam& c = P.a.cams[u.cam];
        double lo[3], hi[3], rho[3], rr[3], s_in, s_out;
        if (u.kind == U_ROOT) {
            for (int d = 0; d < 3; d++) {
                lo[d] = 0.0;
                hi[d] = 1.0;
            }
        } else {
            unit_box(P.a, u, lo, hi);
        }
        pixel_ray(c, i, j, rho, rr);
        if (!slab_hit(c, rho, rr, lo, hi, s_in, s_out)) continue;
        int64_t pg = c.img_off + (int64_t)j * c.w + i;
        if (!FILL) {
            atomicAdd(&P.cnt[pg], 1);
            continue;
        }
        int pos = atomicSub(&P.cnt[pg], 1) - 1;  // the count pass left cnt[pg] slots
        int64_t e = P.loff[pg] + pos;
        if (e >= P.cap) continue;
        float2 ab;
        if (u.kind == U_LEAF)
            ab = P.C.rec_leaf[u.rec0 + k];
        else if (u.kind == U_NODE)
            ab = P.C.rec_node[u.rec0 + k];
        else
            ab = fold_desc<false>(P.C, (int64_t)u.cam * P.C.ninternal + u.id, i, j);
        P.entries[e] = make_float4((float)s_in, (float)s_out, ab.x, ab.y);
    }
}

__device__ inline bool entry_less(const float4& a, const float4& b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    if (a.z != b.z) return a.z < b.z;
    return a.w < b.w;
}

// Each pixel's entries into depth order (a total order on the entry values,
// so the result does not depend on the order the fill pass wrote them in).
__global__ __launch_bounds__(256) void k_sort_lists(int64_t npix, const int64_t* loff, float4* entries, int64_t cap) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int64_t b = loff[p], e = loff[p + 1];
        if (e > cap) continue;
        for (int64_t q = b + 1; q < e; q++) {
            float4 v = entries[q];
            int64_t s = q - 1;
            while (s >= b && entry_less(v, entries[s])) {
                entries[s + 1] = entries[s];
                s--;
            }
            entries[s + 1] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// merge
// ---------------------------------------------------------------------------

constexpr int MAXLISTS = RC_MAXLISTS;

struct MergeArgs {
    const Cam* cams;
    int ncams;
    int64_t npix;
    int nlists;
    const int64_t* off[MAXLISTS];
    const float4* ent[MAXLISTS];
    float *A, *B, *I;
    unsigned long long* overlaps;
};

// eq. segsplit: the piece of (A, B) over the fraction f of its length, A^f and
// B (1 - A^f) / (1 - A), the ratio taken as expm1(f ln A) / expm1(ln A) so
// that it stays accurate as A approaches 1 (where it tends to f).  An opaque
// segment (A = 0) gives (0, B) for any f > 0.  Returns ln A^f in *lnpiece.
__device__ inline float2 seg_piece(float2 s, float f, float* lnpiece) {
    if (f >= 1.0f) {
        *lnpiece = logf(s.x);
        return s;
    }
    float la = logf(s.x);
    float ratio = la == 0.0f ? f : expm1f(f * la) / expm1f(la);
    *lnpiece = f * la;
    return make_float2(expf(f * la), s.y * ratio);
}

__device__ inline float4 list_head(const float4* e, int64_t h, int64_t end) {
    return h < end ? e[h] : make_float4(INFINITY, INFINITY, 1.0f, 0.0f);
}

// One pixel per thread.  Every list is sorted and holds disjoint entries, so
// each list has at most one entry covering the sweep position (act[k], live
// while its s_out lies beyond pos).  The sweep advances to the nearest entry
// start or active end; over the elementary interval it crossed, each active
// entry contributes its piece (eq. segsplit) and several are averaged (the
// geometric mean of the A, the arithmetic mean of the B: eq. segaverage over
// all covering entries); the result is folded nearest first (eq. aggregate).
// A zero-length entry is folded whole at its depth.  NL: lists rounded up to
// a power of two (the rest are empty).
template <int NL>
__global__ __launch_bounds__(256) void k_merge_lists(MergeArgs M) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M.npix; p += stride) {
        int64_t head[NL], end[NL];
        float4 nxt[NL], act[NL];
#pragma unroll
        for (int k = 0; k < NL; k++) {
            head[k] = k < M.nlists ? M.off[k][p] : 0;
            end[k] = k < M.nlists ? M.off[k][p + 1] : 0;
            nxt[k] = k < M.nlists ? list_head(M.ent[k], head[k], end[k]) : list_head(nullptr, 0, 0);
            act[k] = make_float4(0.0f, -INFINITY, 1.0f, 0.0f);
        }
        float2 acc = make_float2(1.0f, 0.0f);
        float pos = -INFINITY;
        unsigned ov = 0;
        bool bad = false;
        for (;;) {
            float ns = INFINITY, ne = INFINITY;
#pragma unroll
            for (int k = 0; k < NL; k++) {
                ns = fminf(ns, nxt[k].x);
                if (act[k].y > pos) ne = fminf(ne, act[k].y);
            }
            float nb = fminf(ns, ne);
            if (!(nb < INFINITY)) break;
            if (nb > pos) {
                float lnA = 0.0f, sumB = 0.0f;
                float2 one = make_float2(1.0f, 0.0f);
                int n = 0;
#pragma unroll
                for (int k = 0; k < NL; k++) {
                    if (act[k].y > pos) {
                        float lp;
                        one = seg_piece(make_float2(act[k].z, act[k].w), (nb - pos) / (act[k].y - act[k].x), &lp);
                        lnA += lp;
                        sumB += one.y;
                        n++;
                    }
                }
                if (n == 1)
                    acc = seg_combine(acc, one);
                else if (n > 1)
                    acc = seg_combine(acc, make_float2(expf(lnA / (float)n), sumB / (float)n));
                pos = nb;
            }
            if (ns != pos) continue;
            // start the least entry beginning here, in (s_in, s_out, A, B) order
            int best = -1;
            float4 x = make_float4(INFINITY, INFINITY, 1.0f, 0.0f);
#pragma unroll
            for (int k = 0; k < NL; k++)
                if (nxt[k].x == pos && (best < 0 || entry_less(nxt[k], x))) {
                    best = k;
                    x = nxt[k];
                }
            bool others = false;
#pragma unroll
            for (int k = 0; k < NL; k++) {
                if (k == best) {
                    head[k]++;
                    nxt[k] = list_head(M.ent[k], head[k], end[k]);
                    if (act[k].y > pos && x.y > x.x) bad = true;  // the list's entries overlap
                    if (x.y > x.x) act[k] = x;
                } else if (act[k].y > pos) {
                    others = true;
                }
            }
            if (!(x.y > x.x))
                acc = seg_combine(acc, make_float2(x.z, x.w));
            else if (others)
                ov++;
        }
        if (bad) acc = make_float2(NAN, NAN);
        int cam = camera_of_pixel_wave(M.cams, M.ncams, p);
        M.A[p] = acc.x;
        M.B[p] = acc.y;
        M.I[p] = fmaf(acc.x, (float)M.cams[cam].bg, acc.y);
        if (ov && M.overlaps) atomicAdd(M.overlaps, (unsigned long long)ov);
    }
}

}  // namespace
}  // namespace rc

using namespace rc;

namespace {

struct ListsLayout {
    size_t complete, uoff, stash, cnt, partial, total;
};

ListsLayout lists_layout(const rc_index* ix, int32_t ncams, int64_t npix) {
    ListsLayout L;
    int64_t nitems = ix->ninternal * 8 * (int64_t)ncams + ncams;
    size_t o = 0;
    L.complete = o;
    o += align_up((size_t)(ix->ninternal > 0 ? ix->ninternal : 1));
    L.uoff = o;
    o += align_up((size_t)(nitems + 1) * 8);
    L.stash = o;
    o += align_up((size_t)nitems * 8);
    L.cnt = o;
    o += align_up((size_t)npix * 4);
    L.partial = o;
    size_t p1 = scan_partial_bytes(nitems, 8), p2 = scan_partial_bytes(npix, 8);
    o += align_up(p1 > p2 ? p1 : p2);
    L.total = o;
    return L;
}

}  // namespace

extern "C" size_t rc_lists_workspace_bytes(const rc_index* ix, int32_t ncams, int64_t total_pixels) {
    if (!ix || ncams <= 0 || total_pixels <= 0) return 0;
    return lists_layout(ix, ncams, total_pixels).total + 256;
}

extern "C" rc_status rc_composite_lists(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                                        const rc_vforest* vf, const float* rec_leaf, float* rec_node, int64_t npix,
                                        int64_t* list_offset, float* entries, int64_t cap_entries,
                                        int64_t* n_entries, void* ws, size_t ws_bytes, const rc_tuning* tune,
                                        void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if (is_curved(f)) return RC_EUNSUPPORTED;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || npix <= 0 || !rec_leaf || !list_offset || !n_entries || cap_entries < 0 ||
        (cap_entries > 0 && !entries) || vf->cap_cand < 1)
        return RC_EINVAL;
    if (rc_node_slots(ix, ncams) > 0 && !rec_node) return RC_EINVAL;
    if ((s = check_tables(vf, ix, ncams)) != RC_OK) return s;
    if (!ws || ws_bytes < rc_lists_workspace_bytes(ix, ncams, npix)) return RC_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    if ((s = fold_levels(C, ix, vf, rec_node, tune, st)) != RC_OK) return s;

    ListsLayout WL = lists_layout(ix, ncams, npix);
    char* w = (char*)ws;
    uint8_t* complete = (uint8_t*)(w + WL.complete);
    int64_t* uoff = (int64_t*)(w + WL.uoff);
    int16_t* stash = (int16_t*)(w + WL.stash);
    int32_t* cnt = (int32_t*)(w + WL.cnt);
    void* partial = (void*)(w + WL.partial);

    if (ix->ninternal > 0) {
        hipLaunchKernelGGL(k_complete, dim3(stride_grid(ix->ninternal, 256, 4096)), dim3(256), 0, st, ix->level,
                           ix->x, ix->y, ix->z, ix->ninternal, f->level, f->x, f->y, f->z, f->nleaves, complete);
        RC_HIP(hipGetLastError());
    }
    UnitArgs ua;
    ua.cams = (const Cam*)dcams;
    ua.ncams = ncams;
    ua.N = f->nleaves;
    ua.ninternal = ix->ninternal;
    ua.root = ix->root;
    ua.child = ix->child;
    ua.complete = complete;
    ua.nlevel = ix->level;
    ua.nx = ix->x;
    ua.ny = ix->y;
    ua.nz = ix->z;
    ua.level = f->level;
    ua.x = f->x;
    ua.y = f->y;
    ua.z = f->z;
    ua.leaf_vis = vf->leaf_vis;
    ua.vis_rect = vf->vis_rect;
    ua.cand_offset = vf->cand_offset;
    ua.node_rect = vf->node_rect;
    ua.node_offset = vf->node_offset;
    ua.L = make_layout(ix, ncams);
    int64_t nitems = ix->ninternal * 8 * (int64_t)ncams + ncams;
    RC_HIP(launch_scan2<int64_t>(nitems, UnitSrc{ua, vf->counts, stash}, UnitStashSrc{stash}, UnitDst{nitems, uoff},
                                 (int64_t*)partial, st));
    int64_t ng = (int64_t)npix;
    hipLaunchKernelGGL(k_zero_i32, dim3(stride_grid(ng, 256, 4096)), dim3(256), 0, st, ng, cnt);
    RC_HIP(hipGetLastError());
    PassArgs P{ua, C, nitems, uoff, stash, cnt, list_offset, (float4*)entries, cap_entries};
    unsigned grid = stride_grid(vf->cap_cand + npix, 256, tuned(tune, 0, 256 * 8));
    hipLaunchKernelGGL((k_unit_pixels<false>), dim3(grid), dim3(256), 0, st, P);
    RC_HIP(hipGetLastError());
    RC_HIP(launch_scan<int64_t>(ng, CountSrc{cnt}, CountDst{ng, list_offset, n_entries}, (int64_t*)partial, st));
    if (cap_entries > 0) {
        hipLaunchKernelGGL((k_unit_pixels<true>), dim3(grid), dim3(256), 0, st, P);
        RC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sort_lists, dim3(stride_grid(ng, 256, 4096)), dim3(256), 0, st, ng,
                           (const int64_t*)list_offset, (float4*)entries, cap_entries);
        RC_HIP(hipGetLastError());
    }
    return RC_OK;
}

extern "C" rc_status rc_merge_lists(const void* dcams, int32_t ncams, int64_t npix, int32_t nlists,
                                    const int64_t* const* list_offsets, const float* const* entries, float* A,
                                    float* B, float* I, int64_t* overlaps, void* stream) {
    if (!dcams || ncams <= 0 || npix <= 0 || nlists < 1 || nlists > RC_MAXLISTS || !list_offsets || !entries ||
        !A || !B || !I)
        return RC_EINVAL;
    MergeArgs M;
    M.cams = (const Cam*)dcams;
    M.ncams = ncams;
    M.npix = npix;
    M.nlists = nlists;
    for (int k = 0; k < RC_MAXLISTS; k++) {
        if (k < nlists && (!list_offsets[k] || !entries[k])) return RC_EINVAL;
        M.off[k] = k < nlists ? list_offsets[k] : nullptr;
        M.ent[k] = k < nlists ? (const float4*)entries[k] : nullptr;
    }
    M.A = A;
    M.B = B;
    M.I = I;
    M.overlaps = (unsigned long long*)overlaps;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid(stride_grid(npix, 256, 4096)), block(256);
    if (nlists <= 2)
        hipLaunchKernelGGL(k_merge_lists<2>, grid, block, 0, st, M);
    else if (nlists <= 4)
        hipLaunchKernelGGL(k_merge_lists<4>, grid, block, 0, st, M);
    else if (nlists <= 8)
        hipLaunchKernelGGL(k_merge_lists<8>, grid, block, 0, st, M);
    else
        hipLaunchKernelGGL(k_merge_lists<16>, grid, block, 0, st, M);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
