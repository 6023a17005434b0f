// rc_prune.hip -- visibility and work partition (Sec. 3.1 culling, Sec. 2.2
// bounding rectangles).  One scan over (camera, leaf) compacts the visible
// leaves in SFC order and prefixes their rectangle areas (the candidate
// offsets, i.e. the paper's visible-pixel weights); one scan over
// (level >= 1, camera, internal node) prefixes the record space of the
// coarsening hierarchy used by compositing.
#include <mutex>

#include "rc_host.h"
#include "rc_internal.h"
#include "rc_shell.h"
#include "rc_surface.h"
#include "rc_surface_ho.h"
#include "rc_volume.h"

namespace rc {
namespace {

// One scan over (camera, leaf) items followed by (level >= 1, camera, node)
// slots; the value counts (visible pairs, candidate records, node records).
struct Item {
    I64x3 val;
    Rect r;
};

struct PruneSrc {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    const uint8_t* nlevel;
    const uint32_t *nx, *ny, *nz;
    int64_t N, nleafitems;
    SlotLayout L;
    const double* geom;      // shell or surface table, or null for the unit cube
    int surface;             // geom holds bilinear tree patches
    int64_t tb[RC_MAXTREES + 1];
    int ntrees;
    int16_t* stash;          // every item's rectangle, for the apply pass
    __device__ Item operator()(int64_t i) const {
        Item it = compute(i);
        store_rect(stash + 4 * i, it.r);
        return it;
    }
    __device__ Item compute(int64_t i) const {
        Item it;
        double lo[3], hi[3];
        if (i < nleafitems) {
            // the camera of the wave's first item, then of this one (a wave
            // holds items of at most a few cameras)
            const int64_t i0 = uniform64(i);
            int64_t cam = divu(i0, N), l = i - cam * N;
            while (l >= N) {
                l -= N;
                cam++;
            }
            if (geom) {
                int k = 0;
                while (k + 1 < ntrees && l >= tb[k + 1]) k++;
                if (surface) {
                    it.r = surf_rect(cams[cam], geom + 12 * k, level[l], x[l], y[l]);
                } else {
                    ShellElem e = shell_elem(geom, k, level[l], x[l], y[l], z[l]);
                    it.r = shell_rect(cams[cam], e);
                }
            } else {
                node_box(level[l], x[l], y[l], z[l], lo, hi);
                int c0 = __builtin_amdgcn_readfirstlane((int)cam);
                if (__all(cam == c0)) {
                    Cam cs = load_cam_scalar(cams, c0);
                    it.r = box_rect(cs, lo, hi);
                } else {
                    it.r = box_rect(cams[cam], lo, hi);
                }
            }
            it.val = it.r.empty() ? I64x3{0, 0, 0} : I64x3{1, it.r.area(), 0};
        } else {
            // the level of the wave's first slot (a uniform search), then of
            // this one
            const int64_t s = i - nleafitems, s0 = uniform64(s);
            int lv = 1;
            while (lv < L.maxlevel && s0 >= L.slot_begin[lv + 1]) lv++;
            while (lv < L.maxlevel && s >= L.slot_begin[lv + 1]) lv++;
            int64_t M = L.level_begin[lv + 1] - L.level_begin[lv];
            int64_t loc = s - L.slot_begin[lv];
            int64_t cam = divu(loc, M);
            int64_t m = L.level_begin[lv] + (loc - cam * M);
            node_box(nlevel[m], nx[m], ny[m], nz[m], lo, hi);
            int c0 = __builtin_amdgcn_readfirstlane((int)cam);
            if (__all(cam == c0)) {
                Cam cs = load_cam_scalar(cams, c0);
                it.r = box_rect(cs, lo, hi);
            } else {
                it.r = box_rect(cams[cam], lo, hi);
            }
            it.val = I64x3{0, 0, it.r.area()};
        }
        return it;
    }
};

// Leaves of a degree-R surface forest: rectangles from the camera-space
// Bernstein coefficients of the leaf (App. A.2).
template <int R>
struct PruneSrcHo {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y;
    int64_t N;
    HoGeom G;
    int64_t tb[7];
    int ntrees;
    int16_t* stash;
    __device__ Item operator()(int64_t i) const {
        Item it;
        int64_t cam = divu(i, N), l = i - cam * N;
        int k = 0;
        while (k + 1 < ntrees && l >= tb[k + 1]) k++;
        it.r = ho_rect<R>(cams[cam], G, k, level[l], x[l], y[l]);
        it.val = it.r.empty() ? I64x3{0, 0, 0} : I64x3{1, it.r.area(), 0};
        store_rect(stash + 4 * i, it.r);
        return it;
    }
};

// Leaves of a degree-R volume forest: rectangles from the camera-space
// Bernstein coefficients of the map over the leaf's cube (App. A.2).
template <int R>
struct PruneSrcVol {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    VolGeom V;
    int64_t tb[7];
    int ntrees;
    int16_t* stash;
    __device__ Item operator()(int64_t i) const {
        Item it;
        int64_t cam = divu(i, N), l = i - cam * N;
        int k = 0;
        while (k + 1 < ntrees && l >= tb[k + 1]) k++;
        it.r = vol_rect<R>(cams[cam], V, k, level[l], x[l], y[l], z[l]);
        it.val = it.r.empty() ? I64x3{0, 0, 0} : I64x3{1, it.r.area(), 0};
        store_rect(stash + 4 * i, it.r);
        return it;
    }
};

// The apply pass reads the rectangles the reduce pass computed.
struct StashSrc {
    const int16_t* stash;
    int64_t nleafitems;
    __device__ Item operator()(int64_t i) const {
        Item it;
        it.r = load_rect(stash + 4 * i);
        if (i < nleafitems)
            it.val = it.r.empty() ? I64x3{0, 0, 0} : I64x3{1, it.r.area(), 0};
        else
            it.val = I64x3{0, 0, it.r.area()};
        return it;
    }
};

struct PruneDst {
    int64_t N, nleafitems, nslots, cap_vis, cap_cand, cap_rec;
    int32_t* vis_leaf;
    int16_t* vis_cam;
    int16_t* vis_rect;
    int64_t* cand_offset;
    int32_t* leaf_vis;
    int16_t* node_rect;
    int64_t* node_offset;
    int64_t* counts;
    __device__ void operator()(int64_t i, I64x3 pre, const Item& it) const {
        if (i < nleafitems) {
            int32_t v = -1;
            if (it.val.a && pre.a < cap_vis && pre.b + it.val.b <= cap_cand) {
                int64_t cam = divu(i, N);
                v = (int32_t)pre.a;
                vis_leaf[v] = (int32_t)(i - cam * N);
                vis_cam[v] = (int16_t)cam;
                store_rect(vis_rect + 4 * (int64_t)v, it.r);
                cand_offset[v] = pre.b;
            }
            leaf_vis[i] = v;
        } else {
            int64_t s = i - nleafitems;
            store_rect(node_rect + 4 * s, it.r);
            node_offset[s] = pre.c;
        }
    }
    __device__ void total(I64x3 t) const {
        counts[0] = t.a;
        counts[1] = t.b;
        counts[2] = t.c;
        if (t.a <= cap_vis) cand_offset[t.a] = t.b;
        if (node_offset) node_offset[nslots] = t.c;
        counts[3] = ((t.a > cap_vis || t.b > cap_cand) ? 1 : 0) | (t.c > cap_rec ? 2 : 0);
    }
};

// Curved geometry: a node's rectangle is the union of its children's, level by
// level from the deepest (the lenient boxes of curved elements do not nest).
__global__ __launch_bounds__(256) void k_union_level(const int32_t* child, const int32_t* leaf_vis,
                                                     const int16_t* vis_rect, int16_t* node_rect, int64_t N, int l,
                                                     SlotLayout L) {
    int64_t s0 = L.slot_begin[l], s1 = L.slot_begin[l + 1];
    int64_t M = L.level_begin[l + 1] - L.level_begin[l];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < s1; s += stride) {
        int64_t loc = s - s0;
        int64_t cam = divu(loc, M);
        int64_t m = L.level_begin[l] + (loc - cam * M);
        Rect u{1, 0, 1, 0};
        for (int q = 0; q < 8; q++) {
            int32_t ref = child[m * 8 + q];
            Rect r{1, 0, 1, 0};
            if (ref <= -2) {
                int32_t v = leaf_vis[cam * N + (-2 - (int64_t)ref)];
                if (v >= 0) r = load_rect(vis_rect + 4 * (int64_t)v);
            } else if (ref >= 0) {
                int lc = l + 1;
                int64_t Mc = L.level_begin[lc + 1] - L.level_begin[lc];
                r = load_rect(node_rect + 4 * (L.slot_begin[lc] + cam * Mc + (ref - L.level_begin[lc])));
            }
            if (r.empty()) continue;
            if (u.empty()) {
                u = r;
            } else {
                u.i0 = r.i0 < u.i0 ? r.i0 : u.i0;
                u.i1 = r.i1 > u.i1 ? r.i1 : u.i1;
                u.j0 = r.j0 < u.j0 ? r.j0 : u.j0;
                u.j1 = r.j1 > u.j1 ? r.j1 : u.j1;
            }
        }
        store_rect(node_rect + 4 * s, u);
    }
}

struct AreaItem {
    int64_t val;
};

struct NodeAreaSrc {
    const int16_t* node_rect;
    __device__ AreaItem operator()(int64_t s) const { return AreaItem{load_rect(node_rect + 4 * s).area()}; }
};

struct NodeAreaDst {
    int64_t nslots, cap_rec;
    int64_t* node_offset;
    int64_t* counts;
    __device__ void operator()(int64_t s, int64_t pre, const AreaItem&) const { node_offset[s] = pre; }
    __device__ void total(int64_t t) const {
        node_offset[nslots] = t;
        counts[2] = t;
        if (t > cap_rec) counts[3] |= 2;
    }
};

// table[w] = the item k whose range [off[k], off[k+1]) holds index 64 w,
// searched for one chunk.
__device__ inline void chunk_entry(const int64_t* off, int64_t n, int64_t w, int32_t* table) {
    table[w] = (int32_t)upper_index_wide(off, 0, n, w * WAVE);
}

// The same table written by the items: item k (valid in this lane) fills the chunks whose
// first index lies in its range.  Ranges of more than four chunks are filled
// by the whole wave, one item at a time.  Items with empty ranges write
// nothing, so a chunk gets the one item that holds its first index.
// Wave-uniform control: every lane of the wave calls it.
__device__ inline void chunk_scatter(const int64_t* off, int64_t k, bool valid, int64_t nchunks, int32_t* table) {
    int64_t c0 = 0, c1 = 0;
    if (valid) {
        c0 = (off[k] + WAVE - 1) / WAVE;
        c1 = (off[k + 1] + WAVE - 1) / WAVE;
        if (c1 > nchunks) c1 = nchunks;
    }
    bool big = c1 - c0 > 4;
    if (!big)
        for (int64_t c = c0; c < c1; c++) table[c] = (int32_t)k;
    uint64_t bm = __ballot(big);
    const int lane = threadIdx.x & (WAVE - 1);
    while (bm) {
        int src = __ffsll((unsigned long long)bm) - 1;
        bm &= bm - 1;
        int64_t b0 = __shfl(c0, src), b1 = __shfl(c1, src);
        int32_t bk = (int32_t)__shfl(k, src);
        for (int64_t c = b0 + lane; c < b1; c += WAVE) table[c] = bk;
    }
}

// Children of every (camera, internal node) in view order with their
// rectangles and record offsets.
struct DescArgs {
    const Cam* cams;
    int64_t N, ninternal, total;
    const int32_t* child;
    const uint32_t *nx, *ny, *nz;
    const int32_t* leaf_vis;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int16_t* node_rect;
    const int64_t* node_offset;
    const int64_t* counts;
    ChildDesc* desc;
    SlotLayout L;
    int natural;  // 1: children in Morton order (curved geometry), 0: view order
};

// Descriptors t0 .. t0 + 63 (t0 a multiple of 64, wave-uniform): lanes
// 8k .. 8k + 7 write the eight children of (camera, internal node)
// t0 / 8 + k, in view order.  A node of level >= 1 whose own rectangle is
// empty holds no record, so nothing reads its descriptors and they are not
// written; the roots' always are.  The loads that do not depend on one another
// go out together: the node's own rectangle, anchor and children (in natural
// order, then permuted to view order across the node's lanes) and the camera
// through the scalar cache when the wave has one; then the children's tables.
// lb, sb: the slot layout's level_begin and slot_begin in LDS.
__device__ inline void child_desc_wave(const DescArgs& a, const int64_t* lb, const int64_t* sb, int64_t t0,
                                       int lane) {
    const int64_t t = t0 + lane;
    const bool valid = t < a.total;
    const int q = lane & 7;
    const int64_t d0 = uniform64(t0 >> 3);
    int64_t cam = divu(d0, a.ninternal);
    int64_t m = d0 - cam * a.ninternal + (lane >> 3);
    while (m >= a.ninternal) {
        m -= a.ninternal;
        cam++;
    }
    if (!valid) cam = m = 0;  // in-bounds loads, nothing stored
    // the node's level: nodes are stored level by level, so it is the largest
    // l with lb[l] <= m (lb[0] = 0 <= m < lb[maxlevel] = ninternal)
    int l = 0;
    for (int hi = a.L.maxlevel; hi - l > 1;) {
        int mid = (l + hi) >> 1;
        if (lb[mid] <= m)
            l = mid;
        else
            hi = mid;
    }
    const uint32_t x = a.nx[m], y = a.ny[m], z = a.nz[m];
    const int32_t nat = a.child[m * 8 + q];
    // the own rectangle (of a node below the roots; the roots' slot 0 stands
    // in, read and ignored, so that the load is not behind a branch)
    Rect own{0, 0, 0, 0};
    if (a.L.maxlevel >= 2)  // there are slots
        own = load_rect(a.node_rect + 4 * (l >= 1 ? sb[l] + cam * (lb[l + 1] - lb[l]) + (m - lb[l]) : 0));
    int bits = 0;
    if (!a.natural) {
        const int64_t c0 = uniform64(cam);
        if (__all(cam == c0)) {
            Cam cs = load_cam_scalar(a.cams, (int)c0);
            bits = view_bits(cs, l, x, y, z);
        } else {
            bits = view_bits(a.cams[cam], l, x, y, z);
        }
    }
    const int32_t ref = __shfl(nat, (lane & ~7) | (q ^ bits));
    if (!valid || (l >= 1 && own.empty())) return;
    // a leaf child's pair and an internal child's slot are looked up together
    Rect r{1, 0, 1, 0};
    int64_t off = 0;
    int32_t v = -1;
    if (ref <= -2) v = a.leaf_vis[cam * a.N + (-2 - (int64_t)ref)];
    if (ref >= 0) {
        const int lc = l + 1;
        int64_t slot = sb[lc] + cam * (lb[lc + 1] - lb[lc]) + (ref - lb[lc]);
        r = load_rect(a.node_rect + 4 * slot);
        off = a.node_offset[slot];
    }
    if (v >= 0) {
        r = load_rect(a.vis_rect + 4 * (int64_t)v);
        off = -1 - a.cand_offset[v];
    }
    uint4 u;
    u.x = (uint32_t)(uint16_t)r.i0 | ((uint32_t)(uint16_t)r.i1 << 16);
    u.y = (uint32_t)(uint16_t)r.j0 | ((uint32_t)(uint16_t)r.j1 << 16);
    u.z = (uint32_t)((uint64_t)off & 0xffffffffu);
    u.w = (uint32_t)((uint64_t)off >> 32);
    *reinterpret_cast<uint4*>(a.desc + t) = u;
}

// Chunk tables of candidates and node records, then the child descriptors,
// in one grid: index ranges [0, np) for the candidate table, [np, np + ns)
// for the record table, [np + ns, end) over descriptors.  A table's items are
// its chunks (each searches the offsets) or, with `scatter`, the offsets'
// items (visible pairs or slots; each fills its chunks).  np and ns are
// multiples of the wave size, so a wave stays within one range.
__global__ __launch_bounds__(256) void k_tables(DescArgs a, int64_t nslots, int64_t np, int64_t ns,
                                                int scatter_cand, int scatter_rec, int32_t* cand_chunk,
                                                int32_t* rec_chunk) {
    if (a.counts[3]) return;
    __shared__ int64_t lb[RC_QMAXLEVEL + 2], sb[RC_QMAXLEVEL + 2];
    if (threadIdx.x < RC_QMAXLEVEL + 2) {
        lb[threadIdx.x] = a.L.level_begin[threadIdx.x];
        sb[threadIdx.x] = a.L.slot_begin[threadIdx.x];
    }
    __syncthreads();
    int64_t nvis = a.counts[0];
    int64_t w1 = (a.counts[1] + WAVE - 1) / WAVE, w2 = (a.counts[2] + WAVE - 1) / WAVE;
    int64_t end = np + ns + a.total;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & (WAVE - 1);
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < end; base += stride) {
        int64_t t = base + lane;
        if (base < np) {
            if (scatter_cand)
                chunk_scatter(a.cand_offset, t, t < nvis, w1, cand_chunk);
            else if (t < w1)
                chunk_entry(a.cand_offset, nvis, t, cand_chunk);
        } else if (base < np + ns) {
            int64_t k = t - np;
            if (scatter_rec)
                chunk_scatter(a.node_offset, k, k < nslots, w2, rec_chunk);
            else if (k < w2)
                chunk_entry(a.node_offset, nslots, k, rec_chunk);
        } else {
            child_desc_wave(a, lb, sb, base - np - ns, lane);
        }
    }
}

// A chunk table is searched per chunk while the offsets it searches stay in
// cache (probes cost little), and written from the offsets' items beyond that
// (each probe would be a memory round trip); both give the same table.
constexpr int64_t CHUNK_SEARCH_MAX_ITEMS = (int64_t)1 << 22;

}  // namespace
}  // namespace rc

using namespace rc;

namespace rc {
namespace {

rc_status check_prune_args(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                           const rc_vforest* vf) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || ncams > 32767) return RC_EINVAL;
    return check_tables(vf, ix, ncams);
}

// The prune itself, arguments validated; ws holds prune_ws_bytes() bytes
// (scan partials and the stashed rectangles, all written before they are read).
rc_status prune(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams, rc_vforest* vf, void* ws,
                hipStream_t st) {
    const Cam* cams = (const Cam*)dcams;
    int64_t N = f->nleaves;

    SlotLayout L = make_layout(ix, ncams);
    int64_t nslots = rc_node_slots(ix, ncams);
    int64_t nleafitems = N * (int64_t)ncams;
    bool shell = is_curved(f);  // node rectangles from the children's
    PruneSrc src;
    src.cams = cams;
    src.level = f->level;
    src.x = f->x;
    src.y = f->y;
    src.z = f->z;
    src.nlevel = ix->level;
    src.nx = ix->x;
    src.ny = ix->y;
    src.nz = ix->z;
    src.N = N;
    src.nleafitems = nleafitems;
    src.L = L;
    src.geom = shell ? f->geom_table : nullptr;
    src.surface = is_surface(f) ? 1 : 0;
    src.ntrees = f->ntrees;
    for (int k = 0; k <= RC_MAXTREES; k++) src.tb[k] = k <= f->ntrees ? (f->tree_begin ? f->tree_begin[k] : N) : N;
    int64_t items = shell ? nleafitems : nleafitems + nslots;
    src.stash = (int16_t*)((char*)ws + align_up(scan_partial_bytes(nleafitems + nslots, sizeof(I64x3))));
    StashSrc stash{src.stash, nleafitems};
    PruneDst dst{N,           nleafitems,      nslots,      vf->cap_vis,   vf->cap_cand,
                 vf->cap_rec, vf->vis_leaf,    vf->vis_cam, vf->vis_rect,  vf->cand_offset,
                 vf->leaf_vis, vf->node_rect,  vf->node_offset, vf->counts};
    if (!shell) {
        RC_HIP(launch_scan2<I64x3>(items, src, stash, dst, (I64x3*)ws, st));
    } else {
        // leaves first; node rectangles are unions of their children's
        int R = surface_degree(f);
        if (is_volume(f)) {
            VolGeom V;
            vol_geom_init(volume_degree(f), f->geom_table, V);
            if (volume_degree(f) == 2) {
                PruneSrcVol<2> vs{cams, f->level, f->x, f->y, f->z, N, V, {}, f->ntrees, src.stash};
                for (int k = 0; k < 7; k++) vs.tb[k] = k <= f->ntrees ? f->tree_begin[k] : N;
                RC_HIP(launch_scan2<I64x3>(items, vs, stash, dst, (I64x3*)ws, st));
            } else {
                PruneSrcVol<3> vs{cams, f->level, f->x, f->y, f->z, N, V, {}, f->ntrees, src.stash};
                for (int k = 0; k < 7; k++) vs.tb[k] = k <= f->ntrees ? f->tree_begin[k] : N;
                RC_HIP(launch_scan2<I64x3>(items, vs, stash, dst, (I64x3*)ws, st));
            }
        } else if (is_surface(f) && R > 1) {
            HoGeom G;
            ho_geom_init(R, f->geom_table, G);
            int64_t tb7[7];
            for (int k = 0; k < 7; k++) tb7[k] = k <= f->ntrees ? f->tree_begin[k] : N;
            if (R == 2) {
                PruneSrcHo<2> hs{cams, f->level, f->x, f->y, N, G, {}, f->ntrees, src.stash};
                for (int k = 0; k < 7; k++) hs.tb[k] = tb7[k];
                RC_HIP(launch_scan2<I64x3>(items, hs, stash, dst, (I64x3*)ws, st));
            } else {
                PruneSrcHo<3> hs{cams, f->level, f->x, f->y, N, G, {}, f->ntrees, src.stash};
                for (int k = 0; k < 7; k++) hs.tb[k] = tb7[k];
                RC_HIP(launch_scan2<I64x3>(items, hs, stash, dst, (I64x3*)ws, st));
            }
        } else {
            RC_HIP(launch_scan2<I64x3>(items, src, stash, dst, (I64x3*)ws, st));
        }
        for (int l = ix->maxlevel - 1; l >= 1; l--) {
            int64_t cnt = L.slot_begin[l + 1] - L.slot_begin[l];
            if (cnt == 0) continue;
            hipLaunchKernelGGL(k_union_level, dim3(stride_grid(cnt, 256, 4096)), dim3(256), 0, st, ix->child,
                               vf->leaf_vis, vf->vis_rect, vf->node_rect, N, l, L);
            RC_HIP(hipGetLastError());
        }
        if (nslots > 0) {
            NodeAreaSrc as{vf->node_rect};
            NodeAreaDst ad{nslots, vf->cap_rec, vf->node_offset, vf->counts};
            RC_HIP(launch_scan<int64_t>(nslots, as, ad, (int64_t*)ws, st));
        }
    }

    DescArgs da{cams,          N,            ix->ninternal,   ix->ninternal * ncams * 8,
                ix->child,     ix->x,        ix->y,           ix->z,
                vf->leaf_vis,  vf->vis_rect, vf->cand_offset,
                vf->node_rect, vf->node_offset, vf->counts,   (ChildDesc*)vf->child_desc,
                L,             shell ? 1 : 0};
    int sc = vf->cap_vis > CHUNK_SEARCH_MAX_ITEMS, sr = nslots > CHUNK_SEARCH_MAX_ITEMS;
    int64_t np = sc ? vf->cap_vis : vf->cap_cand / WAVE + 1;
    int64_t ns = nslots == 0 ? 0 : (sr ? nslots : vf->cap_rec / WAVE + 1);
    np = (np + WAVE - 1) / WAVE * WAVE;
    ns = (ns + WAVE - 1) / WAVE * WAVE;
    hipLaunchKernelGGL(k_tables, dim3(stride_grid(np + ns + da.total, 256, 256 * 32)), dim3(256), 0, st, da, nslots,
                       np, ns, sc, sr, vf->cand_chunk, vf->rec_chunk);
    RC_HIP(hipGetLastError());
    return RC_OK;
}

// Workspace of the allocation-free prune: one array per device, holding the
// last call's partials and rectangles until the process ends.
__device__ __align__(256) unsigned char scratch[RC_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES];

// Device address of the current device's scratch array, looked up once per
// device (the array's name is only a host-side stand-in for it).
rc_status scratch_ptr(void** out) {
    int dev = -1;
    RC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return RC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RC_EHIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return RC_OK;
}

}  // namespace
}  // namespace rc

extern "C" rc_status rc_prune_visible(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                                      rc_vforest* vf, void* ws, size_t ws_bytes, void* stream) {
    rc_status s = check_prune_args(f, ix, dcams, ncams, vf);
    if (s != RC_OK) return s;
    if (!ws || ws_bytes < rc_workspace_bytes(f, ix, ncams, nullptr)) return RC_EWORKSPACE;
    return prune(f, ix, dcams, ncams, vf, ws, (hipStream_t)stream);
}

extern "C" rc_status rc_prune_visible_static(const rc_forest* f, const rc_index* ix, const void* dcams,
                                             int32_t ncams, rc_vforest* vf, void* stream) {
    rc_status s = check_prune_args(f, ix, dcams, ncams, vf);
    if (s != RC_OK) return s;
    if (prune_ws_bytes(f, ix, ncams) > RC_STATIC_SCRATCH_BYTES) return RC_EWORKSPACE;
    void* ws = nullptr;
    if ((s = scratch_ptr(&ws)) != RC_OK) return s;
    return prune(f, ix, dcams, ncams, vf, ws, (hipStream_t)stream);
}
