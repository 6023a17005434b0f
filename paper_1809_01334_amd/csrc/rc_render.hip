// rc_render.hip -- the forward of a unit-cube forest with one pass per level
// of the coarsening (Sec. 3.2 ray segments, Sec. 3.3 coarsening and
// aggregation).  The pass of level l computes the records of the level's
// internal nodes; where a child of such a node is a leaf, the pass pairs the
// leaf with the pixel's ray and integrates the segment right there (the
// intra-tile fold):
//
//  * a wave takes 64 records (node, pixel); each lane marks the leaf children
//    whose rectangle holds its pixel;
//  * the marked (lane, child) items are compacted into an LDS list by a wave
//    prefix sum, so that pairing runs with every lane busy whatever the
//    coverage;
//  * hits queue in LDS and are integrated 64 at a time (RK4), and each item's
//    (A, B) lands in its LDS slot (an identity on a miss);
//  * every lane then folds its children in the camera's view order (Sec. 2.4,
//    eq. aggregate): leaf children from LDS, internal children from the
//    records of the level below.
//
// Segment values and the order of the group products are those of
// rc_segments followed by rc_composite, so the images agree bit for bit; no
// leaf record is written or read.
#include "rc_composite.h"

namespace rc {
namespace {

struct RenderArgs {
    FoldCtx C;
    const int32_t* child;          // node table: 8 child slots per internal node
    const uint32_t *nx, *ny, *nz;  // internal node anchors
    const float *kappa, *eps;
    int nsub;
    int eq;                        // closed form with the equilibrium intensity in place of eps
    int32_t root;                  // internal index of the tree's root
    int64_t npix;
    float *A, *B, *I;
};

constexpr int RQ = 128;           // a batch of 64 items adds at most 64 hits to fewer than 64 queued
constexpr int RITEMS = 8 * WAVE;  // at most 8 leaf children per record

// Per-wave LDS: the item slots (a key, owner lane << 3 | view position, until
// the item's (A, B) replaces it) and the hit queue.
struct RenderLDS {
    float2 slot[RITEMS];
    uint16_t qk[RQ];  // item slot of a queued hit
    int32_t qleaf[RQ];
    float qxf0[RQ], qxf1[RQ], qxf2[RQ], qd0[RQ], qd1[RQ], qd2[RQ], qdx[RQ];
};

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix sum over the wave; every lane takes part.
__device__ inline int wave_prefix(int v, int lane, int& total) {
    int x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    total = __shfl(x, WAVE - 1);
    return x - v;
}

// An item's key travels in its slot's first float, bits unchanged.
__device__ inline void put_key(RenderLDS& S, int k, int key) { S.slot[k] = make_float2(__int_as_float(key), 0.0f); }
__device__ inline int get_key(const RenderLDS& S, int k) { return __float_as_int(S.slot[k].x); }

// Segment of queued hit e (KIND 1: constant coefficients through RK4; 2: trilinear).
template <int KIND, int NSUB>
__device__ inline void drain_one(const RenderArgs& a, RenderLDS& S, int e) {
    SegGeom sg;
    sg.xf[0] = S.qxf0[e];
    sg.xf[1] = S.qxf1[e];
    sg.xf[2] = S.qxf2[e];
    sg.dxi[0] = S.qd0[e];
    sg.dxi[1] = S.qd1[e];
    sg.dxi[2] = S.qd2[e];
    sg.dx = S.qdx[e];
    int64_t leaf = S.qleaf[e];
    float2 ab;
    if (KIND == 1) {
        ab = seg_rk4_const<NSUB>(a.kappa[leaf], a.eps[leaf], sg.dx, a.nsub);
    } else {
        float kc[8], ec[8];
        const float4* kp = reinterpret_cast<const float4*>(a.kappa + leaf * 8);
        const float4* ep = reinterpret_cast<const float4*>(a.eps + leaf * 8);
        float4 k0 = kp[0], k1 = kp[1], e0 = ep[0], e1 = ep[1];
        kc[0] = k0.x; kc[1] = k0.y; kc[2] = k0.z; kc[3] = k0.w;
        kc[4] = k1.x; kc[5] = k1.y; kc[6] = k1.z; kc[7] = k1.w;
        ec[0] = e0.x; ec[1] = e0.y; ec[2] = e0.z; ec[3] = e0.w;
        ec[4] = e1.x; ec[5] = e1.y; ec[6] = e1.z; ec[7] = e1.w;
        ab = seg_rk4<NSUB>(kc, ec, sg, a.nsub);
    }
    S.slot[S.qk[e]] = ab;
}

// Pairing of one item: the pixel's ray against the leaf child c of node m
// (level lc = level of m + 1), the same operations as rc_segments' pairing.
template <int MODE>
__device__ inline bool pair_child(const Cam& c, int i, int j, int lc, uint32_t ax, uint32_t ay, uint32_t az,
                                  double lo[3], double rho[3], double r[3], double& s_in, double& s_out) {
    double hi[3];
    node_box(lc, ax, ay, az, lo, hi);
    pixel_ray<MODE>(c, i, j, rho, r);
    return slab_hit(c, rho, r, lo, hi, s_in, s_out);
}

// The records of a window of 64 lanes: lane state (active, camera, pixel,
// internal node m at level l).  Returns the lane's record.
template <int KIND, int NSUB>
__device__ inline float2 render_window(const RenderArgs& a, RenderLDS& S, bool act, int cam, int i, int j, int32_t m,
                                       int l, int lane) {
    const FoldCtx& C = a.C;
    int64_t dslot = (int64_t)cam * C.ninternal + m;
    ChildDesc d[8];
    int64_t d0 = uniform64(dslot);
    if (__all(!act || dslot == d0)) {
#pragma unroll
        for (int q = 0; q < 8; q++) d[q] = load_desc_scalar(C.desc, d0 * 8 + q);
    } else {
        const ChildDesc* dp = C.desc + dslot * 8;
#pragma unroll
        for (int q = 0; q < 8; q++) d[q] = load_desc(dp + q);
    }
    bool has[8];
    unsigned leafmask = 0;
    float2 rv[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        has[q] = act && desc_has(d[q], i, j);
        rv[q] = make_float2(1.0f, 0.0f);
        if (has[q]) {
            if (d[q].off >= 0)
                rv[q] = C.rec_node[d[q].off + desc_index(d[q], i, j)];
            else
                leafmask |= 1u << q;
        }
    }
    int total;
    int base = wave_prefix(__popc(leafmask), lane, total);
    if (total > 0) {
        // view bits of the lane's node: child at view position q is q ^ s
        const Cam& cm = C.cams[cam];
        int sbits = view_bits(cm, l, a.nx[m], a.ny[m], a.nz[m]);
        {
            unsigned mm = leafmask;
            int k = base;
            while (mm) {
                int q = __ffs(mm) - 1;
                mm &= mm - 1;
                put_key(S, k++, (lane << 3) | q);
            }
        }
        wave_lds_sync();
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
        int qn = 0;
        const int lc = l + 1;
        const uint32_t half = 1u << (QMAX - lc);
        for (int b0 = 0; b0 < total; b0 += WAVE) {
            int k = b0 + lane;
            bool valid = k < total;
            int key = valid ? get_key(S, k) : 0;
            int o = key >> 3, q = key & 7;
            int ocam = __shfl(cam, o), oi = __shfl(i, o), oj = __shfl(j, o), om = __shfl(m, o);
            int os = __shfl(sbits, o);
            bool h = false;
            SegGeom sg;
            int32_t leaf = 0;
            int32_t ref = valid ? a.child[(int64_t)om * 8 + (q ^ os)] : 0;
            // the descriptor at view position q is a leaf, so ref is one; anything else pairs nothing
            valid = valid && ref <= -2;
            if (valid) {
                int cc = q ^ os;
                leaf = -2 - ref;
                uint32_t ax = a.nx[om] + ((cc & 1) ? half : 0u);
                uint32_t ay = a.ny[om] + ((cc & 2) ? half : 0u);
                uint32_t az = a.nz[om] + ((cc & 4) ? half : 0u);
                double lo[3], rho[3], rr[3], s_in, s_out;
                int c0 = __builtin_amdgcn_readfirstlane(ocam);
                bool hit;
                if (__all(!valid || ocam == c0)) {
                    Cam cs = load_cam_scalar(C.cams, c0);
                    if (cs.ortho)
                        hit = pair_child<1>(cs, oi, oj, lc, ax, ay, az, lo, rho, rr, s_in, s_out);
                    else
                        hit = pair_child<0>(cs, oi, oj, lc, ax, ay, az, lo, rho, rr, s_in, s_out);
                } else {
                    hit = pair_child<-1>(C.cams[ocam], oi, oj, lc, ax, ay, az, lo, rho, rr, s_in, s_out);
                }
                float2 ab = make_float2(1.0f, 0.0f);
                if (hit) {
                    sg = seg_geom(rho, rr, s_in, s_out, lo, lc);
                    if (KIND == 0) {
                        float kk = a.kappa[leaf], ee = a.eps[leaf];
                        ab = a.eq ? seg_const_eq(kk, ee, sg.dx) : seg_const(kk, ee, sg.dx);
                    } else {
                        h = true;
                    }
                }
                if (!h) S.slot[k] = ab;
            } else if (k < total) {
                S.slot[k] = make_float2(1.0f, 0.0f);
            }
            if (KIND != 0) {
                uint64_t mask = __ballot(h);
                if (h) {
                    int pos = qn + __popcll(mask & below);
                    S.qk[pos] = (uint16_t)k;
                    S.qleaf[pos] = leaf;
                    S.qxf0[pos] = sg.xf[0];
                    S.qxf1[pos] = sg.xf[1];
                    S.qxf2[pos] = sg.xf[2];
                    S.qd0[pos] = sg.dxi[0];
                    S.qd1[pos] = sg.dxi[1];
                    S.qd2[pos] = sg.dxi[2];
                    S.qdx[pos] = sg.dx;
                }
                qn += __popcll(mask);
                wave_lds_sync();
                if (qn >= WAVE) {
                    drain_one<KIND, NSUB>(a, S, qn - WAVE + lane);
                    qn -= WAVE;
                    wave_lds_sync();
                }
            }
        }
        if (KIND != 0 && lane < qn) drain_one<KIND, NSUB>(a, S, lane);
        wave_lds_sync();
    }
    float2 acc = make_float2(1.0f, 0.0f);
    int r = base;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        if (has[q]) {
            float2 v = rv[q];
            if (d[q].off < 0) v = S.slot[r++];
            acc = seg_combine(acc, v);
        }
    }
    // the slots are reused by the next window
    wave_lds_sync();
    return acc;
}

// One pass of the coarsening: level l >= 1 writes the records of the level's
// nodes; level 0 folds the root into the images, one lane per pixel.
template <int KIND, int NSUB>
__global__ __launch_bounds__(256) void k_render_level(RenderArgs a, int l, float2* out) {
    __shared__ RenderLDS LDSW[256 / WAVE];
    const FoldCtx& C = a.C;
    if (C.counts[3]) return;
    int lane = threadIdx.x & (WAVE - 1);
    RenderLDS& S = LDSW[threadIdx.x / WAVE];
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    if (l == 0) {
        for (int64_t w = wave; w * WAVE < a.npix; w += nw) {
            int64_t p = w * WAVE + lane;
            bool act = p < a.npix;
            int64_t pp = act ? p : a.npix - 1;
            int cam = camera_of_pixel_wave(C.cams, C.ncams, pp);
            const Cam& c = C.cams[cam];
            int64_t loc = pp - c.img_off;
            int j = (int)(loc / c.w);
            int i = (int)(loc - (int64_t)j * c.w);
            float2 acc = render_window<KIND, NSUB>(a, S, act, cam, i, j, a.root, 0, lane);
            if (act) {
                a.A[p] = acc.x;
                a.B[p] = acc.y;
                a.I[p] = fmaf(acc.x, (float)c.bg, acc.y);
            }
        }
        return;
    }
    int64_t s0 = C.L.slot_begin[l], s1 = C.L.slot_begin[l + 1];
    int64_t R0 = C.node_offset[s0], R1 = C.node_offset[s1], Rtot = C.node_offset[C.nslots];
    int64_t M = C.L.level_begin[l + 1] - C.L.level_begin[l];
    for (int64_t w = R0 / WAVE + wave; w * WAVE < R1; w += nw) {
        int64_t g = w * WAVE + lane;
        bool act = g >= R0 && g < R1;
        int64_t gg = act ? g : (g < R0 ? R0 : R1 - 1);
        int64_t slot = record_slot(C, gg, w, s0, s1, Rtot);
        int64_t loc = slot - s0;
        int64_t cam = divu(loc, M);
        int32_t m = (int32_t)(C.L.level_begin[l] + (loc - cam * M));
        Rect rc = load_rect(C.node_rect + 4 * slot);
        int k = (int)(gg - C.node_offset[slot]);
        int i, j;
        rect_pixel(rc, k, i, j);
        float2 v = render_window<KIND, NSUB>(a, S, act, (int)cam, i, j, m, l, lane);
        if (act) out[g] = v;
    }
}

template <int KIND, int NSUB>
rc_status launch_render(const RenderArgs& a, const rc_index* ix, const rc_vforest* vf, float* rec_node,
                        const rc_tuning* tune, hipStream_t st) {
    // passes whose children include no leaf are plain folds
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 2048));
    unsigned fgrid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 32));
    unsigned rgrid = stride_grid(a.npix, 256, tuned(tune, 2, 4096));
    // skipped levels stay skipped only where the walk over them reaches no
    // leaf: the leaves' records are not written here
    uint32_t skip = fold_skip_mask(ix, tune);
    if (!fold_skip_ok(skip)) return RC_EINVAL;
    for (int l = 0; l < ix->maxlevel; l++) {
        int d = skip_run(skip, l);
        if (d == 0 || (l > 0 && (skip & (1u << l)))) continue;  // l heads a run of skipped levels below it
        uint32_t reach = ((2u << (l + d + 1)) - 1u) & ~((2u << l) - 1u);  // levels l+1 .. l+d+1
        if (ix->leaf_levels & reach) skip &= ~(((2u << (l + d)) - 1u) & ~((2u << l) - 1u));
    }
    for (int l = ix->maxlevel - 1; l >= 1; l--) {
        if (ix->level_begin[l + 1] == ix->level_begin[l] || (skip & (1u << l))) continue;
        if (ix->leaf_levels & (1 << (l + 1))) {
            hipLaunchKernelGGL((k_render_level<KIND, NSUB>), dim3(grid), dim3(256), 0, st, a, l, (float2*)rec_node);
            RC_HIP(hipGetLastError());
        } else {
            rc_status s = launch_fold_level(a.C, l, skip_run(skip, l), rec_node, fgrid, st);
            if (s != RC_OK) return s;
        }
    }
    if (ix->leaf_levels & 2) {
        hipLaunchKernelGGL((k_render_level<KIND, NSUB>), dim3(rgrid), dim3(256), 0, st, a, 0, (float2*)nullptr);
        RC_HIP(hipGetLastError());
        return RC_OK;
    }
    return launch_fold_root(a.C, a.root, skip_run(skip, 0), a.npix, a.A, a.B, a.I, vf, rgrid, st);
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_render(const rc_forest* f, const rc_index* ix, const rc_fields* fl, const void* dcams,
                               int32_t ncams, const rc_vforest* vf, const rc_integrator* in, float* rec_leaf,
                               float* rec_node, int64_t npix, float* A, float* B, float* I, const rc_tuning* tune,
                               void* stream) {
    // every check of rc_segments and rc_composite, before anything is enqueued
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_fields(fl, in)) != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || ncams > 32767 || npix <= 0 || !A || !B || !I || !vf->cand_chunk) return RC_EINVAL;
    if (is_surface(f) != (fl->kind == RC_FIELD_SURFACE)) return RC_EUNSUPPORTED;
    if (rc_node_slots(ix, ncams) > 0 && !rec_node) return RC_EINVAL;
    if ((s = check_tables(vf, ix, ncams)) != RC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    bool fused = !is_curved(f) && fl->nch == 1 && ix->maxlevel >= 1 && ix->root >= 0 &&
                 (in->method == RC_INT_ANALYTIC || (in->method == RC_INT_RK4 && in->c_rk == 0.0));
    if (!fused) {
        if (!rec_leaf || vf->cap_cand < 1) return RC_EINVAL;
        if ((s = rc_segments(f, fl, dcams, ncams, vf, in, rec_leaf, nullptr, nullptr, tune, stream)) != RC_OK)
            return s;
        if (fl->nch > 1)
            return rc_composite_channels(f, ix, dcams, ncams, vf, fl->nch, rec_leaf, rec_node, npix, A, B, I, tune,
                                         stream);
        return rc_composite(f, ix, dcams, ncams, vf, rec_leaf, rec_node, npix, A, B, I, tune, stream);
    }
    RenderArgs a;
    a.C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    // the plain fold passes read a dummy record where a child misses the pixel:
    // give them a readable address when there are no leaf records
    if (!rec_leaf) a.C.rec_leaf = (const float2*)vf->child_desc;
    a.child = ix->child;
    a.nx = ix->x;
    a.ny = ix->y;
    a.nz = ix->z;
    a.kappa = fl->kappa;
    a.eps = fl->eps;
    a.nsub = in->substeps;
    a.eq = fl->kind == RC_FIELD_CONST_EQ ? 1 : 0;
    a.root = ix->root;
    a.npix = npix;
    a.A = A;
    a.B = B;
    a.I = I;
    if (in->method == RC_INT_ANALYTIC) return launch_render<0, 1>(a, ix, vf, rec_node, tune, st);
    if (fl->kind == RC_FIELD_CONST) {
        switch (in->substeps) {
            case 4: return launch_render<1, 4>(a, ix, vf, rec_node, tune, st);
            default: return launch_render<1, 0>(a, ix, vf, rec_node, tune, st);
        }
    }
    switch (in->substeps) {
        case 1: return launch_render<2, 1>(a, ix, vf, rec_node, tune, st);
        case 2: return launch_render<2, 2>(a, ix, vf, rec_node, tune, st);
        case 4: return launch_render<2, 4>(a, ix, vf, rec_node, tune, st);
        case 8: return launch_render<2, 8>(a, ix, vf, rec_node, tune, st);
        default: return launch_render<2, 0>(a, ix, vf, rec_node, tune, st);
    }
}
