// rc_shell.hip -- segments and compositing for the curved six-tree shell.
//
// A ray meets a shell element in at most two intervals, so every record of a
// leaf or node holds two (s_in, s_out, A, B) intervals (an empty one has
// s_out <= s_in).  Segment values integrate the ODE with RK4 over equal
// substeps; the field points are mapped back to reference coordinates by FP64
// Newton on the tree map (Sec. 2.1 smooth per-tree transformations).  Curved
// children are not ordered by a fixed permutation along a ray, so a node's
// record merges its children's intervals by depth, combining touching
// intervals with the group operation (Sec. 2.4) -- the merge step of the
// paper's per-pixel segment lists (Sec. 3.5).
#include "rc_composite.h"
#include "rc_shell.h"

using namespace rc;

namespace rc {
namespace {

// An empty slot: s_in > s_out.  Shell intervals have positive length; a
// surface hit is a zero-length interval (PTS), valid when s_in <= s_out.
__device__ inline float4 empty_iv() { return make_float4(1.0f, 0.0f, 1.0f, 0.0f); }
template <bool PTS>
__device__ inline bool iv_valid(const float4& v) {
    return PTS ? v.x <= v.y : v.y > v.x;
}

struct ShellSegArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    const float *kappa, *eps;
    int kind;  // RC_FIELD_CONST or RC_FIELD_TRILINEAR
    const double* geom;
    int64_t tb[RC_MAXTREES + 1];
    int ntrees;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    float4* rec;    // 2 per candidate
    uint8_t* hit;   // number of intervals
    double* sio;    // 4 per candidate
};

// RK4 over NSUB substeps of one interval, field points from Newton inversion
// (NSUB = 0: analytic, constant fields).
template <int NSUB>
__device__ inline float2 shell_integrate(const ShellSegArgs& a, int64_t leaf, const ShellElem& e, const double rho[3],
                                         const double r[3], double s_in, double s_out) {
    if constexpr (NSUB == 0) {
        // constant coefficients: the closed form of eq. ABconstant
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        return seg_const(a.kappa[leaf], a.eps[leaf], (float)((s_out - s_in) * rn));
    }
    constexpr int NS = NSUB > 0 ? NSUB : 1;
    float kc[8], ec[8];
    if (a.kind == RC_FIELD_TRILINEAR) {
        const float4* kp = reinterpret_cast<const float4*>(a.kappa + leaf * 8);
        const float4* ep = reinterpret_cast<const float4*>(a.eps + leaf * 8);
        float4 k0 = kp[0], k1 = kp[1], e0 = ep[0], e1 = ep[1];
        kc[0] = k0.x; kc[1] = k0.y; kc[2] = k0.z; kc[3] = k0.w;
        kc[4] = k1.x; kc[5] = k1.y; kc[6] = k1.z; kc[7] = k1.w;
        ec[0] = e0.x; ec[1] = e0.y; ec[2] = e0.z; ec[3] = e0.w;
        ec[4] = e1.x; ec[5] = e1.y; ec[6] = e1.z; ec[7] = e1.w;
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            kc[q] = a.kappa[leaf];
            ec[q] = a.eps[leaf];
        }
    }
    ShellRef sr = shell_ref_init(e);
    double ds = s_out - s_in;
    // field values at the point p / (2 NSUB) of the way from the far end
    auto field_at = [&](int p, float& bv, float& gv) {
        double s = s_out - ds * ((double)p / (double)(2 * NS));
        double pt[3] = {rho[0] + s * r[0], rho[1] + s * r[1], rho[2] + s * r[2]};
        float xi[3];
        shell_ref_point(e, sr, pt, xi);
        bv = trilin(kc, xi[0], xi[1], xi[2]);
        gv = trilin(ec, xi[0], xi[1], xi[2]);
    };
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    float hstep = (float)(ds * rn) / (float)NS;
    float b0, g0;
    field_at(0, b0, g0);
    float2 acc = make_float2(1.0f, 0.0f);
#pragma unroll 1
    for (int q = 0; q < NSUB; q++) {
        float bm, gm, b1, g1;
        field_at(2 * q + 1, bm, gm);
        field_at(2 * q + 2, b1, g1);
        acc = seg_combine(rk4_step(b0, bm, b1, g0, gm, g1, hstep), acc);
        b0 = b1;
        g0 = g1;
    }
    return acc;
}

// Curved pairing runs one candidate per lane; each hit interval goes to a
// per-wave LDS queue and is integrated 64 at a time (the Newton inversions
// dominate, so the integration runs with every lane busy whatever the hit
// rate).  An entry keeps what is needed to rebuild the ray and the element.
constexpr int SQCAP = 192;  // < 64 waiting + up to 2 x 64 new
struct ShellQueue {
    int64_t slot[SQCAP];  // 2 g + interval
    int32_t leaf[SQCAP];
    int32_t cam[SQCAP];
    int32_t pix[SQCAP];  // i | j << 16
    double s_in[SQCAP], s_out[SQCAP];
};

template <int NSUB>
__device__ inline void shell_drain(const ShellSegArgs& a, const ShellQueue& q, int k) {
    int32_t leaf = q.leaf[k];
    const Cam& c = a.cams[q.cam[k]];
    int i = q.pix[k] & 0xffff, j = q.pix[k] >> 16;
    int tr = 0;
    while (tr + 1 < a.ntrees && leaf >= a.tb[tr + 1]) tr++;
    ShellElem e = shell_elem(a.geom, tr, a.level[leaf], a.x[leaf], a.y[leaf], a.z[leaf]);
    double rho[3], r[3];
    pixel_ray(c, i, j, rho, r);
    double s0 = q.s_in[k], s1 = q.s_out[k];
    float2 ab = shell_integrate<NSUB>(a, leaf, e, rho, r, s0, s1);
    a.rec[q.slot[k]] = make_float4((float)s0, (float)s1, ab.x, ab.y);
}

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NSUB>
__global__ __launch_bounds__(256, 4) void k_segments_shell(ShellSegArgs a) {
    __shared__ ShellQueue Q[256 / WAVE];
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    ShellQueue& q = Q[threadIdx.x / WAVE];
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int qn = 0;  // queued intervals, the same in every lane
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        int n = 0, cam = 0, pix = 0;
        int32_t leaf = 0;
        double iv[4] = {0.0, 0.0, 0.0, 0.0};
        if (g < ncand) {
            int64_t v = cand_pair(a.cand_offset, a.cand_chunk, g, w, nvis, ncand);
            leaf = a.vis_leaf[v];
            cam = a.vis_cam[v];
            const Cam& c = a.cams[cam];
            Rect rc = load_rect(a.vis_rect + 4 * v);
            int kk = (int)(g - a.cand_offset[v]);
            int i, j;
            rect_pixel(rc, kk, i, j);
            pix = i | (j << 16);
            int tr = 0;
            while (tr + 1 < a.ntrees && leaf >= a.tb[tr + 1]) tr++;
            ShellElem e = shell_elem(a.geom, tr, a.level[leaf], a.x[leaf], a.y[leaf], a.z[leaf]);
            double rho[3], r[3];
            pixel_ray(c, i, j, rho, r);
            n = shell_pair(c, e, rho, r, iv);
            if (n < 2) a.rec[2 * g + 1] = empty_iv();
            if (n < 1) a.rec[2 * g] = empty_iv();
            if (a.hit) a.hit[g] = (uint8_t)n;
            if (a.sio) {
                a.sio[4 * g] = iv[0];
                a.sio[4 * g + 1] = iv[1];
                a.sio[4 * g + 2] = n > 1 ? iv[2] : 0.0;
                a.sio[4 * g + 3] = n > 1 ? iv[3] : 0.0;
            }
        }
        uint64_t m1 = __ballot(n >= 1), m2 = __ballot(n >= 2);
        int c1 = __popcll(m1);
        if (n >= 1) {
            int pos = qn + __popcll(m1 & below);
            q.slot[pos] = 2 * g;
            q.leaf[pos] = leaf;
            q.cam[pos] = cam;
            q.pix[pos] = pix;
            q.s_in[pos] = iv[0];
            q.s_out[pos] = iv[1];
        }
        if (n >= 2) {
            int pos = qn + c1 + __popcll(m2 & below);
            q.slot[pos] = 2 * g + 1;
            q.leaf[pos] = leaf;
            q.cam[pos] = cam;
            q.pix[pos] = pix;
            q.s_in[pos] = iv[2];
            q.s_out[pos] = iv[3];
        }
        qn += c1 + __popcll(m2);
        wave_sync_lds();
        while (qn >= WAVE) {
            shell_drain<NSUB>(a, q, qn - WAVE + lane);
            qn -= WAVE;
            wave_sync_lds();
        }
    }
    if (lane < qn) shell_drain<NSUB>(a, q, lane);
}

// ---------------------------------------------------------------------------
// compositing by depth-ordered interval merging
// ---------------------------------------------------------------------------

struct ShellFold {
    FoldCtx C;
    const float4* rec_leaf;  // 2 per candidate
    const float4* rec_node;  // 2 per record
};

__device__ inline void child_intervals(const ShellFold& S, const ChildDesc& d, int i, int j, float4& a, float4& b) {
    if (!desc_has(d, i, j)) {
        a = empty_iv();
        b = empty_iv();
        return;
    }
    int64_t k = desc_index(d, i, j);
    const float4* p = d.off >= 0 ? S.rec_node + 2 * (d.off + k) : S.rec_leaf + 2 * (-1 - d.off + k);
    a = p[0];
    b = p[1];
}

__device__ inline float4 join_iv(const float4& p, const float4& q) {
    float2 m = seg_combine(make_float2(p.z, p.w), make_float2(q.z, q.w));
    return make_float4(p.x, q.y > p.y ? q.y : p.y, m.x, m.y);
}

// Merge the children's intervals (up to 16) into the node's, at most two.
// Taken nearest first; an interval that starts where the previous one ends
// (or before) extends it.  A third run can only come from rounding at a
// shared face (the node meets a ray in at most two intervals), so the two
// runs with the smallest gap between them are joined: empty space between
// them is the identity of the group, so the value is unchanged.
template <bool PTS, int NQ>
__device__ inline void merge_runs(const float4 (&iv)[NQ], float4& o0, float4& o1) {
    uint32_t used = 0;
    int nout = 0;
    o0 = empty_iv();
    o1 = empty_iv();
    for (int it = 0; it < NQ; it++) {
        float best = INFINITY;
        float4 cur = empty_iv();
        int bq = -1;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            bool ok = iv_valid<PTS>(iv[q]) && !((used >> q) & 1u) && iv[q].x < best;
            if (ok) {
                best = iv[q].x;
                cur = iv[q];
                bq = q;
            }
        }
        if (bq < 0) break;
        used |= 1u << bq;
        if (nout == 0) {
            o0 = cur;
            nout = 1;
        } else if (nout == 1) {
            if (cur.x <= o0.y) {
                o0 = join_iv(o0, cur);
            } else {
                o1 = cur;
                nout = 2;
            }
        } else if (cur.x <= o1.y) {
            o1 = join_iv(o1, cur);
        } else if (o1.x - o0.y < cur.x - o1.y) {
            o0 = join_iv(o0, o1);
            o1 = cur;
        } else {
            o1 = join_iv(o1, cur);
        }
    }
}

// Children in Morton order; a surface (PTS) is a quadtree with z = 0, so only
// the first four child slots can hold a child.
template <bool PTS, bool UNIFORM>
__device__ inline void shell_node(const ShellFold& S, int64_t dslot, int i, int j, float4& o0, float4& o1) {
    constexpr int NC = PTS ? 4 : 8;
    float4 iv[2 * NC];
#pragma unroll
    for (int q = 0; q < NC; q++) {
        ChildDesc d = UNIFORM ? load_desc_scalar(S.C.desc, dslot * 8 + q) : load_desc(S.C.desc + dslot * 8 + q);
        child_intervals(S, d, i, j, iv[2 * q], iv[2 * q + 1]);
    }
    merge_runs<PTS, 2 * NC>(iv, o0, o1);
}

template <bool PTS>
__device__ inline void shell_node_auto(const ShellFold& S, int64_t dslot, bool active, int i, int j, float4& o0,
                                       float4& o1) {
    int64_t d0 = uniform64(dslot);
    if (__all(!active || dslot == d0))
        shell_node<PTS, true>(S, d0, i, j, o0, o1);
    else
        shell_node<PTS, false>(S, dslot, i, j, o0, o1);
}

template <bool PTS>
__global__ __launch_bounds__(256) void k_fold_level_shell(ShellFold S, int l, float4* out) {
    const FoldCtx& C = S.C;
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
        float4 o0, o1;
        shell_node_auto<PTS>(S, cam * C.ninternal + m, act, i, j, o0, o1);
        if (act) {
            out[2 * g] = o0;
            out[2 * g + 1] = o1;
        }
    }
}

// Roots: each tree's intervals, then all trees folded front to back.
template <bool PTS>
__global__ __launch_bounds__(256) void k_fold_root_shell(ShellFold S, int ntrees, int32_t r0, int32_t r1, int32_t r2,
                                                         int32_t r3, int32_t r4, int32_t r5, int64_t npix, float* A,
                                                         float* B, float* I, const int32_t* leaf_vis,
                                                         const int16_t* vis_rect, const int64_t* cand_offset) {
    const FoldCtx& C = S.C;
    if (C.counts[3]) return;
    int32_t roots[6] = {r0, r1, r2, r3, r4, r5};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int cam = camera_of_pixel_wave(C.cams, C.ncams, p);
        const Cam& c = C.cams[cam];
        int64_t loc = p - c.img_off;
        int j = (int)(loc / c.w);
        int i = (int)(loc - (int64_t)j * c.w);
        float4 iv[12];
#pragma clang loop unroll(full)
        for (int t = 0; t < 6; t++) {
            iv[2 * t] = empty_iv();
            iv[2 * t + 1] = empty_iv();
            int32_t root = t < ntrees ? roots[t] : RC_ABSENT;
            if (root >= 0) {
                shell_node_auto<PTS>(S, (int64_t)cam * C.ninternal + root, true, i, j, iv[2 * t], iv[2 * t + 1]);
            } else if (root <= -2) {
                int32_t v = leaf_vis[(int64_t)cam * C.N + (-2 - (int64_t)root)];
                if (v >= 0) {
                    Rect r = load_rect(vis_rect + 4 * (int64_t)v);
                    if (r.contains(i, j)) {
                        const float4* q = S.rec_leaf + 2 * (cand_offset[v] + (int64_t)(j - r.j0) * r.width() + (i - r.i0));
                        iv[2 * t] = q[0];
                        iv[2 * t + 1] = q[1];
                    }
                }
            }
        }
        // every interval in depth order; gaps between them hold nothing
        uint32_t used = 0;
        float2 acc = make_float2(1.0f, 0.0f);
        for (int it = 0; it < 12; it++) {
            float best = INFINITY;
            float4 cur = empty_iv();
            int bq = -1;
#pragma unroll
            for (int q = 0; q < 12; q++) {
                bool ok = iv_valid<PTS>(iv[q]) && !((used >> q) & 1u) && iv[q].x < best;
                if (ok) {
                    best = iv[q].x;
                    cur = iv[q];
                    bq = q;
                }
            }
            if (bq < 0) break;
            used |= 1u << bq;
            acc = seg_combine(acc, make_float2(cur.z, cur.w));
        }
        A[p] = acc.x;
        B[p] = acc.y;
        I[p] = fmaf(acc.x, (float)c.bg, acc.y);
    }
}

}  // namespace
}  // namespace rc

// Called by rc_segments and rc_composite for RC_GEOM_SHELL6 forests.
rc_status rc::rc_shell_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                            const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                            const rc_tuning* tune, hipStream_t st) {
    if (fl->kind == RC_FIELD_CONST_EQ || (in->method != RC_INT_ANALYTIC && in->method != RC_INT_RK4) ||
        in->c_rk > 0.0)
        return RC_EUNSUPPORTED;
    ShellSegArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.z = f->z;
    a.N = f->nleaves;
    a.kappa = fl->kappa;
    a.eps = fl->eps;
    a.kind = fl->kind;
    a.geom = f->geom_table;
    for (int k = 0; k <= RC_MAXTREES; k++) a.tb[k] = k <= f->ntrees ? f->tree_begin[k] : f->nleaves;
    a.ntrees = f->ntrees;
    a.vis_leaf = vf->vis_leaf;
    a.vis_cam = vf->vis_cam;
    a.vis_rect = vf->vis_rect;
    a.cand_offset = vf->cand_offset;
    a.counts = vf->counts;
    a.cand_chunk = vf->cand_chunk;
    a.cap_cand = vf->cap_cand;
    a.rec = (float4*)rec_leaf;
    a.hit = hit;
    a.sio = sio;
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 16384))), B(256);
    int ns = in->method == RC_INT_ANALYTIC ? 0 : in->substeps;
    switch (ns) {
        case 0: hipLaunchKernelGGL((k_segments_shell<0>), G, B, 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_segments_shell<1>), G, B, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_segments_shell<2>), G, B, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_segments_shell<4>), G, B, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_segments_shell<8>), G, B, 0, st, a); break;
        default: return RC_EUNSUPPORTED;
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}

rc_status rc::rc_shell_composite(const rc_forest* f, const rc_index* ix, const void* dcams, int32_t ncams,
                             const rc_vforest* vf, const float* rec_leaf, float* rec_node, int64_t npix, float* A,
                             float* B, float* I, const rc_tuning* tune, hipStream_t st) {
    ShellFold S;
    S.C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    S.rec_leaf = (const float4*)rec_leaf;
    S.rec_node = (const float4*)rec_node;
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 16));
    bool pts = is_surface(f);
    for (int l = ix->maxlevel - 1; l >= 1; l--) {
        if (ix->level_begin[l + 1] == ix->level_begin[l]) continue;
        if (pts)
            hipLaunchKernelGGL(k_fold_level_shell<true>, dim3(grid), dim3(256), 0, st, S, l, (float4*)rec_node);
        else
            hipLaunchKernelGGL(k_fold_level_shell<false>, dim3(grid), dim3(256), 0, st, S, l, (float4*)rec_node);
        RC_HIP(hipGetLastError());
    }
    int32_t r[6];
    for (int k = 0; k < 6; k++) r[k] = k < ix->ntrees ? ix->roots[k] : RC_ABSENT;
    dim3 rg(stride_grid(npix, 256, tuned(tune, 2, 256 * 16))), rb(256);
    if (pts)
        hipLaunchKernelGGL(k_fold_root_shell<true>, rg, rb, 0, st, S, ix->ntrees, r[0], r[1], r[2], r[3], r[4], r[5],
                           npix, A, B, I, vf->leaf_vis, vf->vis_rect, vf->cand_offset);
    else
        hipLaunchKernelGGL(k_fold_root_shell<false>, rg, rb, 0, st, S, ix->ntrees, r[0], r[1], r[2], r[3], r[4], r[5],
                           npix, A, B, I, vf->leaf_vis, vf->vis_rect, vf->cand_offset);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
