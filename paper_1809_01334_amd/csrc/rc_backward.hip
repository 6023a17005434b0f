// rc_backward.hip -- adjoint of the rendered images with respect to the
// per-leaf coefficients.
//
// The image of a pixel is the group product of its segments (eq. aggregate),
// so with T the transmittance in front of a segment and J the intensity that
// enters it from behind, dI/dA = T J and dI/dB = T.  These pairs are passed
// top-down through the same coarsening hierarchy the forward fold used: a
// node hands each child (g T_front, J_behind) with prefix products of the
// nearer siblings and suffix folds of the farther ones (no division).  At the
// leaves the segment evaluation is recomputed from the coefficients and
// differentiated in reverse; the per-leaf sums use a fixed reduction order.
#include "rc_composite.h"
#include "rc_steps.h"

using namespace rc;

namespace rc {
namespace {

// Hand the adjoint (gT, J) of descriptor slot `dslot` at pixel (i, j) to the
// node's children: the nearer siblings' transmittances multiply gT, the
// farther siblings' fold applied to J gives the intensity from behind.
template <bool UNIFORM>
__device__ inline void push_children(const FoldCtx& C, int64_t dslot, int i, int j, float gT, float J,
                                     float2* adj_leaf, float2* adj_node) {
    ChildDesc d[8];
    float2 rv[8];
    bool has[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        d[q] = UNIFORM ? load_desc_scalar(C.desc, dslot * 8 + q) : load_desc(C.desc + dslot * 8 + q);
        has[q] = desc_has(d[q], i, j);
        rv[q] = *desc_ptr(C, d[q], has[q], i, j);
    }
#pragma unroll
    for (int q = 0; q < 8; q++)
        if (!has[q]) rv[q] = make_float2(1.0f, 0.0f);
    float Jq[8];
    float Jc = J;
#pragma unroll
    for (int q = 7; q >= 0; q--) {
        Jq[q] = Jc;
        Jc = fmaf(rv[q].x, Jc, rv[q].y);
    }
    float T = gT;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        if (has[q]) {
            int64_t k = desc_index(d[q], i, j);
            if (d[q].off >= 0)
                adj_node[d[q].off + k] = make_float2(T, Jq[q]);
            else
                adj_leaf[-1 - d[q].off + k] = make_float2(T, Jq[q]);
        }
        T *= rv[q].x;
    }
}

__device__ inline void push_children_auto(const FoldCtx& C, int64_t dslot, bool active, int i, int j, float gT,
                                          float J, float2* adj_leaf, float2* adj_node) {
    int64_t d0 = uniform64(dslot);
    if (__all(!active || dslot == d0)) {
        if (active) push_children<true>(C, d0, i, j, gT, J, adj_leaf, adj_node);
    } else if (active) {
        push_children<false>(C, dslot, i, j, gT, J, adj_leaf, adj_node);
    }
}

__global__ __launch_bounds__(256) void k_adj_root(FoldCtx C, int32_t root, int64_t npix, const float* dLdI,
                                                  float2* adj_leaf, float2* adj_node, const int32_t* leaf_vis,
                                                  const int16_t* vis_rect, const int64_t* cand_offset) {
    if (C.counts[3]) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int cam = camera_of_pixel_wave(C.cams, C.ncams, p);
        const Cam& c = C.cams[cam];
        int64_t loc = p - c.img_off;
        int j = (int)(loc / c.w);
        int i = (int)(loc - (int64_t)j * c.w);
        float g = dLdI[p];
        float bg = (float)c.bg;
        if (root >= 0) {
            push_children_auto(C, (int64_t)cam * C.ninternal + root, true, i, j, g, bg, adj_leaf, adj_node);
        } else if (root <= -2) {
            int32_t v = leaf_vis[(int64_t)cam * C.N + (-2 - (int64_t)root)];
            if (v >= 0) {
                Rect r = load_rect(vis_rect + 4 * (int64_t)v);
                if (r.contains(i, j))
                    adj_leaf[cand_offset[v] + (int64_t)(j - r.j0) * r.width() + (i - r.i0)] = make_float2(g, bg);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_adj_level(FoldCtx C, int l, float2* adj_leaf, float2* adj_node) {
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
        float2 a = adj_node[gg];
        push_children_auto(C, cam * C.ninternal + m, act, i, j, a.x, a.y, adj_leaf, adj_node);
    }
}

// Reverse of field_cubic: corner adjoints vb[8] from the adjoints pb[4] of
// the cubic's coefficients.
__device__ inline void field_cubic_bwd(const float a[3], const float d[3], const float pb[4], float vb[8]) {
    float G0b = fmaf(a[2], pb[0], d[2] * pb[1]);
    float G1b = fmaf(a[2], pb[1], d[2] * pb[2]);
    float G2b = fmaf(a[2], pb[2], d[2] * pb[3]);
    float fb[2][3] = {{pb[0] - G0b, pb[1] - G1b, pb[2] - G2b}, {G0b, G1b, G2b}};
    float e0b[4], e1b[4];
#pragma unroll
    for (int z = 0; z < 2; z++) {
        float D0b = fmaf(a[1], fb[z][0], d[1] * fb[z][1]);
        float D1b = fmaf(a[1], fb[z][1], d[1] * fb[z][2]);
        e0b[2 * z] = fb[z][0] - D0b;
        e0b[2 * z + 1] = D0b;
        e1b[2 * z] = fb[z][1] - D1b;
        e1b[2 * z + 1] = D1b;
    }
#pragma unroll
    for (int m = 0; m < 4; m++) {
        float dvb = fmaf(a[0], e0b[m], d[0] * e1b[m]);
        vb[2 * m] = e0b[m] - dvb;
        vb[2 * m + 1] = dvb;
    }
}

// Stage point p of NSUB equal pieces as a fraction of the segment from its far
// end: RK4 and Simpson use the ends and middle of every piece (2 NSUB + 1
// points, shared between neighbours), Gauss the two points 1/2 -+ sqrt(3)/6 of
// every piece (2 NSUB points).
template <int METHOD, int NSUB>
__device__ inline float stage_t(int p) {
    if (METHOD == RC_INT_GAUSS2) {
        const float c0 = 0.21132486540518713f, c1 = 0.78867513459481287f;  // 1/2 -+ sqrt(3)/6
        return ((float)(p >> 1) + ((p & 1) ? c1 : c0)) * (1.0f / (float)NSUB);
    }
    return (float)p * (0.5f / (float)NSUB);
}

// Gradient of one segment's (A, B) contribution: grad[0..nc) kappa corners,
// grad[nc..2nc) eps corners.  gT = g T_front, J = intensity from behind.
// METHOD: RK4, Gauss or Simpson over NSUB equal pieces.
template <int KIND, int NSUB, int METHOD>
__device__ inline void segment_grad(const float kc[8], const float ec[8], const SegGeom& sg, float gT, float J,
                                    float grad[GRAD_MAX]) {
    if (KIND == 3) {
        // eq. BIrelation: A = exp(-k dx), B = I (1 - A) with I in place of eps
        float k = kc[0], I = ec[0], dx = sg.dx;
        float A = expf(-k * dx);
        grad[0] = gT * dx * A * (I - J);
        grad[1] = gT * -expm1f(-k * dx);
        return;
    }
    if (KIND == 0) {
        float k = kc[0], e = ec[0], dx = sg.dx;
        float x = k * dx;
        float A = expf(-x);
        float phi, dphi;
        if (fabsf(x) < 0.1f) {
            phi = fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 720.0f, -1.0f / 120.0f), 1.0f / 24.0f), -1.0f / 6.0f),
                       0.5f);
            phi = fmaf(-x, phi, 1.0f);
            dphi = fmaf(x, fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 840.0f, -1.0f / 144.0f), 1.0f / 30.0f),
                                        -1.0f / 8.0f),
                                1.0f / 3.0f),
                        -0.5f);
        } else {
            float om = -expm1f(-x);
            phi = om / x;
            dphi = (x * A - om) / (x * x);
        }
        float dAdk = -dx * A;
        float dBdk = e * dx * dx * dphi;
        float dBde = dx * phi;
        grad[0] = gT * (J * dAdk + dBdk);
        grad[1] = gT * dBde;
        return;
    }
    // forward: field values at the stage points, substep values and the
    // intensity entering each substep
    constexpr int NP = METHOD == RC_INT_GAUSS2 ? 2 * NSUB : 2 * NSUB + 1;
    const float inv = 1.0f / (float)NSUB;
    float h = sg.dx * inv;
    float pk[4], pe[4];
    if (KIND == 2) {
        field_cubic(kc, sg.xf, sg.dxi, pk);
        field_cubic(ec, sg.xf, sg.dxi, pe);
    } else {
        pk[0] = kc[0];
        pe[0] = ec[0];
        pk[1] = pk[2] = pk[3] = pe[1] = pe[2] = pe[3] = 0.0f;
    }
    float bs[NP], gs[NP];
#pragma unroll
    for (int p = 0; p < NP; p++) {
        float t = stage_t<METHOD, NSUB>(p);
        bs[p] = horner3(pk, t);
        gs[p] = horner3(pe, t);
    }
    float Iin[NSUB], av[NSUB];
    float Ic = J;
#pragma unroll
    for (int q = 0; q < NSUB; q++) {
        float2 st;
        if (METHOD == RC_INT_GAUSS2)
            st = gauss2_step(bs[2 * q], bs[2 * q + 1], gs[2 * q], gs[2 * q + 1], h);
        else if (METHOD == RC_INT_SIMPSON)
            st = simpson_step(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], gs[2 * q + 2], h);
        else
            st = rk4_step(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], gs[2 * q + 2], h);
        Iin[q] = Ic;
        av[q] = st.x;
        Ic = fmaf(st.x, Ic, st.y);
    }
    // reverse: G = dL/d(intensity leaving substep q), nearest first
    float dbs[NP], dgs[NP];
#pragma unroll
    for (int p = 0; p < NP; p++) {
        dbs[p] = 0.0f;
        dgs[p] = 0.0f;
    }
    float G = gT;
#pragma unroll
    for (int q = NSUB - 1; q >= 0; q--) {
        if (METHOD == RC_INT_GAUSS2)
            gauss2_step_bwd(bs[2 * q], bs[2 * q + 1], gs[2 * q], gs[2 * q + 1], h, G * Iin[q], G, dbs[2 * q],
                            dbs[2 * q + 1], dgs[2 * q], dgs[2 * q + 1]);
        else if (METHOD == RC_INT_SIMPSON)
            simpson_step_bwd(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], gs[2 * q + 2], h,
                             G * Iin[q], G, dbs[2 * q], dbs[2 * q + 1], dbs[2 * q + 2], dgs[2 * q], dgs[2 * q + 1],
                             dgs[2 * q + 2]);
        else
            rk4_step_bwd(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], h, G * Iin[q], G,
                         dbs[2 * q], dbs[2 * q + 1], dbs[2 * q + 2], dgs[2 * q], dgs[2 * q + 1], dgs[2 * q + 2]);
        G *= av[q];
    }
    if (KIND == 1) {
        float sk = 0.0f, se = 0.0f;
#pragma unroll
        for (int p = 0; p < NP; p++) {
            sk += dbs[p];
            se += dgs[p];
        }
        grad[0] = sk;
        grad[1] = se;
        return;
    }
    // adjoints of the cubic coefficients: moments of the point adjoints
    float pkb[4] = {0.0f, 0.0f, 0.0f, 0.0f}, peb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int p = 0; p < NP; p++) {
        float t = stage_t<METHOD, NSUB>(p);
        float tn = 1.0f;
#pragma unroll
        for (int n = 0; n < 4; n++) {
            pkb[n] = fmaf(dbs[p], tn, pkb[n]);
            peb[n] = fmaf(dgs[p], tn, peb[n]);
            tn *= t;
        }
    }
    field_cubic_bwd(sg.xf, sg.dxi, pkb, grad);
    field_cubic_bwd(sg.xf, sg.dxi, peb, grad + 8);
}

struct LeafAdjArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    const float *kappa, *eps;
    int nsub;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    const float2* adj_leaf;
    float* partial;  // [(nchunks + nvis)][GRAD_MAX], entry (chunk w, pair v) at w + v
};

// Zero the (chunk, pair) partial slots that the leaf adjoint may leave unwritten.
__global__ __launch_bounds__(256) void k_fill_partials(const int64_t* counts, int64_t cap_cand, float* partial) {
    if (counts[3]) return;
    int64_t ncand = counts[1] < cap_cand ? counts[1] : cap_cand;
    int64_t n = ((ncand + WAVE - 1) / WAVE + counts[0] + 1) * GRAD_MAX;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) partial[t] = 0.0f;
}

// Leaf adjoint.  Pairing runs one candidate per lane; hits go through a
// per-wave FIFO in LDS and are differentiated 64 at a time.  Each batch sums
// its lanes per (chunk w, pair v) key with a segmented shuffle scan (keys are
// non-decreasing in FIFO order); a key that continues into the next batch is
// carried, so every (w, v) slot at index w + v is written once, in a fixed
// order.
constexpr int BQCAP = 128;
struct AdjQueue {
    int64_t key[BQCAP];
    int32_t leaf[BQCAP];
    float xf0[BQCAP], xf1[BQCAP], xf2[BQCAP], d0[BQCAP], d1[BQCAP], d2[BQCAP], dx[BQCAP], gT[BQCAP], J[BQCAP];
};

template <int KIND, int NSUB, int METHOD>
__device__ inline void adj_drain(const LeafAdjArgs& a, AdjQueue& q, int head, int tail, int n, int lane,
                                 float* carry, int64_t& carry_key) {
    constexpr int NPAR = KIND == 2 ? 16 : 2;
    const int mask = BQCAP - 1;
    int e = (head + lane) & mask;
    bool act = lane < n;
    int64_t key = act ? q.key[e] : INT64_MAX;
    float grad[GRAD_MAX];
#pragma unroll
    for (int c = 0; c < GRAD_MAX; c++) grad[c] = 0.0f;
    if (act) {
        SegGeom sg;
        sg.xf[0] = q.xf0[e];
        sg.xf[1] = q.xf1[e];
        sg.xf[2] = q.xf2[e];
        sg.dxi[0] = q.d0[e];
        sg.dxi[1] = q.d1[e];
        sg.dxi[2] = q.d2[e];
        sg.dx = q.dx[e];
        int64_t leaf = q.leaf[e];
        float kc[8], ec[8];
        if (KIND == 2) {
            const float4* kp = reinterpret_cast<const float4*>(a.kappa + leaf * 8);
            const float4* ep = reinterpret_cast<const float4*>(a.eps + leaf * 8);
            float4 k0 = kp[0], k1 = kp[1], e0 = ep[0], e1 = ep[1];
            kc[0] = k0.x; kc[1] = k0.y; kc[2] = k0.z; kc[3] = k0.w;
            kc[4] = k1.x; kc[5] = k1.y; kc[6] = k1.z; kc[7] = k1.w;
            ec[0] = e0.x; ec[1] = e0.y; ec[2] = e0.z; ec[3] = e0.w;
            ec[4] = e1.x; ec[5] = e1.y; ec[6] = e1.z; ec[7] = e1.w;
        } else {
#pragma unroll
            for (int c = 0; c < 8; c++) {
                kc[c] = a.kappa[leaf];
                ec[c] = a.eps[leaf];
            }
        }
        segment_grad<KIND, NSUB, METHOD>(kc, ec, sg, q.gT[e], q.J[e], grad);
    }
    // segmented inclusive scan over lanes with equal keys
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int64_t kd = __shfl_up(key, d);
        bool same = lane >= d && kd == key;
#pragma unroll
        for (int c = 0; c < NPAR; c++) {
            float y = __shfl_up(grad[c], d);
            if (same) grad[c] += y;
        }
    }
    int64_t knext = __shfl_down(key, 1);
    bool last = act && ((lane == WAVE - 1) || knext != key);
    int64_t key0 = __shfl(key, 0);
    int64_t next_key = (tail - head > n) ? q.key[(head + n) & mask] : -2;
    int64_t key_end = __shfl(key, n - 1);
    bool cont = key_end == next_key;  // the batch's last key goes on in the queue
    float val[NPAR];
#pragma unroll
    for (int c = 0; c < NPAR; c++) val[c] = grad[c] + ((key == key0 && key == carry_key) ? carry[c] : 0.0f);
    if (last && !(cont && lane == n - 1)) {
        float* dst = a.partial + key * GRAD_MAX;
#pragma unroll
        for (int c = 0; c < NPAR; c++) dst[c] = val[c];
    }
    if (cont) {
#pragma unroll
        for (int c = 0; c < NPAR; c++) carry[c] = __shfl(val[c], n - 1);
        carry_key = key_end;
    } else {
        carry_key = -1;
    }
}

template <int KIND, int NSUB, int METHOD>
__global__ __launch_bounds__(256) void k_adj_leaf(LeafAdjArgs a) {
    __shared__ AdjQueue Q[256 / WAVE];
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    AdjQueue& q = Q[threadIdx.x / WAVE];
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int head = 0, tail = 0;  // FIFO positions (mod BQCAP), the same in every lane
    float carry[GRAD_MAX];
#pragma unroll
    for (int c = 0; c < GRAD_MAX; c++) carry[c] = 0.0f;
    int64_t carry_key = -1;
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        bool h = false;
        SegGeom sg;
        int32_t leaf = 0;
        int64_t key = 0;
        float2 ad = make_float2(0.0f, 0.0f);
        if (g < ncand) {
            int64_t v = 0;
            Pairing p = pair_candidate(a, g, w, nvis, ncand, &v);
            key = w + v;
            h = p.hit;
            leaf = p.leaf;
            if (h) {
                sg = seg_geom(p.rho, p.rr, p.s_in, p.s_out, p.lo, p.lv);
                ad = a.adj_leaf[g];
            }
        }
        uint64_t m = __ballot(h);
        if (h) {
            int e = (tail + __popcll(m & below)) & (BQCAP - 1);
            q.key[e] = key;
            q.leaf[e] = leaf;
            q.xf0[e] = sg.xf[0];
            q.xf1[e] = sg.xf[1];
            q.xf2[e] = sg.xf[2];
            q.d0[e] = sg.dxi[0];
            q.d1[e] = sg.dxi[1];
            q.d2[e] = sg.dxi[2];
            q.dx[e] = sg.dx;
            q.gT[e] = ad.x;
            q.J[e] = ad.y;
        }
        tail += __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (tail - head >= WAVE) {
            adj_drain<KIND, NSUB, METHOD>(a, q, head, tail, WAVE, lane, carry, carry_key);
            head += WAVE;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (tail - head > 0) adj_drain<KIND, NSUB, METHOD>(a, q, head, tail, tail - head, lane, carry, carry_key);
}

// Per (leaf, parameter): over the cameras in order, add the chunk partials of
// the leaf's visible pair in chunk order, into the leaf-major coefficient
// layout.  A fixed order, so the sums are deterministic.
__global__ __launch_bounds__(256) void k_grad_leaves(const int64_t* counts, int64_t N, int ncams, const int32_t* leaf_vis,
                                                     const int64_t* cand_offset, int64_t cap_cand,
                                                     const float* partial, int nc, float* dk, float* de,
                                                     int accumulate) {
    if (counts[3]) return;
    int64_t npar = 2 * nc;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * npar; t += stride) {
        int64_t l = divu(t, npar);
        int c = (int)(t - l * npar);
        float acc = 0.0f;
        for (int cam = 0; cam < ncams; cam++) {
            int32_t v = leaf_vis[(int64_t)cam * N + l];
            if (v < 0) continue;
            int64_t c0 = cand_offset[v], c1 = cand_offset[v + 1];
            if (c1 > cap_cand) c1 = cap_cand;
            if (c1 <= c0) continue;
            int64_t w0 = c0 / WAVE, w1 = (c1 - 1) / WAVE;
            for (int64_t w = w0; w <= w1; w++) acc += partial[(w + v) * GRAD_MAX + c];
        }
        float* dst = c < nc ? dk + l * nc + c : de + l * nc + (c - nc);
        *dst = accumulate ? *dst + acc : acc;
    }
}

// The leaf adjoint for NSUB in {1, 2, 4, 8} pieces (checked before any launch).
template <int KIND, int METHOD>
rc_status launch_adj_leaf(int nsub, dim3 G, dim3 B, hipStream_t st, const LeafAdjArgs& la) {
    switch (nsub) {
        case 1: hipLaunchKernelGGL((k_adj_leaf<KIND, 1, METHOD>), G, B, 0, st, la); break;
        case 2: hipLaunchKernelGGL((k_adj_leaf<KIND, 2, METHOD>), G, B, 0, st, la); break;
        case 4: hipLaunchKernelGGL((k_adj_leaf<KIND, 4, METHOD>), G, B, 0, st, la); break;
        case 8: hipLaunchKernelGGL((k_adj_leaf<KIND, 8, METHOD>), G, B, 0, st, la); break;
        default: return RC_EUNSUPPORTED;
    }
    return RC_OK;
}

}  // namespace
}  // namespace rc

static rc_status backward_one(const rc_forest* f, const rc_index* ix, const rc_fields* fl, const void* dcams,
                              int32_t ncams, const rc_vforest* vf, const rc_integrator* in, const float* rec_leaf,
                              const float* rec_node, int64_t npix, const float* dLdI, float* adj_leaf,
                              float* adj_node, float* dk, float* de, int32_t accumulate, void* ws,
                              const rc_tuning* tune, hipStream_t st);

extern "C" rc_status rc_segments_backward(const rc_forest* f, const rc_index* ix, const rc_fields* fl,
                                          const void* dcams, int32_t ncams, const rc_vforest* vf,
                                          const rc_integrator* in, const float* rec_leaf, const float* rec_node,
                                          int64_t npix, const float* dLdI, float* adj_leaf, float* adj_node,
                                          float* dk, float* de, int32_t accumulate, void* ws, size_t ws_bytes,
                                          const rc_tuning* tune, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if (is_curved(f)) return RC_EUNSUPPORTED;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_fields(fl, in)) != RC_OK) return s;
    if (!adjoint_supported(fl, in)) return RC_EUNSUPPORTED;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || npix <= 0 || !rec_leaf || !dLdI || !adj_leaf || !dk || !de || vf->cap_cand < 1)
        return RC_EINVAL;
    bool nodes = rc_node_slots(ix, ncams) > 0;
    if (nodes && (!rec_node || !adj_node)) return RC_EINVAL;
    // equal pieces: the leaf adjoint's instantiations; with the recursion any
    // power of two (checked with the fields)
    if (in->method != RC_INT_ANALYTIC && in->c_rk == 0.0 && in->substeps != 1 && in->substeps != 2 &&
        in->substeps != 4 && in->substeps != 8)
        return RC_EUNSUPPORTED;
    if ((s = check_tables(vf, ix, ncams)) != RC_OK) return s;
    if (!ws || ws_bytes < rc_workspace_bytes(f, ix, ncams, vf)) return RC_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    // channels one after the other, in channel-major blocks of every per-channel array
    int64_t fstride = f->nleaves * (fl->kind == RC_FIELD_TRILINEAR ? 8 : 1);
    for (int ch = 0; ch < fl->nch; ch++) {
        rc_fields one = *fl;
        one.nch = 1;
        one.kappa = fl->kappa + ch * fstride;
        one.eps = fl->eps + ch * fstride;
        s = backward_one(f, ix, &one, dcams, ncams, vf, in, rec_leaf + ch * vf->cap_cand * 2,
                         nodes ? rec_node + ch * vf->cap_rec * 2 : rec_node, npix, dLdI + ch * npix, adj_leaf,
                         adj_node, dk + ch * fstride, de + ch * fstride, accumulate, ws, tune, st);
        if (s != RC_OK) return s;
    }
    return RC_OK;
}

// One channel of rc_segments_backward (arguments validated).
static rc_status backward_one(const rc_forest* f, const rc_index* ix, const rc_fields* fl, const void* dcams,
                              int32_t ncams, const rc_vforest* vf, const rc_integrator* in, const float* rec_leaf,
                              const float* rec_node, int64_t npix, const float* dLdI, float* adj_leaf,
                              float* adj_node, float* dk, float* de, int32_t accumulate, void* ws,
                              const rc_tuning* tune, hipStream_t st) {
    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    hipLaunchKernelGGL(k_adj_root, dim3(stride_grid(npix, 256, tuned(tune, 2, 256 * 16))), dim3(256), 0, st, C,
                       ix->root, npix, dLdI,
                       (float2*)adj_leaf, (float2*)adj_node, vf->leaf_vis, vf->vis_rect, vf->cand_offset);
    RC_HIP(hipGetLastError());
    unsigned grid = stride_grid(vf->cap_rec, 256, tuned(tune, 1, 256 * 16));
    for (int l = 1; l < ix->maxlevel; l++) {
        if (ix->level_begin[l + 1] == ix->level_begin[l]) continue;
        hipLaunchKernelGGL(k_adj_level, dim3(grid), dim3(256), 0, st, C, l, (float2*)adj_leaf, (float2*)adj_node);
        RC_HIP(hipGetLastError());
    }

    int64_t nchunks = (vf->cap_cand + WAVE - 1) / WAVE;
    float* partial = (float*)ws;
    LeafAdjArgs la{(const Cam*)dcams, f->level,       f->x,          f->y,         f->z,
                   f->nleaves,        fl->kappa,      fl->eps,       in->substeps, vf->vis_leaf,
                   vf->vis_cam,       vf->vis_rect,   vf->cand_offset, vf->counts, vf->cand_chunk,
                   vf->cap_cand,      (const float2*)adj_leaf, partial};
    hipLaunchKernelGGL(k_fill_partials, dim3(stride_grid((nchunks + vf->cap_vis + 1) * GRAD_MAX, 256, 256 * 16)),
                       dim3(256), 0, st, vf->counts, vf->cap_cand, partial);
    RC_HIP(hipGetLastError());
    unsigned lg = stride_grid(nchunks * WAVE, 256, tuned(tune, 3, 256 * 8));
    int nc = fl->kind == RC_FIELD_TRILINEAR ? 8 : 1;
    dim3 G(lg), B(256);
    rc_status s = RC_OK;
    if (in->method == RC_INT_ANALYTIC && fl->kind == RC_FIELD_CONST_EQ) {
        hipLaunchKernelGGL((k_adj_leaf<3, 1, RC_INT_ANALYTIC>), G, B, 0, st, la);
    } else if (in->method == RC_INT_ANALYTIC) {
        hipLaunchKernelGGL((k_adj_leaf<0, 1, RC_INT_ANALYTIC>), G, B, 0, st, la);
    } else if (in->c_rk > 0.0) {
        if ((s = rc_adjoint_pieces(f, fl, dcams, vf, in, adj_leaf, partial, tune, st)) != RC_OK) return s;
    } else {
        bool tri = fl->kind == RC_FIELD_TRILINEAR;
        switch (in->method) {
            case RC_INT_RK4:
                s = tri ? launch_adj_leaf<2, RC_INT_RK4>(in->substeps, G, B, st, la)
                        : launch_adj_leaf<1, RC_INT_RK4>(in->substeps, G, B, st, la);
                break;
            case RC_INT_GAUSS2:
                s = tri ? launch_adj_leaf<2, RC_INT_GAUSS2>(in->substeps, G, B, st, la)
                        : launch_adj_leaf<1, RC_INT_GAUSS2>(in->substeps, G, B, st, la);
                break;
            default:
                s = tri ? launch_adj_leaf<2, RC_INT_SIMPSON>(in->substeps, G, B, st, la)
                        : launch_adj_leaf<1, RC_INT_SIMPSON>(in->substeps, G, B, st, la);
                break;
        }
        if (s != RC_OK) return s;
    }
    RC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_leaves, dim3(stride_grid(f->nleaves * 2 * nc, 256, 256 * 32)), dim3(256), 0, st,
                       vf->counts, f->nleaves, ncams, vf->leaf_vis, vf->cand_offset, vf->cap_cand, partial, nc, dk,
                       de, accumulate);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
