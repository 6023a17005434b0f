// rc_integrators.hip -- segment integrators beyond the closed form and the
// fixed-step RK4 (Sec. 2.7): implicit Gauss with two stages (eq. gaussAB,
// eq. gaussABab), Simpson quadrature of the closed form (eq. simpson), and
// the recursion of Alg. adaptiverk around any of them.
//
// A segment [s_in, s_out] is cut into dyadic pieces: piece (k, d) is the
// fraction [k, k+1] / 2^d counted from the near end.  Pieces are evaluated
// from the nearest to the farthest and combined with the group operation.
// Positions and the split test (dx kappa(xi_i) > c_RK at the method's stage
// points) are FP64 with a fixed operation order, so every split decision is
// reproducible; each step itself is FP32.
#include "rc_host.h"
#include "rc_internal.h"
#include "rc_steps.h"

namespace rc {
namespace {

struct GenArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    const float *kappa, *eps;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    float2* rec;
    uint8_t* hit;
    double2* sio;
    int d0;       // substeps = 2^d0 initial pieces
    double c_rk;  // > 0: recursion on
};

// Gauss stage positions from the far end of a piece: 1/2 -+ sqrt(3)/6.
__device__ inline double gauss_c0() { return 0.5 - sqrt(3.0) / 6.0; }
__device__ inline double gauss_c1() { return 0.5 + sqrt(3.0) / 6.0; }

// One leaf's segment: ray, box and the coefficients in both precisions.
struct Piecewise {
    double rho[3], r[3], lo[3], scale;  // scale = 2^level
    double s_in, s_out, rnorm;
    float kc[8], ec[8];
    double kd[8];
};

// Ray parameter of the stage point at c (from the far end) of piece (k, d).
__device__ inline double piece_s(const Piecewise& P, int64_t k, int d, double c) {
#pragma clang fp contract(off)
    double u = ((double)(k + 1) - c) * ldexp(1.0, -d);
    return P.s_in + u * (P.s_out - P.s_in);
}

__device__ inline double piece_dx(const Piecewise& P, int64_t k, int d) {
#pragma clang fp contract(off)
    return (piece_s(P, k, d, 0.0) - piece_s(P, k, d, 1.0)) * P.rnorm;
}

__device__ inline double ray_norm64(const double r[3]) {
#pragma clang fp contract(off)
    return sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
}

// Reference coordinates of ray parameter s.
__device__ inline void piece_xi(const Piecewise& P, double s, double xi[3]) {
#pragma clang fp contract(off)
    for (int k = 0; k < 3; k++) xi[k] = (P.rho[k] + s * P.r[k] - P.lo[k]) * P.scale;
}

// FP64 trilinear kappa: the split test's value (corners in order, each weight
// a product over the axes).
template <int KIND>
__device__ inline double kappa64(const Piecewise& P, double s) {
#pragma clang fp contract(off)
    if (KIND != RC_FIELD_TRILINEAR) return P.kd[0];
    double xi[3];
    piece_xi(P, s, xi);
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        double w = 1.0;
#pragma unroll
        for (int k = 0; k < 3; k++) w *= ((c >> k) & 1) ? xi[k] : 1.0 - xi[k];
        v += P.kd[c] * w;
    }
    return v;
}

template <int KIND>
__device__ inline void fields32(const Piecewise& P, double s, float& b, float& g) {
    if (KIND != RC_FIELD_TRILINEAR) {
        b = P.kc[0];
        g = P.ec[0];
        return;
    }
    double xi[3];
    piece_xi(P, s, xi);
    b = trilin(P.kc, (float)xi[0], (float)xi[1], (float)xi[2]);
    g = trilin(P.ec, (float)xi[0], (float)xi[1], (float)xi[2]);
}

template <int KIND, int METHOD>
__device__ inline bool split_test(const Piecewise& P, int64_t k, int d, double c_rk) {
#pragma clang fp contract(off)
    double dx = piece_dx(P, k, d);
    if (METHOD == RC_INT_GAUSS2) {
        if (dx * kappa64<KIND>(P, piece_s(P, k, d, gauss_c0())) > c_rk) return true;
        return dx * kappa64<KIND>(P, piece_s(P, k, d, gauss_c1())) > c_rk;
    }
    // RK4 (0, 1/2, 1/2, 1) and Simpson (0, 1/2, 1)
    if (dx * kappa64<KIND>(P, piece_s(P, k, d, 0.0)) > c_rk) return true;
    if (dx * kappa64<KIND>(P, piece_s(P, k, d, 0.5)) > c_rk) return true;
    return dx * kappa64<KIND>(P, piece_s(P, k, d, 1.0)) > c_rk;
}

template <int KIND, int METHOD>
__device__ inline float2 piece_step(const Piecewise& P, int64_t k, int d) {
    float h = (float)piece_dx(P, k, d);
    if (METHOD == RC_INT_GAUSS2) {
        float b0, b1, g0, g1;
        fields32<KIND>(P, piece_s(P, k, d, gauss_c0()), b0, g0);
        fields32<KIND>(P, piece_s(P, k, d, gauss_c1()), b1, g1);
        return gauss2_step(b0, b1, g0, g1, h);
    }
    float b0, bm, b1, g0, gm, g1;
    fields32<KIND>(P, piece_s(P, k, d, 0.0), b0, g0);
    fields32<KIND>(P, piece_s(P, k, d, 0.5), bm, gm);
    fields32<KIND>(P, piece_s(P, k, d, 1.0), b1, g1);
    if (METHOD == RC_INT_SIMPSON) return simpson_step(b0, bm, b1, g0, gm, g1, h);
    return rk4_step(b0, bm, b1, g0, gm, g1, h);
}

// The pieces of one segment, nearest first: descend while the recursion asks
// for a split, step, then move to the next piece (the far sibling, after
// climbing out of finished far halves).
template <int KIND, int METHOD>
__device__ inline float2 integrate_pieces(const Piecewise& P, int d0, double c_rk) {
    float2 acc = make_float2(1.0f, 0.0f);
    int64_t k = 0;
    int d = d0;
    const int64_t n0 = (int64_t)1 << d0;
    for (;;) {
        if (c_rk > 0.0)
            while (d < RC_ADAPT_MAXDEPTH && split_test<KIND, METHOD>(P, k, d, c_rk)) {
                k <<= 1;
                d++;
            }
        acc = seg_combine(acc, piece_step<KIND, METHOD>(P, k, d));
        while (d > d0 && (k & 1)) {
            k >>= 1;
            d--;
        }
        k++;
        if (d == d0 && k == n0) break;
    }
    return acc;
}

template <int KIND, int METHOD>
__global__ __launch_bounds__(256) void k_segments_general(GenArgs a) {
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        if (g >= ncand) continue;
        Pairing p = pair_candidate(a, g, w, nvis, ncand);
        float2 ab = make_float2(1.0f, 0.0f);
        if (p.hit) {
            Piecewise P;
            for (int k = 0; k < 3; k++) {
                P.rho[k] = p.rho[k];
                P.r[k] = p.rr[k];
                P.lo[k] = p.lo[k];
            }
            P.scale = ldexp(1.0, p.lv);
            P.s_in = p.s_in;
            P.s_out = p.s_out;
            P.rnorm = ray_norm64(p.rr);
            int nc = KIND == RC_FIELD_TRILINEAR ? 8 : 1;
            for (int c = 0; c < 8; c++) {
                int cc = c < nc ? c : 0;
                P.kc[c] = a.kappa[(int64_t)p.leaf * nc + cc];
                P.ec[c] = a.eps[(int64_t)p.leaf * nc + cc];
                P.kd[c] = (double)P.kc[c];
            }
            ab = integrate_pieces<KIND, METHOD>(P, a.d0, a.c_rk);
        }
        a.rec[g] = ab;
        if (a.hit) a.hit[g] = p.hit ? 1 : 0;
        if (a.sio) a.sio[g] = p.hit ? make_double2(p.s_in, p.s_out) : make_double2(0.0, 0.0);
    }
}

// ---------------------------------------------------------------------------
// adjoint with the recursion (c_rk > 0)
// ---------------------------------------------------------------------------

// Record of the subtree of piece (k0, dr): its pieces nearest first, the same
// split decisions as integrate_pieces (forced above the initial depth d0).
template <int KIND, int METHOD>
__device__ inline float2 eval_subtree(const Piecewise& P, int64_t k0, int dr, int d0, double c_rk) {
    float2 acc = make_float2(1.0f, 0.0f);
    int64_t k = k0;
    int d = dr;
    for (;;) {
        while (d < d0 || (d < RC_ADAPT_MAXDEPTH && split_test<KIND, METHOD>(P, k, d, c_rk))) {
            k <<= 1;
            d++;
        }
        acc = seg_combine(acc, piece_step<KIND, METHOD>(P, k, d));
        while (d > dr && (k & 1)) {
            k >>= 1;
            d--;
        }
        if (d == dr) break;
        k++;
    }
    return acc;
}

// One piece's step and its reverse: adds the corner adjoints of the stage
// values for (Abar, Bbar), the adjoints of the piece's (A, B); returns (A, B).
template <int KIND, int METHOD>
__device__ inline float2 piece_grad(const Piecewise& P, int64_t k, int d, float Abar, float Bbar,
                                    float grad[GRAD_MAX]) {
    constexpr int M = METHOD == RC_INT_GAUSS2 ? 2 : 3;
    float h = (float)piece_dx(P, k, d);
    double cs[3] = {0.0, 0.5, 1.0};
    if (METHOD == RC_INT_GAUSS2) {
        cs[0] = gauss_c0();
        cs[1] = gauss_c1();
    }
    double sp[3];
    float b[3], g[3], db[3] = {0.0f, 0.0f, 0.0f}, dg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < M; i++) {
        sp[i] = piece_s(P, k, d, cs[i]);
        fields32<KIND>(P, sp[i], b[i], g[i]);
    }
    float2 st;
    if (METHOD == RC_INT_GAUSS2) {
        st = gauss2_step(b[0], b[1], g[0], g[1], h);
        gauss2_step_bwd(b[0], b[1], g[0], g[1], h, Abar, Bbar, db[0], db[1], dg[0], dg[1]);
    } else if (METHOD == RC_INT_SIMPSON) {
        st = simpson_step(b[0], b[1], b[2], g[0], g[1], g[2], h);
        simpson_step_bwd(b[0], b[1], b[2], g[0], g[1], g[2], h, Abar, Bbar, db[0], db[1], db[2], dg[0], dg[1],
                         dg[2]);
    } else {
        st = rk4_step(b[0], b[1], b[2], g[0], g[1], g[2], h);
        rk4_step_bwd(b[0], b[1], b[2], g[0], g[1], h, Abar, Bbar, db[0], db[1], db[2], dg[0], dg[1], dg[2]);
    }
#pragma unroll
    for (int i = 0; i < M; i++) {
        if (KIND == RC_FIELD_TRILINEAR) {
            double xi[3];
            piece_xi(P, sp[i], xi);
            float x = (float)xi[0], y = (float)xi[1], z = (float)xi[2];
#pragma unroll
            for (int c = 0; c < 8; c++) {
                float w = ((c & 1) ? x : 1.0f - x) * ((c & 2) ? y : 1.0f - y) * ((c & 4) ? z : 1.0f - z);
                grad[c] = fmaf(db[i], w, grad[c]);
                grad[8 + c] = fmaf(dg[i], w, grad[8 + c]);
            }
        } else {
            grad[0] += db[i];
            grad[1] += dg[i];
        }
    }
    return st;
}

// Coefficient adjoints of one segment whose pieces follow the recursion.
// The pieces are visited nearest first as in integrate_pieces, starting from
// the whole segment (0, 0) with splits forced down to d0.  T, the product of
// the A of the nearer pieces, runs along; Js[d * 256] holds the intensity
// entering the current node at depth d from behind: on entering a node's near
// half it is the far half's record applied to the node's, on moving to the far
// half the node's own.  gT = g T_front and J enter the segment as in the
// closed-form adjoint; a piece receives dL/dA = gT T J_piece and dL/dB = gT T.
template <int KIND, int METHOD>
__device__ inline void pieces_grad(const Piecewise& P, int d0, double c_rk, float gT, float J, float* Js,
                                   float grad[GRAD_MAX]) {
    Js[0] = J;
    float T = 1.0f;
    int64_t k = 0;
    int d = 0;
    for (;;) {
        while (d < d0 || (d < RC_ADAPT_MAXDEPTH && split_test<KIND, METHOD>(P, k, d, c_rk))) {
            float2 far = eval_subtree<KIND, METHOD>(P, 2 * k + 1, d + 1, d0, c_rk);
            Js[(d + 1) * 256] = fmaf(far.x, Js[d * 256], far.y);
            k <<= 1;
            d++;
        }
        float gTT = gT * T;
        float2 st = piece_grad<KIND, METHOD>(P, k, d, gTT * Js[d * 256], gTT, grad);
        T *= st.x;
        while (d > 0 && (k & 1)) {
            k >>= 1;
            d--;
        }
        if (d == 0) break;
        k++;
        Js[d * 256] = Js[(d - 1) * 256];
    }
}

struct AdjGenArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    int64_t N;
    const float *kappa, *eps;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    const float2* adj_leaf;  // (g T_front, J_behind) per candidate
    float* partial;          // [(nchunks + nvis)][GRAD_MAX], entry (chunk w, pair v) at w + v
    int d0;
    double c_rk;
};

// One candidate per lane; the lanes of a wave chunk sum their gradients per
// (chunk w, pair v) key with a segmented shuffle scan (keys are
// non-decreasing across the lanes) and each key's last lane writes its slot.
template <int KIND, int METHOD>
__global__ __launch_bounds__(256) void k_adj_pieces(AdjGenArgs a) {
    __shared__ float Js[(RC_ADAPT_MAXDEPTH + 1) * 256];
    if (a.counts[3]) return;
    constexpr int NPAR = KIND == RC_FIELD_TRILINEAR ? 16 : 2;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        int64_t key = INT64_MAX;
        float grad[GRAD_MAX];
#pragma unroll
        for (int c = 0; c < GRAD_MAX; c++) grad[c] = 0.0f;
        if (g < ncand) {
            int64_t v = 0;
            Pairing p = pair_candidate(a, g, w, nvis, ncand, &v);
            key = w + v;
            if (p.hit) {
                Piecewise P;
                for (int k = 0; k < 3; k++) {
                    P.rho[k] = p.rho[k];
                    P.r[k] = p.rr[k];
                    P.lo[k] = p.lo[k];
                }
                P.scale = ldexp(1.0, p.lv);
                P.s_in = p.s_in;
                P.s_out = p.s_out;
                P.rnorm = ray_norm64(p.rr);
                int nc = KIND == RC_FIELD_TRILINEAR ? 8 : 1;
                for (int c = 0; c < 8; c++) {
                    int cc = c < nc ? c : 0;
                    P.kc[c] = a.kappa[(int64_t)p.leaf * nc + cc];
                    P.ec[c] = a.eps[(int64_t)p.leaf * nc + cc];
                    P.kd[c] = (double)P.kc[c];
                }
                float2 ad = a.adj_leaf[g];
                pieces_grad<KIND, METHOD>(P, a.d0, a.c_rk, ad.x, ad.y, Js + threadIdx.x, grad);
            }
        }
#pragma unroll
        for (int dd = 1; dd < WAVE; dd <<= 1) {
            int64_t kd = __shfl_up(key, dd);
            bool same = lane >= dd && kd == key;
#pragma unroll
            for (int c = 0; c < NPAR; c++) {
                float y = __shfl_up(grad[c], dd);
                if (same) grad[c] += y;
            }
        }
        int64_t knext = __shfl_down(key, 1);
        bool last = key != INT64_MAX && (lane == WAVE - 1 || knext != key);
        if (last) {
            float* dst = a.partial + key * GRAD_MAX;
#pragma unroll
            for (int c = 0; c < NPAR; c++) dst[c] = grad[c];
        }
    }
}

}  // namespace
}  // namespace rc

using namespace rc;

rc_status rc::rc_segments_general(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                  const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                                  const rc_tuning* tune, hipStream_t st) {
    GenArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.z = f->z;
    a.N = f->nleaves;
    a.kappa = fl->kappa;
    a.eps = fl->eps;
    a.vis_leaf = vf->vis_leaf;
    a.vis_cam = vf->vis_cam;
    a.vis_rect = vf->vis_rect;
    a.cand_offset = vf->cand_offset;
    a.counts = vf->counts;
    a.cand_chunk = vf->cand_chunk;
    a.cap_cand = vf->cap_cand;
    a.rec = (float2*)rec_leaf;
    a.hit = hit;
    a.sio = (double2*)sio;
    a.d0 = 0;
    while ((1 << a.d0) < in->substeps) a.d0++;
    a.c_rk = in->c_rk;
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 16384))), B(256);
    bool tri = fl->kind == RC_FIELD_TRILINEAR;
    switch (in->method) {
        case RC_INT_RK4:
            if (tri)
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_TRILINEAR, RC_INT_RK4>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_CONST, RC_INT_RK4>), G, B, 0, st, a);
            break;
        case RC_INT_GAUSS2:
            if (tri)
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_TRILINEAR, RC_INT_GAUSS2>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_CONST, RC_INT_GAUSS2>), G, B, 0, st, a);
            break;
        case RC_INT_SIMPSON:
            if (tri)
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_TRILINEAR, RC_INT_SIMPSON>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_segments_general<RC_FIELD_CONST, RC_INT_SIMPSON>), G, B, 0, st, a);
            break;
        default:
            return RC_EUNSUPPORTED;
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}

rc_status rc::rc_adjoint_pieces(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                const rc_integrator* in, const float* adj_leaf, float* partial, const rc_tuning* tune,
                                hipStream_t st) {
    AdjGenArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.z = f->z;
    a.N = f->nleaves;
    a.kappa = fl->kappa;
    a.eps = fl->eps;
    a.vis_leaf = vf->vis_leaf;
    a.vis_cam = vf->vis_cam;
    a.vis_rect = vf->vis_rect;
    a.cand_offset = vf->cand_offset;
    a.counts = vf->counts;
    a.cand_chunk = vf->cand_chunk;
    a.cap_cand = vf->cap_cand;
    a.adj_leaf = (const float2*)adj_leaf;
    a.partial = partial;
    a.d0 = 0;
    while ((1 << a.d0) < in->substeps) a.d0++;
    a.c_rk = in->c_rk;
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 3, 256 * 8))), B(256);
    bool tri = fl->kind == RC_FIELD_TRILINEAR;
    switch (in->method) {
        case RC_INT_RK4:
            if (tri)
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_TRILINEAR, RC_INT_RK4>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_CONST, RC_INT_RK4>), G, B, 0, st, a);
            break;
        case RC_INT_GAUSS2:
            if (tri)
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_TRILINEAR, RC_INT_GAUSS2>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_CONST, RC_INT_GAUSS2>), G, B, 0, st, a);
            break;
        case RC_INT_SIMPSON:
            if (tri)
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_TRILINEAR, RC_INT_SIMPSON>), G, B, 0, st, a);
            else
                hipLaunchKernelGGL((k_adj_pieces<RC_FIELD_CONST, RC_INT_SIMPSON>), G, B, 0, st, a);
            break;
        default:
            return RC_EUNSUPPORTED;
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}
