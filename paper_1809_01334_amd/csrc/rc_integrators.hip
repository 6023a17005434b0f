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
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 256 * 8))), B(256);
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
