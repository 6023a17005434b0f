// rc_segments.hip -- leaf-level rendering (Sec. 3.2): every candidate
// (visible leaf, pixel of its rectangle) intersects the pixel's ray with the
// leaf and integrates the attenuation/emission ODE over the hit interval.
// Work is distributed by candidate index, so a wavefront covers 64
// consecutive candidates of one or a few leaves in SFC order regardless of
// how unevenly the leaves' rectangles are sized.
#include "rc_host.h"
#include "rc_internal.h"

namespace rc {
namespace {

struct SegArgs {
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
    float2* rec;
    uint8_t* hit;
    double2* sio;
    int eq;          // RC_FIELD_CONST_EQ: eps holds the equilibrium intensity I
    int64_t fstride; // floats between channels of kappa and eps (N * corners)
    int64_t rstride; // records between channels of rec (cap_cand)
};

// Channel ch of the segment (channels share the pairing and the geometry).
template <int KIND, int NSUB>
__device__ inline float2 integrate(const SegArgs& a, int64_t leaf, const SegGeom& sg, int ch) {
    const float* kap = a.kappa + ch * a.fstride;
    const float* eps = a.eps + ch * a.fstride;
    if (KIND == 1) return seg_rk4_const<NSUB>(kap[leaf], eps[leaf], sg.dx, a.nsub);
    float kc[8], ec[8];
    const float4* kp = reinterpret_cast<const float4*>(kap + leaf * 8);
    const float4* ep = reinterpret_cast<const float4*>(eps + leaf * 8);
    float4 k0 = kp[0], k1 = kp[1], e0 = ep[0], e1 = ep[1];
    kc[0] = k0.x; kc[1] = k0.y; kc[2] = k0.z; kc[3] = k0.w;
    kc[4] = k1.x; kc[5] = k1.y; kc[6] = k1.z; kc[7] = k1.w;
    ec[0] = e0.x; ec[1] = e0.y; ec[2] = e0.z; ec[3] = e0.w;
    ec[4] = e1.x; ec[5] = e1.y; ec[6] = e1.z; ec[7] = e1.w;
    return seg_rk4<NSUB>(kc, ec, sg, a.nsub);
}

// Closed-form constant coefficients: one candidate per lane, NCH channels.
template <int NCH>
__global__ __launch_bounds__(256) void k_segments_analytic(SegArgs a) {
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
        SegGeom sg;
        if (p.hit) sg = seg_geom(p.rho, p.rr, p.s_in, p.s_out, p.lo, p.lv);
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) {
            float2 ab = make_float2(1.0f, 0.0f);
            if (p.hit) {
                float k = a.kappa[ch * a.fstride + p.leaf], e = a.eps[ch * a.fstride + p.leaf];
                ab = a.eq ? seg_const_eq(k, e, sg.dx) : seg_const(k, e, sg.dx);
            }
            a.rec[ch * a.rstride + g] = ab;
        }
        if (a.hit) a.hit[g] = p.hit ? 1 : 0;
        if (a.sio) a.sio[g] = p.hit ? make_double2(p.s_in, p.s_out) : make_double2(0.0, 0.0);
    }
}

// RK4 segments.  Pairing runs one candidate per lane; hits go to a per-wave
// LDS queue and are integrated 64 at a time, so the RK4 stages run with every
// lane busy whatever the hit rate of the candidates.
constexpr int QCAP = 128;
struct HitQueue {
    int64_t g[QCAP];
    int32_t leaf[QCAP];
    float xf0[QCAP], xf1[QCAP], xf2[QCAP], d0[QCAP], d1[QCAP], d2[QCAP], dx[QCAP];
};

template <int KIND, int NSUB, int NCH>
__device__ inline void drain(const SegArgs& a, HitQueue& q, int e) {
    SegGeom sg;
    sg.xf[0] = q.xf0[e];
    sg.xf[1] = q.xf1[e];
    sg.xf[2] = q.xf2[e];
    sg.dxi[0] = q.d0[e];
    sg.dxi[1] = q.d1[e];
    sg.dxi[2] = q.d2[e];
    sg.dx = q.dx[e];
    int64_t g = q.g[e];
    int64_t leaf = q.leaf[e];
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) a.rec[ch * a.rstride + g] = integrate<KIND, NSUB>(a, leaf, sg, ch);
}

template <int KIND, int NSUB, int NCH>
__global__ __launch_bounds__(256) void k_segments_rk4(SegArgs a) {
    __shared__ HitQueue Q[256 / WAVE];
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    HitQueue& q = Q[threadIdx.x / WAVE];
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int qn = 0;  // queued hits, the same in every lane
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        bool h = false;
        SegGeom sg;
        int32_t leaf = 0;
        if (g < ncand) {
            Pairing p = pair_candidate(a, g, w, nvis, ncand);
            h = p.hit;
            leaf = p.leaf;
            if (h)
                sg = seg_geom(p.rho, p.rr, p.s_in, p.s_out, p.lo, p.lv);
            else
#pragma unroll
                for (int ch = 0; ch < NCH; ch++) a.rec[ch * a.rstride + g] = make_float2(1.0f, 0.0f);
            if (a.hit) a.hit[g] = h ? 1 : 0;
            if (a.sio) a.sio[g] = h ? make_double2(p.s_in, p.s_out) : make_double2(0.0, 0.0);
        }
        uint64_t mask = __ballot(h);
        if (h) {
            int pos = qn + __popcll(mask & below);
            q.g[pos] = g;
            q.leaf[pos] = leaf;
            q.xf0[pos] = sg.xf[0];
            q.xf1[pos] = sg.xf[1];
            q.xf2[pos] = sg.xf[2];
            q.d0[pos] = sg.dxi[0];
            q.d1[pos] = sg.dxi[1];
            q.d2[pos] = sg.dxi[2];
            q.dx[pos] = sg.dx;
        }
        qn += __popcll(mask);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (qn >= WAVE) {
            drain<KIND, NSUB, NCH>(a, q, qn - WAVE + lane);
            qn -= WAVE;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (lane < qn) drain<KIND, NSUB, NCH>(a, q, lane);
}

}  // namespace
}  // namespace rc

using namespace rc;

template <int KIND, int NCH>
static void launch_rk4(const SegArgs& a, int substeps, dim3 G, dim3 B, hipStream_t st) {
    if (NCH == 1) {
        switch (substeps) {
            case 1: hipLaunchKernelGGL((k_segments_rk4<KIND, 1, 1>), G, B, 0, st, a); break;
            case 2: hipLaunchKernelGGL((k_segments_rk4<KIND, 2, 1>), G, B, 0, st, a); break;
            case 4: hipLaunchKernelGGL((k_segments_rk4<KIND, 4, 1>), G, B, 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_segments_rk4<KIND, 8, 1>), G, B, 0, st, a); break;
            default: hipLaunchKernelGGL((k_segments_rk4<KIND, 0, 1>), G, B, 0, st, a); break;
        }
    } else if (substeps == 4) {
        hipLaunchKernelGGL((k_segments_rk4<KIND, 4, NCH>), G, B, 0, st, a);
    } else {
        hipLaunchKernelGGL((k_segments_rk4<KIND, 0, NCH>), G, B, 0, st, a);
    }
}

// Floats per leaf and channel of the field arrays, and per candidate of the records.
static int64_t field_corners(const rc_fields* fl) {
    return fl->kind == RC_FIELD_TRILINEAR ? 8 : fl->kind == RC_FIELD_SURFACE ? 4 : 1;
}

extern "C" rc_status rc_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, int32_t ncams,
                                 const rc_vforest* vf, const rc_integrator* in, float* rec_leaf, uint8_t* hit,
                                 double* sio, const rc_tuning* tune, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_fields(fl, in)) != RC_OK) return s;
    if ((s = check_vforest(vf, false)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || !rec_leaf || !vf->cand_chunk) return RC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // surface data goes with surface forests only
    if (is_surface(f) != (fl->kind == RC_FIELD_SURFACE)) return RC_EUNSUPPORTED;
    int64_t fstride = f->nleaves * field_corners(fl);
    bool fused = !is_curved(f) && (in->method == RC_INT_ANALYTIC || (in->method == RC_INT_RK4 && in->c_rk == 0.0));
    if (!fused) {
        // one channel at a time; the pairing outputs come with the first
        int64_t rstride = vf->cap_cand * (is_curved(f) ? 8 : 2);
        for (int ch = 0; ch < fl->nch; ch++) {
            rc_fields one = *fl;
            one.nch = 1;
            one.kappa = fl->kappa + ch * fstride;
            one.eps = fl->eps + ch * fstride;
            float* rec = rec_leaf + ch * rstride;
            uint8_t* h = ch == 0 ? hit : nullptr;
            double* io = ch == 0 ? sio : nullptr;
            if (is_volume(f))
                s = rc_volume_segments(f, &one, dcams, vf, in, rec, h, io, tune, st);
            else if (is_surface(f) && surface_degree(f) > 1)
                s = rc_surface_ho_segments(f, &one, dcams, vf, in, rec, h, io, tune, st);
            else if (is_surface(f))
                s = rc_surface_segments(f, &one, dcams, vf, in, rec, h, io, tune, st);
            else if (is_shell(f))
                s = rc_shell_segments(f, &one, dcams, vf, in, rec, h, io, tune, st);
            else
                s = rc_segments_general(f, &one, dcams, vf, in, rec, h, io, tune, st);
            if (s != RC_OK) return s;
        }
        return RC_OK;
    }
    SegArgs a{(const Cam*)dcams, f->level,       f->x,           f->y,         f->z,        f->nleaves,
              fl->kappa,        fl->eps,        in->substeps,   vf->vis_leaf, vf->vis_cam, vf->vis_rect,
              vf->cand_offset,  vf->counts,     vf->cand_chunk, vf->cap_cand, (float2*)rec_leaf, hit,
              (double2*)sio,    fl->kind == RC_FIELD_CONST_EQ ? 1 : 0, fstride, vf->cap_cand};
    unsigned grid = stride_grid(vf->cap_cand, 256, tuned(tune, 0, 8192));
    dim3 G(grid), B(256);
    int nch = fl->nch;
    if (in->method == RC_INT_ANALYTIC) {
        if (nch == 1)
            hipLaunchKernelGGL(k_segments_analytic<1>, G, B, 0, st, a);
        else if (nch == 2)
            hipLaunchKernelGGL(k_segments_analytic<2>, G, B, 0, st, a);
        else
            hipLaunchKernelGGL(k_segments_analytic<3>, G, B, 0, st, a);
    } else if (fl->kind == RC_FIELD_CONST) {
        if (nch == 1)
            launch_rk4<1, 1>(a, in->substeps, G, B, st);
        else if (nch == 2)
            launch_rk4<1, 2>(a, in->substeps, G, B, st);
        else
            launch_rk4<1, 3>(a, in->substeps, G, B, st);
    } else {
        if (nch == 1)
            launch_rk4<2, 1>(a, in->substeps, G, B, st);
        else if (nch == 2)
            launch_rk4<2, 2>(a, in->substeps, G, B, st);
        else
            launch_rk4<2, 3>(a, in->substeps, G, B, st);
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}
