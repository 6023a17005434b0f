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

using namespace rc;

namespace rc {
namespace {

constexpr int MAXSUB_BWD = 16;

// Hand the adjoint (gT, J) of node m (level l) at pixel (i, j) to its children.
__device__ inline void push_children(const FoldCtx& C, int cam, int64_t m, int l, int i, int j, float gT, float J,
                                     float2* adj_leaf, float2* adj_node) {
    int sb = view_bits(C.cams[cam], l, C.nx[m], C.ny[m], C.nz[m]);
    const int32_t* ch = C.child + m * 8;
    float2 rv[8];
    int kind[8];
    int64_t idx[8];
    for (int q = 0; q < 8; q++) {
        idx[q] = 0;
        kind[q] = child_slot(C, cam, ch[q ^ sb], l, i, j, idx[q]);
        rv[q] = kind[q] == 1 ? C.rec_leaf[idx[q]] : kind[q] == 2 ? C.rec_node[idx[q]] : make_float2(1.0f, 0.0f);
    }
    float Jq[8];
    float Jc = J;
    for (int q = 7; q >= 0; q--) {
        Jq[q] = Jc;
        Jc = fmaf(rv[q].x, Jc, rv[q].y);
    }
    float T = gT;
    for (int q = 0; q < 8; q++) {
        if (kind[q] == 1) adj_leaf[idx[q]] = make_float2(T, Jq[q]);
        if (kind[q] == 2) adj_node[idx[q]] = make_float2(T, Jq[q]);
        T *= rv[q].x;
    }
}

__global__ __launch_bounds__(256) void k_adj_root(FoldCtx C, int32_t root, int64_t npix, const float* dLdI,
                                                  float2* adj_leaf, float2* adj_node) {
    if (C.counts[3]) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
        int cam = camera_of_pixel(C.cams, C.ncams, p);
        const Cam& c = C.cams[cam];
        int64_t loc = p - c.img_off;
        int j = (int)(loc / c.w);
        int i = (int)(loc - (int64_t)j * c.w);
        float g = dLdI[p];
        float bg = (float)c.bg;
        if (root >= 0) {
            push_children(C, cam, root, 0, i, j, g, bg, adj_leaf, adj_node);
        } else if (root <= -2) {
            int64_t idx = 0;
            if (child_slot(C, cam, root, 0, i, j, idx) == 1) adj_leaf[idx] = make_float2(g, bg);
        }
    }
}

__global__ __launch_bounds__(256) void k_adj_level(FoldCtx C, int l, float2* adj_leaf, float2* adj_node) {
    if (C.counts[3]) return;
    int64_t s0 = C.L.slot_begin[l], s1 = C.L.slot_begin[l + 1];
    int64_t R0 = C.node_offset[s0], R1 = C.node_offset[s1];
    int64_t M = C.L.level_begin[l + 1] - C.L.level_begin[l];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = R0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < R1; g += stride) {
        int64_t slot = upper_index(C.node_offset, s0, s1, g);
        int64_t loc = slot - s0;
        int cam = (int)(loc / M);
        int64_t m = C.L.level_begin[l] + (loc - (int64_t)cam * M);
        Rect r = load_rect(C.node_rect + 4 * slot);
        int k = (int)(g - C.node_offset[slot]);
        int wr = r.width();
        int j = r.j0 + k / wr;
        int i = r.i0 + (k - (k / wr) * wr);
        float2 a = adj_node[g];
        push_children(C, cam, m, l, i, j, a.x, a.y, adj_leaf, adj_node);
    }
}

// Reverse of rk4_step: adds the adjoints of (b0, bm, b1, g0, gm, g1) given
// those of the step's (A, B).
__device__ inline void rk4_step_bwd(float b0, float bm, float b1, float g0, float gm, float h, float Abar, float Bbar,
                                    float& db0, float& dbm, float& db1, float& dg0, float& dgm, float& dg1) {
    (void)g0;
    float hh = 0.5f * h;
    // forward intermediates
    float A1 = fmaf(-hh, b0, 1.0f);
    float A2 = fmaf(-hh * bm, A1, 1.0f);
    float A3 = fmaf(-h * bm, A2, 1.0f);
    float B1 = hh * g0;
    float f1 = fmaf(-bm, B1, gm);
    float B2 = hh * f1;
    float f2 = fmaf(-bm, B2, gm);
    float B3 = h * f2;
    // A = 1 - (h/6) (b0 + 2 bm (A1 + A2) + b1 A3)
    float sa = -h * (1.0f / 6.0f) * Abar;
    db0 += sa;
    dbm += 2.0f * (A1 + A2) * sa;
    float A1b = 2.0f * bm * sa, A2b = 2.0f * bm * sa;
    db1 += A3 * sa;
    float A3b = b1 * sa;
    // B = (h/6) (g0 + 2 (f1 + f2) + f3)
    float sb = h * (1.0f / 6.0f) * Bbar;
    dg0 += sb;
    float f1b = 2.0f * sb, f2b = 2.0f * sb, f3b = sb;
    // f3 = g1 - b1 B3
    dg1 += f3b;
    db1 -= B3 * f3b;
    float B3b = -b1 * f3b;
    f2b += h * B3b;  // B3 = h f2
    // f2 = gm - bm B2
    dgm += f2b;
    dbm -= B2 * f2b;
    float B2b = -bm * f2b;
    f1b += hh * B2b;  // B2 = hh f1
    // f1 = gm - bm B1
    dgm += f1b;
    dbm -= B1 * f1b;
    float B1b = -bm * f1b;
    dg0 += hh * B1b;  // B1 = hh g0
    // A3 = 1 - h bm A2
    dbm -= h * A2 * A3b;
    A2b -= h * bm * A3b;
    // A2 = 1 - hh bm A1
    dbm -= hh * A1 * A2b;
    A1b -= hh * bm * A2b;
    // A1 = 1 - hh b0
    db0 -= hh * A1b;
}

__device__ inline void trilin_weights(float x, float y, float z, float w[8]) {
    float x0 = 1.0f - x, y0 = 1.0f - y, z0 = 1.0f - z;
    w[0] = x0 * y0 * z0;
    w[1] = x * y0 * z0;
    w[2] = x0 * y * z0;
    w[3] = x * y * z0;
    w[4] = x0 * y0 * z;
    w[5] = x * y0 * z;
    w[6] = x0 * y * z;
    w[7] = x * y * z;
}

// Gradient of one segment's (A, B) contribution: grad[0..nc) kappa corners,
// grad[nc..2nc) eps corners.  gT = g T_front, J = intensity from behind.
template <int KIND>
__device__ inline void segment_grad(const float kc[8], const float ec[8], const SegGeom& sg, int nsub, float gT,
                                    float J, float grad[GRAD_MAX]) {
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
    // forward: substep values and the intensity entering each substep
    float inv = 1.0f / (float)nsub;
    float h = sg.dx * inv;
    float bs[2 * MAXSUB_BWD + 1], gs[2 * MAXSUB_BWD + 1];
    float px[2 * MAXSUB_BWD + 1], py[2 * MAXSUB_BWD + 1], pz[2 * MAXSUB_BWD + 1];
    int np = 2 * nsub + 1;
    for (int p = 0; p < np; p++) {
        float t = (float)p * (0.5f * inv);
        if (p % 2 == 0) t = (float)(p / 2) * inv;
        px[p] = fmaf(t, sg.dxi[0], sg.xf[0]);
        py[p] = fmaf(t, sg.dxi[1], sg.xf[1]);
        pz[p] = fmaf(t, sg.dxi[2], sg.xf[2]);
        bs[p] = trilin(kc, px[p], py[p], pz[p]);
        gs[p] = trilin(ec, px[p], py[p], pz[p]);
    }
    float Iin[MAXSUB_BWD], av[MAXSUB_BWD];
    float Ic = J;
    for (int q = 0; q < nsub; q++) {
        float2 s = rk4_step(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], gs[2 * q + 2], h);
        Iin[q] = Ic;
        av[q] = s.x;
        Ic = fmaf(s.x, Ic, s.y);
    }
    // reverse: G = dL/d(intensity leaving substep q), nearest first
    float dbs[2 * MAXSUB_BWD + 1], dgs[2 * MAXSUB_BWD + 1];
    for (int p = 0; p < np; p++) {
        dbs[p] = 0.0f;
        dgs[p] = 0.0f;
    }
    float G = gT;
    for (int q = nsub - 1; q >= 0; q--) {
        rk4_step_bwd(bs[2 * q], bs[2 * q + 1], bs[2 * q + 2], gs[2 * q], gs[2 * q + 1], h, G * Iin[q], G,
                     dbs[2 * q], dbs[2 * q + 1], dbs[2 * q + 2], dgs[2 * q], dgs[2 * q + 1], dgs[2 * q + 2]);
        G *= av[q];
    }
    if (KIND == 1) {
        float sk = 0.0f, se = 0.0f;
        for (int p = 0; p < np; p++) {
            sk += dbs[p];
            se += dgs[p];
        }
        grad[0] = sk;
        grad[1] = se;
        return;
    }
    for (int c = 0; c < 16; c++) grad[c] = 0.0f;
    for (int p = 0; p < np; p++) {
        float w[8];
        trilin_weights(px[p], py[p], pz[p], w);
        for (int c = 0; c < 8; c++) {
            grad[c] = fmaf(dbs[p], w[c], grad[c]);
            grad[8 + c] = fmaf(dgs[p], w[c], grad[8 + c]);
        }
    }
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
    int64_t cap_cand;
    const float2* adj_leaf;
    float* partial;  // [(nchunks + nvis)][GRAD_MAX], entry (chunk w, pair v) at w + v
};

// One wavefront per 64 consecutive candidates; per-pair sums by a segmented
// shuffle scan in a fixed order.
template <int KIND>
__global__ __launch_bounds__(256) void k_adj_leaf(LeafAdjArgs a) {
    if (a.counts[3]) return;
    constexpr int NPAR = KIND == 2 ? 16 : 2;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int64_t nchunks = (ncand + WAVE - 1) / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t wstride = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t w = wave; w < nchunks; w += wstride) {
        int64_t g = w * WAVE + lane;
        float grad[GRAD_MAX];
        for (int c = 0; c < GRAD_MAX; c++) grad[c] = 0.0f;
        int64_t key = -1;
        if (g < ncand) {
            int64_t v = upper_index(a.cand_offset, 0, nvis, g);
            key = v;
            int32_t leaf = a.vis_leaf[v];
            const Cam& c = a.cams[a.vis_cam[v]];
            Rect r = load_rect(a.vis_rect + 4 * v);
            int k = (int)(g - a.cand_offset[v]);
            int wr = r.width();
            int j = r.j0 + k / wr;
            int i = r.i0 + (k - (k / wr) * wr);
            int lv = a.level[leaf];
            double lo[3], hi[3], rho[3], rr[3], s_in, s_out;
            node_box(lv, a.x[leaf], a.y[leaf], a.z[leaf], lo, hi);
            pixel_ray(c, i, j, rho, rr);
            if (slab_hit(c, rho, rr, lo, hi, s_in, s_out)) {
                SegGeom sg = seg_geom(rho, rr, s_in, s_out, lo, lv);
                float2 ad = a.adj_leaf[g];
                float kc[8], ec[8];
                if (KIND == 2) {
                    for (int q = 0; q < 8; q++) {
                        kc[q] = a.kappa[(int64_t)q * a.N + leaf];
                        ec[q] = a.eps[(int64_t)q * a.N + leaf];
                    }
                } else {
                    for (int q = 0; q < 8; q++) {
                        kc[q] = a.kappa[leaf];
                        ec[q] = a.eps[leaf];
                    }
                }
                segment_grad<KIND>(kc, ec, sg, a.nsub, ad.x, ad.y, grad);
            }
        }
        // segmented inclusive scan over lanes with equal (sorted) keys
        for (int d = 1; d < WAVE; d <<= 1) {
            int64_t kd = __shfl_up(key, d);
            bool same = lane >= d && kd == key;
            for (int c = 0; c < NPAR; c++) {
                float y = __shfl_up(grad[c], d);
                if (same) grad[c] += y;
            }
        }
        int64_t knext = __shfl_down(key, 1);
        bool last = (lane == WAVE - 1) || knext != key;
        if (key >= 0 && last) {
            float* dst = a.partial + (w + key) * GRAD_MAX;
            for (int c = 0; c < NPAR; c++) dst[c] = grad[c];
        }
    }
}

// Per visible pair: add its chunk partials in chunk order.
__global__ __launch_bounds__(256) void k_grad_pairs(const int64_t* counts, int64_t cap_cand, const int64_t* cand_offset,
                                                    const float* partial, float* gvis, int npar) {
    if (counts[3]) return;
    int64_t nvis = counts[0];
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvis; v += stride) {
        int64_t c0 = cand_offset[v], c1 = cand_offset[v + 1];
        if (c1 > cap_cand) c1 = cap_cand;
        float acc[GRAD_MAX];
        for (int c = 0; c < GRAD_MAX; c++) acc[c] = 0.0f;
        if (c1 > c0) {
            int64_t w0 = c0 / WAVE, w1 = (c1 - 1) / WAVE;
            for (int64_t w = w0; w <= w1; w++) {
                const float* src = partial + (w + v) * GRAD_MAX;
                for (int c = 0; c < npar; c++) acc[c] += src[c];
            }
        }
        for (int c = 0; c < npar; c++) gvis[v * GRAD_MAX + c] = acc[c];
    }
}

// Per leaf: sum over cameras in camera order into the coefficient layout.
__global__ __launch_bounds__(256) void k_grad_leaves(const int64_t* counts, int64_t N, int ncams, const int32_t* leaf_vis,
                                                     const float* gvis, int nc, float* dk, float* de, int accumulate) {
    if (counts[3]) return;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < N; l += stride) {
        float acc[GRAD_MAX];
        for (int c = 0; c < GRAD_MAX; c++) acc[c] = 0.0f;
        for (int cam = 0; cam < ncams; cam++) {
            int32_t v = leaf_vis[(int64_t)cam * N + l];
            if (v < 0) continue;
            for (int c = 0; c < 2 * nc; c++) acc[c] += gvis[(int64_t)v * GRAD_MAX + c];
        }
        for (int c = 0; c < nc; c++) {
            int64_t o = (int64_t)c * N + l;
            dk[o] = accumulate ? dk[o] + acc[c] : acc[c];
            de[o] = accumulate ? de[o] + acc[nc + c] : acc[nc + c];
        }
    }
}

}  // namespace
}  // namespace rc

extern "C" rc_status rc_segments_backward(const rc_forest* f, const rc_index* ix, const rc_fields* fl,
                                          const void* dcams, int32_t ncams, const rc_vforest* vf,
                                          const rc_integrator* in, const float* rec_leaf, const float* rec_node,
                                          int64_t npix, const float* dLdI, float* adj_leaf, float* adj_node,
                                          float* dk, float* de, int32_t accumulate, void* ws, size_t ws_bytes,
                                          void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_index(ix)) != RC_OK) return s;
    if ((s = check_fields(fl, in)) != RC_OK) return s;
    if ((s = check_vforest(vf, ix->maxlevel >= 1)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || npix <= 0 || !rec_leaf || !dLdI || !adj_leaf || !dk || !de) return RC_EINVAL;
    bool nodes = rc_node_slots(ix, ncams) > 0;
    if (nodes && (!rec_node || !adj_node)) return RC_EINVAL;
    if (in->method == RC_INT_RK4 && in->substeps > MAXSUB_BWD) return RC_EUNSUPPORTED;
    if (!ws || ws_bytes < rc_workspace_bytes(f, ix, ncams, vf)) return RC_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;

    FoldCtx C = make_fold_ctx(f, ix, dcams, ncams, vf, rec_leaf, rec_node);
    hipLaunchKernelGGL(k_adj_root, dim3(stride_grid(npix, 256, 256 * 16)), dim3(256), 0, st, C, ix->root, npix, dLdI,
                       (float2*)adj_leaf, (float2*)adj_node);
    RC_HIP(hipGetLastError());
    unsigned grid = stride_grid(vf->cap_rec, 256, 256 * 16);
    for (int l = 1; l < ix->maxlevel; l++) {
        if (ix->level_begin[l + 1] == ix->level_begin[l]) continue;
        hipLaunchKernelGGL(k_adj_level, dim3(grid), dim3(256), 0, st, C, l, (float2*)adj_leaf, (float2*)adj_node);
        RC_HIP(hipGetLastError());
    }

    int64_t nchunks = (vf->cap_cand + WAVE - 1) / WAVE;
    float* partial = (float*)ws;
    float* gvis = (float*)((char*)ws + align_up((size_t)(nchunks + vf->cap_vis + 1) * GRAD_MAX * sizeof(float)));
    LeafAdjArgs la{(const Cam*)dcams, f->level,       f->x,          f->y,         f->z,
                   f->nleaves,        fl->kappa,      fl->eps,       in->substeps, vf->vis_leaf,
                   vf->vis_cam,       vf->vis_rect,   vf->cand_offset, vf->counts, vf->cap_cand,
                   (const float2*)adj_leaf, partial};
    unsigned lg = stride_grid(nchunks * WAVE, 256, 256 * 8);
    int nc = fl->kind == RC_FIELD_TRILINEAR ? 8 : 1;
    if (in->method == RC_INT_ANALYTIC)
        hipLaunchKernelGGL(k_adj_leaf<0>, dim3(lg), dim3(256), 0, st, la);
    else if (fl->kind == RC_FIELD_CONST)
        hipLaunchKernelGGL(k_adj_leaf<1>, dim3(lg), dim3(256), 0, st, la);
    else
        hipLaunchKernelGGL(k_adj_leaf<2>, dim3(lg), dim3(256), 0, st, la);
    RC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_pairs, dim3(stride_grid(vf->cap_vis, 256, 256 * 16)), dim3(256), 0, st, vf->counts,
                       vf->cap_cand, vf->cand_offset, partial, gvis, 2 * nc);
    RC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_leaves, dim3(stride_grid(f->nleaves, 256, 256 * 16)), dim3(256), 0, st, vf->counts,
                       f->nleaves, ncams, vf->leaf_vis, gvis, nc, dk, de, accumulate);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
