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
    int64_t cap_cand;
    float2* rec;
    uint8_t* hit;
    double2* sio;
};

// KIND: 0 = constant analytic, 1 = constant RK4, 2 = trilinear RK4
template <int KIND>
__global__ __launch_bounds__(256) void k_segments(SegArgs a) {
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ncand; g += stride) {
        int64_t v = upper_index(a.cand_offset, 0, nvis, g);
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
        bool h = slab_hit(c, rho, rr, lo, hi, s_in, s_out);
        float2 ab = make_float2(1.0f, 0.0f);
        if (h) {
            SegGeom sg = seg_geom(rho, rr, s_in, s_out, lo, lv);
            if (KIND == 0) {
                ab = seg_const(a.kappa[leaf], a.eps[leaf], sg.dx);
            } else if (KIND == 1) {
                float kc[8], ec[8];
                float kv = a.kappa[leaf], ev = a.eps[leaf];
                for (int q = 0; q < 8; q++) {
                    kc[q] = kv;
                    ec[q] = ev;
                }
                ab = seg_rk4(kc, ec, sg, a.nsub);
            } else {
                float kc[8], ec[8];
                for (int q = 0; q < 8; q++) {
                    kc[q] = a.kappa[(int64_t)q * a.N + leaf];
                    ec[q] = a.eps[(int64_t)q * a.N + leaf];
                }
                ab = seg_rk4(kc, ec, sg, a.nsub);
            }
        }
        a.rec[g] = ab;
        if (a.hit) a.hit[g] = h ? 1 : 0;
        if (a.sio) a.sio[g] = h ? make_double2(s_in, s_out) : make_double2(0.0, 0.0);
    }
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, int32_t ncams,
                                 const rc_vforest* vf, const rc_integrator* in, float* rec_leaf, uint8_t* hit,
                                 double* sio, void* stream) {
    rc_status s = check_forest(f);
    if (s != RC_OK) return s;
    if ((s = check_fields(fl, in)) != RC_OK) return s;
    if ((s = check_vforest(vf, false)) != RC_OK) return s;
    if (!dcams || ncams <= 0 || !rec_leaf) return RC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    SegArgs a{(const Cam*)dcams, f->level,       f->x,           f->y,         f->z,        f->nleaves,
              fl->kappa,        fl->eps,        in->substeps,   vf->vis_leaf, vf->vis_cam, vf->vis_rect,
              vf->cand_offset,  vf->counts,     vf->cap_cand,   (float2*)rec_leaf, hit,    (double2*)sio};
    unsigned grid = stride_grid(vf->cap_cand, 256, 256 * 8);
    if (in->method == RC_INT_ANALYTIC)
        hipLaunchKernelGGL(k_segments<0>, dim3(grid), dim3(256), 0, st, a);
    else if (fl->kind == RC_FIELD_CONST)
        hipLaunchKernelGGL(k_segments<1>, dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_segments<2>, dim3(grid), dim3(256), 0, st, a);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
