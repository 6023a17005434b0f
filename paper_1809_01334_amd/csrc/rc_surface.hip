// rc_surface.hip -- ray segments of surface forests (Sec. 2.8): each candidate
// (visible leaf, pixel of its rectangle) intersects the pixel's ray with the
// leaf's tree patch (App. A.1, the bilinear case) and keeps the hits that lie
// in the leaf's parameter square, as zero-length records (s, s, A, B) from
// the thin-surface model.  Compositing merges them by depth like the shell's
// intervals.
#include "rc_host.h"
#include "rc_surface.h"

namespace rc {
namespace {

struct SurfArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y;
    const float4 *As, *Is;  // corner transparency and intensity, one float4 per leaf
    const double* geom;     // 12 doubles per tree
    int64_t tb[7];
    int ntrees;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    float4* rec;   // 2 per candidate
    uint8_t* hit;  // hits in the leaf, 0 .. 2
    double* sio;   // 4 per candidate
};

__device__ inline void surf_candidate(const SurfArgs& a, int64_t g, int64_t v, const Cam& c) {
    int32_t leaf = a.vis_leaf[v];
    Rect r = load_rect(a.vis_rect + 4 * v);
    int k = (int)(g - a.cand_offset[v]);
    int i, j;
    rect_pixel(r, k, i, j);
    double rho[3], rr[3];
    pixel_ray(c, i, j, rho, rr);
    int t = 0;
    while (t + 1 < a.ntrees && leaf >= a.tb[t + 1]) t++;
    SurfPatch S = surf_patch(a.geom + 12 * t);
    double hs[2], h1[2], h2[2];
    int nh = surf_hits(c, S, rho, rr, hs, h1, h2);
    int lv = a.level[leaf];
    uint32_t x = a.x[leaf], y = a.y[leaf];
    float4 o0 = make_float4(1.0f, 0.0f, 1.0f, 0.0f), o1 = o0;
    double s0 = 0.0, s1 = 0.0;
    int cnt = 0;
    if (nh > 0) {
        float4 As = a.As[leaf], Is = a.Is[leaf];
#pragma unroll
        for (int m = 0; m < 2; m++) {
            if (m >= nh) break;
            double u, w;
            double t1 = m == 0 ? h1[0] : h1[1], t2 = m == 0 ? h2[0] : h2[1], s = m == 0 ? hs[0] : hs[1];
            if (!surf_leaf_has(lv, x, y, t1, t2, u, w)) continue;
            float2 ab = surf_value(As, Is, S, rr, t1, t2, u, w);
            float4 rec = make_float4((float)s, (float)s, ab.x, ab.y);
            if (cnt == 0) {
                o0 = rec;
                s0 = s;
            } else {
                o1 = rec;
                s1 = s;
            }
            cnt++;
        }
    }
    a.rec[2 * g] = o0;
    a.rec[2 * g + 1] = o1;
    if (a.hit) a.hit[g] = (uint8_t)cnt;
    if (a.sio) {
        a.sio[4 * g] = s0;
        a.sio[4 * g + 1] = s0;
        a.sio[4 * g + 2] = s1;
        a.sio[4 * g + 3] = s1;
    }
}

// One candidate per lane; the camera comes through the scalar cache when the
// wave's candidates share it.
__global__ __launch_bounds__(256) void k_segments_surface(SurfArgs a) {
    if (a.counts[3]) return;
    int64_t nvis = a.counts[0];
    int64_t ncand = a.counts[1] < a.cap_cand ? a.counts[1] : a.cap_cand;
    int lane = threadIdx.x & (WAVE - 1);
    int64_t wave = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t w = wave; w * WAVE < ncand; w += nw) {
        int64_t g = w * WAVE + lane;
        if (g >= ncand) continue;
        int64_t v = cand_pair(a.cand_offset, a.cand_chunk, g, w, nvis, ncand);
        int cam = a.vis_cam[v];
        int c0 = __builtin_amdgcn_readfirstlane(cam);
        if (__all(cam == c0)) {
            Cam cs = load_cam_scalar(a.cams, c0);
            surf_candidate(a, g, v, cs);
        } else {
            surf_candidate(a, g, v, a.cams[cam]);
        }
    }
}

}  // namespace
}  // namespace rc

using namespace rc;

rc_status rc::rc_surface_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                  const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                                  const rc_tuning* tune, hipStream_t st) {
    if (fl->kind != RC_FIELD_SURFACE || in->method != RC_INT_ANALYTIC) return RC_EUNSUPPORTED;
    SurfArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.As = (const float4*)fl->kappa;
    a.Is = (const float4*)fl->eps;
    a.geom = f->geom_table;
    for (int k = 0; k < 7; k++) a.tb[k] = k <= f->ntrees ? f->tree_begin[k] : f->nleaves;
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
    hipLaunchKernelGGL(k_segments_surface, dim3(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 8192))), dim3(256),
                       0, st, a);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
