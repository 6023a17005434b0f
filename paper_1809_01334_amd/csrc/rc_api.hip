// rc_api.hip -- host-side entry points of librc: status names, sizes and the
// per-view camera set-up (Sec. 2.2).
#include <math.h>
#include <string.h>

#include <vector>

#include "rc_internal.h"
#include "rc_host.h"

using rc::Cam;

extern "C" const char* rc_strerror(rc_status s) {
    switch (s) {
        case RC_OK: return "ok";
        case RC_EINVAL: return "invalid argument";
        case RC_EUNSUPPORTED: return "unsupported combination";
        case RC_EWORKSPACE: return "workspace too small";
        case RC_ECAPACITY: return "capacity exceeded";
        case RC_EFOREST: return "leaves not in space-filling-curve order or overlapping";
        case RC_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

extern "C" size_t rc_camera_bytes(int32_t ncams) { return (ncams > 0 ? (size_t)ncams : 0) * sizeof(Cam); }

extern "C" int64_t rc_node_slots(const rc_index* ix, int32_t ncams) {
    if (!ix || ncams <= 0 || ix->maxlevel < 1) return 0;
    return (int64_t)ncams * (ix->level_begin[ix->maxlevel] - ix->level_begin[1]);
}

namespace rc {

// Derived camera quantities, evaluated in plain double arithmetic without
// contraction so that every implementation of the same formulas agrees.
static rc_status derive_camera(const double* raw, Cam& c) {
#pragma clang fp contract(off)
    memset(&c, 0, sizeof(c));
    for (int k = 0; k < 3; k++) {
        c.o[k] = raw[k];
        c.v[k] = raw[3 + k];
        c.t[k] = raw[6 + k];
        c.u[k] = raw[9 + k];
    }
    c.ell = raw[12];
    c.zfar = raw[13];
    double w = raw[14], h = raw[15];
    if (!(w >= 1.0 && w <= 32767.0 && w == floor(w))) return RC_EINVAL;
    if (!(h >= 1.0 && h <= 32767.0 && h == floor(h))) return RC_EINVAL;
    c.w = (int32_t)w;
    c.h = (int32_t)h;
    c.ortho = raw[16] != 0.0 ? 1 : 0;
    c.bg = raw[17];
    for (int k = 0; k < 18; k++)
        if (!isfinite(raw[k])) return RC_EINVAL;
    c.n = sqrt((c.v[0] * c.v[0] + c.v[1] * c.v[1]) + c.v[2] * c.v[2]);
    if (!(c.n > 0.0) || !(c.ell > 0.0) || !(c.zfar > c.n)) return RC_EINVAL;
    for (int k = 0; k < 3; k++) c.vh[k] = c.v[k] / c.n;
    auto dot = [](const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; };
    const double tol = 1e-9;
    if (fabs(dot(c.t, c.t) - 1.0) > tol || fabs(dot(c.u, c.u) - 1.0) > tol) return RC_EINVAL;
    if (fabs(dot(c.t, c.u)) > tol || fabs(dot(c.t, c.vh)) > tol || fabs(dot(c.u, c.vh)) > tol) return RC_EINVAL;
    // left-handed frame (t, u, v/n): t x u = -v/n
    double cr[3] = {c.t[1] * c.u[2] - c.t[2] * c.u[1], c.t[2] * c.u[0] - c.t[0] * c.u[2],
                    c.t[0] * c.u[1] - c.t[1] * c.u[0]};
    if (dot(cr, c.vh) > -1.0 + 1e-6) return RC_EINVAL;
    c.sc = c.n / c.ell;
    c.cx = (c.w - 1) / 2.0;
    c.cy = (c.h - 1) / 2.0;
    c.smin = c.ortho ? c.n : 1.0;
    c.smax = c.ortho ? c.zfar : c.zfar / c.n;
    return RC_OK;
}

}  // namespace rc

extern "C" rc_status rc_camera_prepare(const double* cams, int32_t ncams, void* dcams, int64_t* total_pixels,
                                       void* stream) {
    if (!cams || !dcams || ncams <= 0 || ncams > 32767) return RC_EINVAL;
    std::vector<Cam> hc((size_t)ncams);
    int64_t off = 0;
    for (int32_t k = 0; k < ncams; k++) {
        rc_status s = rc::derive_camera(cams + (size_t)k * RC_CAMERA_DOUBLES, hc[(size_t)k]);
        if (s != RC_OK) return s;
        hc[(size_t)k].img_off = off;
        off += (int64_t)hc[(size_t)k].w * hc[(size_t)k].h;
    }
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(dcams, hc.data(), sizeof(Cam) * hc.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return RC_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return RC_EHIP;
    if (total_pixels) *total_pixels = off;
    return RC_OK;
}

extern "C" size_t rc_workspace_bytes(const rc_forest* f, const rc_index* ix, int32_t ncams, const rc_vforest* vf) {
    if (!f) return 0;
    int64_t N = f->nleaves;
    int64_t nc = ncams > 0 ? ncams : 1;
    size_t b = 0;
    // rc_forest_index: status words, per-leaf current node, scan partials
    size_t bi = rc::IX_CUR + rc::align_up((size_t)N * 4) + rc::scan_partial_bytes(N, 8);
    b = bi > b ? bi : b;
    // rc_prune_visible: partials of the joint scan over leaves and node slots,
    // then the rectangles of the reduce pass (8 bytes per item)
    size_t bp = rc::prune_ws_bytes(f, ix, ncams);
    b = bp > b ? bp : b;
    // rc_segments_backward: gradient partials per (wave chunk, visible pair)
    if (vf) {
        size_t bb = rc::backward_ws_bytes(vf->cap_cand, vf->cap_vis, nc, N);
        b = bb > b ? bb : b;
    }
    return rc::align_up(b) + 256;
}
