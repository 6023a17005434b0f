// rc_internal.h -- device-side building blocks of librc (gfx950).
//
// Geometry predicates here decide integers (visibility rectangles, hit or
// miss), so they run in FP64 with floating-point contraction switched off and
// with correctly rounded division: the same sequence of IEEE operations
// always gives the same bits.  Segment values run in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

constexpr int QMAX = RC_QMAXLEVEL;
constexpr double QSCALE = 1.0 / 524288.0;  // 2^-19, exact

// Derived camera (Sec. 2.2), prepared on the host by rc_camera_prepare.
struct Cam {
    double o[3], v[3], t[3], u[3], vh[3];
    double ell, n, zfar;
    double sc;          // n / ell: projection-plane to pixel scale
    double cx, cy;      // (w - 1) / 2, (h - 1) / 2
    double smin, smax;  // ray-parameter clip range: [1, zfar / n] or [n, zfar]
    double bg;          // background intensity I_b
    int32_t w, h, ortho, pad;
    int64_t img_off;    // first pixel of this camera in the concatenated images
};

struct Rect {
    int i0, i1, j0, j1;
    __device__ __host__ bool empty() const { return i0 > i1 || j0 > j1; }
    __device__ __host__ int width() const { return i1 - i0 + 1; }
    __device__ __host__ int64_t area() const { return empty() ? 0 : (int64_t)(i1 - i0 + 1) * (j1 - j0 + 1); }
    __device__ __host__ bool contains(int i, int j) const { return i >= i0 && i <= i1 && j >= j0 && j <= j1; }
};

// Pixel (i, j) of the k-th pixel (row-major) of rectangle r.  Below 2^22 the
// row comes from an FP32 reciprocal estimate (relative error under 2e-7, so
// off by at most one) and one exact correction step.
__device__ inline void rect_pixel(const Rect& r, int k, int& i, int& j) {
    int wr = r.width();
    if (k < (1 << 22)) {
        int q = (int)((float)k * __builtin_amdgcn_rcpf((float)wr));
        int rem = k - q * wr;
        if (rem < 0) {
            q--;
            rem += wr;
        } else if (rem >= wr) {
            q++;
            rem -= wr;
        }
        j = r.j0 + q;
        i = r.i0 + rem;
    } else {
        int q = (int)((uint32_t)k / (uint32_t)wr);
        j = r.j0 + q;
        i = r.i0 + (k - q * wr);
    }
}

__device__ inline Rect load_rect(const int16_t* r4) {
    // one 64-bit load of four int16
    uint64_t bits = *reinterpret_cast<const uint64_t*>(r4);
    Rect r;
    r.i0 = (int16_t)(bits & 0xffff);
    r.i1 = (int16_t)((bits >> 16) & 0xffff);
    r.j0 = (int16_t)((bits >> 32) & 0xffff);
    r.j1 = (int16_t)((bits >> 48) & 0xffff);
    return r;
}

__device__ inline void store_rect(int16_t* r4, const Rect& r) {
    uint64_t bits = (uint64_t)(uint16_t)r.i0 | ((uint64_t)(uint16_t)r.i1 << 16) |
                    ((uint64_t)(uint16_t)r.j0 << 32) | ((uint64_t)(uint16_t)r.j1 << 48);
    *reinterpret_cast<uint64_t*>(r4) = bits;
}

// Position of a node's anchor on the space-filling curve (Morton order, x in
// the lowest bit of every triple), and the curve length a level-l node spans.
__device__ inline uint64_t morton(uint32_t x, uint32_t y, uint32_t z) {
    uint64_t k = 0;
    for (int b = 0; b < QMAX; b++) {
        k |= (uint64_t)((x >> b) & 1u) << (3 * b);
        k |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

__device__ inline uint64_t curve_span(int level) { return (uint64_t)1 << (3 * (QMAX - level)); }

// Box of a node in the unit cube: exact dyadic values.
__device__ inline void node_box(int level, uint32_t x, uint32_t y, uint32_t z, double lo[3], double hi[3]) {
    uint32_t len = 1u << (QMAX - level);
    lo[0] = (double)x * QSCALE;
    lo[1] = (double)y * QSCALE;
    lo[2] = (double)z * QSCALE;
    hi[0] = (double)(x + len) * QSCALE;
    hi[1] = (double)(y + len) * QSCALE;
    hi[2] = (double)(z + len) * QSCALE;
}

// ---------------------------------------------------------------------------
// canonical visibility rectangle (Sec. 2.2: camera-aligned AABB of the box,
// projected to the image).  Every operation is monotone, so a child's
// rectangle lies inside its parent's bit for bit.
// ---------------------------------------------------------------------------

__device__ inline double extent_lo(const double a[3], const double lo[3], const double hi[3], const double o[3]) {
#pragma clang fp contract(off)
    double p0 = a[0] * ((a[0] >= 0.0 ? lo[0] : hi[0]) - o[0]);
    double p1 = a[1] * ((a[1] >= 0.0 ? lo[1] : hi[1]) - o[1]);
    double p2 = a[2] * ((a[2] >= 0.0 ? lo[2] : hi[2]) - o[2]);
    return (p0 + p1) + p2;
}

__device__ inline double extent_hi(const double a[3], const double lo[3], const double hi[3], const double o[3]) {
#pragma clang fp contract(off)
    double p0 = a[0] * ((a[0] >= 0.0 ? hi[0] : lo[0]) - o[0]);
    double p1 = a[1] * ((a[1] >= 0.0 ? hi[1] : lo[1]) - o[1]);
    double p2 = a[2] * ((a[2] >= 0.0 ? hi[2] : lo[2]) - o[2]);
    return (p0 + p1) + p2;
}

__device__ inline void axis_pixels(const Cam& c, double e0, double e1, double z0, double z1, double ctr, int npx,
                                   int& k0, int& k1) {
#pragma clang fp contract(off)
    double p0, p1;
    if (c.ortho) {
        p0 = e0 / c.ell + ctr;
        p1 = e1 / c.ell + ctr;
    } else {
        double q0 = (e0 >= 0.0) ? e0 / z1 : e0 / z0;
        double q1 = (e1 >= 0.0) ? e1 / z0 : e1 / z1;
        p0 = q0 * c.sc + ctr;
        p1 = q1 * c.sc + ctr;
    }
    double a = ceil(p0);
    double b = floor(p1);
    if (a < 0.0) a = 0.0;
    if (b > (double)(npx - 1)) b = (double)(npx - 1);
    if (a > b) {
        k0 = 1;
        k1 = 0;
    } else {
        k0 = (int)a;
        k1 = (int)b;
    }
}

// Pixel rectangle of a camera-aligned box [x0, x1] x [y0, y1] x [z0, z1]
// (coordinates along t, u and vh from the eye), clipped to depth [n, f].
__device__ inline Rect cam_rect(const Cam& c, double x0, double x1, double y0, double y1, double z0, double z1) {
    Rect r{1, 0, 1, 0};
    if (z1 < c.n || z0 > c.zfar) return r;
    double zc0 = z0 < c.n ? c.n : z0;
    double zc1 = z1 > c.zfar ? c.zfar : z1;
    Rect q;
    axis_pixels(c, x0, x1, zc0, zc1, c.cx, c.w, q.i0, q.i1);
    axis_pixels(c, y0, y1, zc0, zc1, c.cy, c.h, q.j0, q.j1);
    if (q.empty()) return r;
    return q;
}

__device__ inline Rect box_rect(const Cam& c, const double lo[3], const double hi[3]) {
    double z0 = extent_lo(c.vh, lo, hi, c.o);
    double z1 = extent_hi(c.vh, lo, hi, c.o);
    if (z1 < c.n || z0 > c.zfar) return Rect{1, 0, 1, 0};
    double x0 = extent_lo(c.t, lo, hi, c.o), x1 = extent_hi(c.t, lo, hi, c.o);
    double y0 = extent_lo(c.u, lo, hi, c.o), y1 = extent_hi(c.u, lo, hi, c.o);
    return cam_rect(c, x0, x1, y0, y1, z0, z1);
}

// ---------------------------------------------------------------------------
// pixel ray (eq. ray) and the slab test against a box
// ---------------------------------------------------------------------------

// MODE 0: perspective, 1: orthographic, -1: read from the camera.  A wave
// whose lanes share one camera branches once on its mode, so the lanes do not
// compute both rays and select.
template <int MODE = -1>
__device__ inline void pixel_ray(const Cam& c, int i, int j, double rho[3], double r[3]) {
#pragma clang fp contract(off)
    double a = c.ell * ((double)i - c.cx);
    double b = c.ell * ((double)j - c.cy);
    const bool ortho = MODE < 0 ? c.ortho != 0 : MODE == 1;
    for (int k = 0; k < 3; k++) {
        double off = a * c.t[k] + b * c.u[k];
        if (ortho) {
            rho[k] = c.o[k] + off;
            r[k] = c.vh[k];
        } else {
            rho[k] = c.o[k];
            r[k] = c.v[k] + off;
        }
    }
}

// Hit interval of the ray in the box, clipped to [smin, smax].  A face enters
// as (face - rho) * (1 / r_k), so two boxes sharing a face produce the same
// crossing parameter; a ray parallel to a slab is inside iff lo <= rho < hi.
__device__ inline bool slab_hit(const Cam& c, const double rho[3], const double r[3], const double lo[3],
                                const double hi[3], double& s_in, double& s_out) {
#pragma clang fp contract(off)
    double a = c.smin, b = c.smax;
    bool ok = true;
    for (int k = 0; k < 3; k++) {
        if (r[k] != 0.0) {
            double inv = 1.0 / r[k];
            double t0 = (lo[k] - rho[k]) * inv;
            double t1 = (hi[k] - rho[k]) * inv;
            a = fmax(a, fmin(t0, t1));
            b = fmin(b, fmax(t0, t1));
        } else if (!(rho[k] >= lo[k] && rho[k] < hi[k])) {
            ok = false;
        }
    }
    s_in = a;
    s_out = b;
    return ok && (b > a);
}

// View order of a node's children: child c is visited at position c ^ bits,
// bit k set when the camera lies on the high side of the node's k-midplane
// (orthographic: when the view direction points toward decreasing k).
__device__ inline int view_bits(const Cam& c, int level, uint32_t x, uint32_t y, uint32_t z) {
    if (c.ortho) return (c.vh[0] < 0.0 ? 1 : 0) | (c.vh[1] < 0.0 ? 2 : 0) | (c.vh[2] < 0.0 ? 4 : 0);
    uint32_t half = 1u << (QMAX - level - 1);
    double m0 = (double)(x + half) * QSCALE;
    double m1 = (double)(y + half) * QSCALE;
    double m2 = (double)(z + half) * QSCALE;
    return (c.o[0] >= m0 ? 1 : 0) | (c.o[1] >= m1 ? 2 : 0) | (c.o[2] >= m2 ? 4 : 0);
}

// Child of an internal node as seen by one camera: pixel rectangle and the
// record index of its (0,0) corner pixel; off >= 0 indexes internal-node
// records, off < 0 leaf records at -1 - off.  An empty rectangle marks a child
// that is absent or invisible.  16 bytes, loaded as one 128-bit word.
struct ChildDesc {
    int16_t i0, i1, j0, j1;
    int64_t off;
};

__device__ inline ChildDesc load_desc(const ChildDesc* p) {
    uint4 u = *reinterpret_cast<const uint4*>(p);
    ChildDesc d;
    d.i0 = (int16_t)(u.x & 0xffff);
    d.i1 = (int16_t)(u.x >> 16);
    d.j0 = (int16_t)(u.y & 0xffff);
    d.j1 = (int16_t)(u.y >> 16);
    d.off = (int64_t)(((uint64_t)u.w << 32) | (uint64_t)u.z);
    return d;
}

// Wave-uniform 64-bit value (first active lane's).
__device__ inline int64_t uniform64(int64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v & 0xffffffffu));
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Descriptor load through the scalar cache: `idx` must be wave-uniform.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) u32x4* const_u32x4_ptr;
__device__ inline ChildDesc load_desc_scalar(const ChildDesc* base, int64_t idx) {
    u32x4 u = ((const_u32x4_ptr)base)[idx];
    ChildDesc d;
    d.i0 = (int16_t)(u.x & 0xffff);
    d.i1 = (int16_t)(u.x >> 16);
    d.j0 = (int16_t)(u.y & 0xffff);
    d.j1 = (int16_t)(u.y >> 16);
    d.off = (int64_t)(((uint64_t)u.w << 32) | (uint64_t)u.z);
    return d;
}

// Camera through the scalar cache: `idx` must be wave-uniform.
typedef const __attribute__((address_space(4))) uint64_t* const_u64_ptr;
__device__ inline Cam load_cam_scalar(const Cam* cams, int idx) {
    static_assert(sizeof(Cam) % 8 == 0, "Cam is copied as 64-bit words");
    Cam c;
    const_u64_ptr src = (const_u64_ptr)(cams + idx);
    uint64_t* dst = reinterpret_cast<uint64_t*>(&c);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(Cam) / 8); k++) dst[k] = src[k];
    return c;
}

// ---------------------------------------------------------------------------
// segment group (eq. aggregate): near (+) far
// ---------------------------------------------------------------------------

__device__ inline float2 seg_combine(float2 near2, float2 far1) {
    return make_float2(near2.x * far1.x, fmaf(near2.x, far1.y, near2.y));
}

// ---------------------------------------------------------------------------
// segment evaluation in FP32
// ---------------------------------------------------------------------------

// Geometry of one hit: reference coordinates at the far end, their change to
// the near end, and the real length dx (Sec. 2.3: x runs far -> near).
struct SegGeom {
    float xf[3];
    float dxi[3];
    float dx;
};

__device__ inline SegGeom seg_geom(const double rho[3], const double r[3], double s_in, double s_out,
                                   const double lo[3], int level) {
    SegGeom g;
    double scale = (double)(1u << level);
    for (int k = 0; k < 3; k++) {
        double pf = rho[k] + s_out * r[k];
        g.xf[k] = (float)((pf - lo[k]) * scale);
        g.dxi[k] = (float)((s_in - s_out) * r[k] * scale);
    }
    // the ray's length scale is needed to FP32 accuracy only: the hardware
    // square root (within 1 ulp; |r|^2 is far from the denormal range)
    float rn = __builtin_amdgcn_sqrtf((float)(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]));
    g.dx = (float)(s_out - s_in) * rn;
    return g;
}

// Trilinear interpolation, corner c = bx + 2 by + 4 bz.
__device__ inline float trilin(const float v[8], float x, float y, float z) {
    float c00 = fmaf(x, v[1] - v[0], v[0]);
    float c10 = fmaf(x, v[3] - v[2], v[2]);
    float c01 = fmaf(x, v[5] - v[4], v[4]);
    float c11 = fmaf(x, v[7] - v[6], v[6]);
    float c0 = fmaf(y, c10 - c00, c00);
    float c1 = fmaf(y, c11 - c01, c01);
    return fmaf(z, c1 - c0, c0);
}

// One classical RK4 step of eq. ODEsAB from (A, B) = (1, 0) over length h with
// the stage values of eq. RKresultAB; b0/g0 at the far end, bm/gm at the
// midpoint (stages 1 and 2), b1/g1 at the near end.
__device__ inline float2 rk4_step(float b0, float bm, float b1, float g0, float gm, float g1, float h) {
    float hh = 0.5f * h;
    float A1 = fmaf(-hh, b0, 1.0f);
    float A2 = fmaf(-hh * bm, A1, 1.0f);
    float A3 = fmaf(-h * bm, A2, 1.0f);
    float sa = fmaf(b1, A3, fmaf(2.0f * bm, A1 + A2, b0));
    float A = fmaf(-h * (1.0f / 6.0f), sa, 1.0f);
    float B1 = hh * g0;
    float f1 = fmaf(-bm, B1, gm);
    float B2 = hh * f1;
    float f2 = fmaf(-bm, B2, gm);
    float B3 = h * f2;
    float f3 = fmaf(-b1, B3, g1);
    float sb = fmaf(2.0f, f1 + f2, g0 + f3);
    float B = h * (1.0f / 6.0f) * sb;
    return make_float2(A, B);
}

// Restriction of a trilinear field to the segment: with reference
// coordinates xi(t) = a + d t (t = 0 far end, t = 1 near end) the
// interpolant is exactly the cubic p0 + p1 t + p2 t^2 + p3 t^3, built by
// interpolating along x, then y, then z on polynomial coefficients.
__device__ inline void field_cubic(const float v[8], const float a[3], const float d[3], float p[4]) {
    float e0[4], e1[4];  // linear in t per (y, z) corner pair m = y + 2 z
#pragma unroll
    for (int m = 0; m < 4; m++) {
        float dv = v[2 * m + 1] - v[2 * m];
        e0[m] = fmaf(a[0], dv, v[2 * m]);
        e1[m] = d[0] * dv;
    }
    float f[2][3];  // quadratic in t per z
#pragma unroll
    for (int z = 0; z < 2; z++) {
        float D0 = e0[2 * z + 1] - e0[2 * z], D1 = e1[2 * z + 1] - e1[2 * z];
        f[z][0] = fmaf(a[1], D0, e0[2 * z]);
        f[z][1] = fmaf(d[1], D0, fmaf(a[1], D1, e1[2 * z]));
        f[z][2] = d[1] * D1;
    }
    float G0 = f[1][0] - f[0][0], G1 = f[1][1] - f[0][1], G2 = f[1][2] - f[0][2];
    p[0] = fmaf(a[2], G0, f[0][0]);
    p[1] = fmaf(d[2], G0, fmaf(a[2], G1, f[0][1]));
    p[2] = fmaf(d[2], G1, fmaf(a[2], G2, f[0][2]));
    p[3] = d[2] * G2;
}

__device__ inline float horner3(const float p[4], float t) { return fmaf(t, fmaf(t, fmaf(t, p[3], p[2]), p[1]), p[0]); }

// RK4 over NSUB equal substeps (NSUB = 0: `nsub` at run time), farthest
// first, combined with (+).  Field values come from the cubic restriction.
template <int NSUB>
__device__ inline float2 seg_rk4(const float kc[8], const float ec[8], const SegGeom& g, int nsub) {
    const int ns = NSUB > 0 ? NSUB : nsub;
    float inv = 1.0f / (float)ns;
    float h = g.dx * inv;
    float pk[4], pe[4];
    field_cubic(kc, g.xf, g.dxi, pk);
    field_cubic(ec, g.xf, g.dxi, pe);
    float kf = pk[0], ef = pe[0];
    float2 acc = make_float2(1.0f, 0.0f);
    auto substep = [&](int q) {
        float tm = ((float)q + 0.5f) * inv, tn = (float)(q + 1) * inv;
        float km = horner3(pk, tm), em = horner3(pe, tm);
        float kn = horner3(pk, tn), en = horner3(pe, tn);
        float2 s = rk4_step(kf, km, kn, ef, em, en, h);
        acc = seg_combine(s, acc);
        kf = kn;
        ef = en;
    };
    if constexpr (NSUB > 0) {
#pragma unroll
        for (int q = 0; q < NSUB; q++) substep(q);
    } else {
        for (int q = 0; q < ns; q++) substep(q);
    }
    return acc;
}

// Constant-per-leaf coefficients through the same RK4 stages.
template <int NSUB>
__device__ inline float2 seg_rk4_const(float k, float e, float dx, int nsub) {
    const int ns = NSUB > 0 ? NSUB : nsub;
    float h = dx / (float)ns;
    float2 s = rk4_step(k, k, k, e, e, e, h);
    float2 acc = s;
    for (int q = 1; q < ns; q++) acc = seg_combine(s, acc);
    return acc;
}

// Constant coefficients (eq. ABconstant): A = e^{-k dx}, B = e dx (1 - A)/(k dx).
// Constant absorption k and equilibrium intensity I (eq. BIrelation):
// A = exp(-k dx), B = I (1 - A).
__device__ inline float2 seg_const_eq(float k, float I, float dx) {
    float x = k * dx;
    return make_float2(expf(-x), -I * expm1f(-x));
}

__device__ inline float2 seg_const(float k, float e, float dx) {
    float x = k * dx;
    float A = expf(-x);
    float phi = (fabsf(x) < 1e-4f) ? fmaf(x, fmaf(x, 1.0f / 6.0f, -0.5f), 1.0f) : -expm1f(-x) / x;
    return make_float2(A, e * dx * phi);
}

// ---------------------------------------------------------------------------
// searches and index arithmetic
// ---------------------------------------------------------------------------

// a / b for non-negative operands: 32-bit division whenever both fit.
__device__ inline int64_t divu(int64_t a, int64_t b) {
    if (a < b) return 0;
    if ((uint64_t)a <= 0xffffffffull && (uint64_t)b <= 0xffffffffull) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}

// Largest s in [lo, hi) with off[s] <= g, for nondecreasing off and off[lo] <= g.
__device__ inline int64_t upper_index(const int64_t* off, int64_t lo, int64_t hi, int64_t g) {
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// upper_index with seven independent probes per step: about log8 of the range
// in dependent load rounds instead of log2.
__device__ inline int64_t upper_index_wide(const int64_t* off, int64_t lo, int64_t hi, int64_t g) {
    while (hi - lo > 8) {
        int64_t step = (hi - lo) >> 3;
        int64_t v[7];
#pragma unroll
        for (int k = 0; k < 7; k++) v[k] = off[lo + (k + 1) * step];
        int c = 0;
#pragma unroll
        for (int k = 0; k < 7; k++) c += v[k] <= g ? 1 : 0;
        int64_t nlo = lo + c * step;
        if (c < 7) hi = nlo + step;
        lo = nlo;
    }
    return upper_index(off, lo, hi, g);
}

// Visible pair holding candidate g of wave chunk w: between the pairs of the
// chunk's first candidate and the next chunk's (at most 64 pairs apart).
__device__ inline int64_t cand_pair(const int64_t* cand_offset, const int32_t* cand_chunk, int64_t g, int64_t w,
                                    int64_t nvis, int64_t ncand) {
    int64_t lo = cand_chunk[w];
    int64_t hi = ((w + 1) * 64 < ncand) ? (int64_t)cand_chunk[w + 1] + 1 : nvis;
    return upper_index(cand_offset, lo, hi, g);
}

// Pairing of candidate g (Sec. 2.1, 2.2): its leaf, the pixel's ray and the
// hit interval.  Args provides the vforest and leaf arrays.
struct Pairing {
    int32_t leaf;
    int lv;
    bool hit;
    double lo[3], rho[3], rr[3], s_in, s_out;
};

template <int MODE, typename Args>
__device__ inline Pairing pair_with(const Args& a, int64_t g, int64_t v, const Cam& c) {
    Pairing p;
    p.leaf = a.vis_leaf[v];
    Rect r = load_rect(a.vis_rect + 4 * v);
    int k = (int)(g - a.cand_offset[v]);
    int i, j;
    rect_pixel(r, k, i, j);
    p.lv = a.level[p.leaf];
    double hi[3];
    node_box(p.lv, a.x[p.leaf], a.y[p.leaf], a.z[p.leaf], p.lo, hi);
    pixel_ray<MODE>(c, i, j, p.rho, p.rr);
    p.hit = slab_hit(c, p.rho, p.rr, p.lo, hi, p.s_in, p.s_out);
    return p;
}

// The camera comes through the scalar cache when the wave's candidates share
// it (all but the waves that straddle two images).
template <typename Args>
__device__ inline Pairing pair_candidate(const Args& a, int64_t g, int64_t w, int64_t nvis, int64_t ncand,
                                         int64_t* vout = nullptr) {
    int64_t v = cand_pair(a.cand_offset, a.cand_chunk, g, w, nvis, ncand);
    if (vout) *vout = v;
    int cam = a.vis_cam[v];
    int c0 = __builtin_amdgcn_readfirstlane(cam);
    if (__all(cam == c0)) {
        Cam cs = load_cam_scalar(a.cams, c0);
        if (cs.ortho) return pair_with<1>(a, g, v, cs);
        return pair_with<0>(a, g, v, cs);
    }
    return pair_with<-1>(a, g, v, a.cams[cam]);
}

// Camera of a pixel in the concatenated images.
__device__ inline int camera_of_pixel(const Cam* cams, int ncams, int64_t p) {
    int lo = 0, hi = ncams;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cams[mid].img_off <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan (reduce, scan of block sums, re-scan and apply);
// deterministic and independent of timing.  Each thread takes ITEMS
// consecutive items; ITEMS grows with n so the block count stays moderate.
// ---------------------------------------------------------------------------

constexpr int SCAN_NT = 256;
constexpr int SCAN_MAX_ITEMS = 16;

struct I64x2 {
    int64_t a, b;
    __device__ __host__ I64x2 operator+(const I64x2& o) const { return I64x2{a + o.a, b + o.b}; }
};

struct I64x3 {
    int64_t a, b, c;
    __device__ __host__ I64x3 operator+(const I64x3& o) const { return I64x3{a + o.a, b + o.b, c + o.c}; }
};

__device__ inline int64_t shfl_up_t(int64_t v, int d) { return __shfl_up(v, d); }
__device__ inline I64x2 shfl_up_t(I64x2 v, int d) { return I64x2{__shfl_up(v.a, d), __shfl_up(v.b, d)}; }
__device__ inline I64x3 shfl_up_t(I64x3 v, int d) {
    return I64x3{__shfl_up(v.a, d), __shfl_up(v.b, d), __shfl_up(v.c, d)};
}

// Exclusive scan over the block; `sh` holds NT/64 wave totals.
template <typename T, int NT>
__device__ inline T block_exclusive_scan(T v, T* sh, T& total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int d = 1; d < 64; d <<= 1) {
        T y = shfl_up_t(x, d);
        if (lane >= d) x = x + y;
    }
    T ex = shfl_up_t(x, 1);
    if (lane == 0) ex = T();
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    T wpre = T();
    total = T();
    for (int k = 0; k < NT / 64; k++) {
        T t = sh[k];
        if (k < wid) wpre = wpre + t;
        total = total + t;
    }
    __syncthreads();
    return wpre + ex;
}

// Src: __device__ Item operator()(int64_t i) with member `T val`.  Block b
// covers items [b * SCAN_NT * ITEMS, (b + 1) * SCAN_NT * ITEMS); in step k its
// threads take SCAN_NT consecutive items, so every load and store of a step is
// coalesced across the wave.
template <typename T, int ITEMS, typename Src>
__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(int64_t n, Src src, T* partial) {
    __shared__ T sh[SCAN_NT / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_NT * ITEMS + threadIdx.x;
    T acc = T();
    for (int k = 0; k < ITEMS; k++) {
        int64_t i = base + (int64_t)k * SCAN_NT;
        if (i < n) acc = acc + src(i).val;
    }
    T total;
    block_exclusive_scan<T, SCAN_NT>(acc, sh, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Single block: partial[0..nb) -> exclusive prefix, partial[nb] = total.
template <typename T>
__global__ __launch_bounds__(SCAN_NT) void k_scan_partials(int64_t nb, T* partial) {
    __shared__ T sh[SCAN_NT / 64];
    constexpr int PI = 4;
    T carry = T();
    for (int64_t base = 0; base < nb; base += SCAN_NT * PI) {
        int64_t i0 = base + (int64_t)threadIdx.x * PI;
        T v[PI];
        T acc = T();
        for (int k = 0; k < PI; k++) {
            v[k] = (i0 + k < nb) ? partial[i0 + k] : T();
            acc = acc + v[k];
        }
        T total;
        T run = carry + block_exclusive_scan<T, SCAN_NT>(acc, sh, total);
        for (int k = 0; k < PI; k++) {
            if (i0 + k < nb) partial[i0 + k] = run;
            run = run + v[k];
        }
        carry = carry + total;
    }
    if (threadIdx.x == 0) partial[nb] = carry;
}

// Dst: __device__ void operator()(int64_t i, T prefix, const Item& item) and
//      __device__ void total(T tot)  (called once, by the last block).
// Items as in k_scan_reduce; each step scans its SCAN_NT items across the
// block and carries the step's total into the next.
template <typename T, int ITEMS, typename Src, typename Dst>
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(int64_t n, int64_t nb, Src src, Dst dst, const T* partial) {
    typedef decltype(src(int64_t(0))) ItemT;
    __shared__ T sh[SCAN_NT / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_NT * ITEMS + threadIdx.x;
    T carry = partial[blockIdx.x];
    for (int k = 0; k < ITEMS; k++) {
        int64_t i = base + (int64_t)k * SCAN_NT;
        if (i - threadIdx.x >= n) break;  // the block's remaining steps are empty (uniform)
        bool in = i < n;
        ItemT item{};
        T v = T();
        if (in) {
            item = src(i);
            v = item.val;
        }
        T tot;
        T ex = block_exclusive_scan<T, SCAN_NT>(v, sh, tot);
        if (in) dst(i, carry + ex, item);
        carry = carry + tot;
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) dst.total(partial[nb]);
}

inline int scan_items(int64_t n) {
    if (n <= (int64_t)SCAN_NT * 1024) return 1;
    if (n <= (int64_t)SCAN_NT * 4 * 2048) return 4;
    return SCAN_MAX_ITEMS;
}

inline int64_t scan_blocks(int64_t n) {
    int64_t chunk = (int64_t)SCAN_NT * scan_items(n);
    int64_t nb = (n + chunk - 1) / chunk;
    return nb < 1 ? 1 : nb;
}

// Up to this many blocks each block of the apply pass sums the totals of the
// blocks before it itself (integer sums, exact in any order), and the
// partials pass is left out: one launch fewer for at most 48 KB of cached
// reads per block.
constexpr int64_t SCAN_FUSED_MAX_BLOCKS = 2048;

// k_scan_apply whose blocks take their carry from the reduce pass's block
// totals (partial[0 .. nb)) instead of an exclusive prefix of them; the last
// block hands the grand total to dst.total.
template <typename T, int ITEMS, typename Src, typename Dst>
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply_fused(int64_t n, int64_t nb, Src src, Dst dst,
                                                              const T* partial) {
    typedef decltype(src(int64_t(0))) ItemT;
    __shared__ T sh[SCAN_NT / 64];
    T acc = T();
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += SCAN_NT) acc = acc + partial[k];
    T carry;
    block_exclusive_scan<T, SCAN_NT>(acc, sh, carry);
    int64_t base = (int64_t)blockIdx.x * SCAN_NT * ITEMS + threadIdx.x;
    for (int k = 0; k < ITEMS; k++) {
        int64_t i = base + (int64_t)k * SCAN_NT;
        if (i - threadIdx.x >= n) break;  // the block's remaining steps are empty (uniform)
        bool in = i < n;
        ItemT item{};
        T v = T();
        if (in) {
            item = src(i);
            v = item.val;
        }
        T tot;
        T ex = block_exclusive_scan<T, SCAN_NT>(v, sh, tot);
        if (in) dst(i, carry + ex, item);
        carry = carry + tot;
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) dst.total(carry);
}

template <typename T, int ITEMS, typename Src, typename Dst>
inline void launch_scan_tail(int64_t n, int64_t nb, Src src, Dst dst, T* partial, hipStream_t st) {
    if (nb <= SCAN_FUSED_MAX_BLOCKS) {
        hipLaunchKernelGGL((k_scan_apply_fused<T, ITEMS, Src, Dst>), dim3((unsigned)nb), dim3(SCAN_NT), 0, st, n,
                           nb, src, dst, (const T*)partial);
        return;
    }
    hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(SCAN_NT), 0, st, nb, partial);
    hipLaunchKernelGGL((k_scan_apply<T, ITEMS, Src, Dst>), dim3((unsigned)nb), dim3(SCAN_NT), 0, st, n, nb, src,
                       dst, (const T*)partial);
}

template <typename T, int ITEMS, typename Src, typename Dst>
inline hipError_t launch_scan_n(int64_t n, int64_t nb, Src src, Dst dst, T* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_scan_reduce<T, ITEMS, Src>), dim3((unsigned)nb), dim3(SCAN_NT), 0, st, n, src, partial);
    launch_scan_tail<T, ITEMS>(n, nb, src, dst, partial, st);
    return hipGetLastError();
}

// As launch_scan_n, with separate item sources for the reduce and the apply
// passes (they must agree on every item's value).
template <typename T, int ITEMS, typename SrcR, typename SrcA, typename Dst>
inline hipError_t launch_scan2_n(int64_t n, int64_t nb, SrcR sr, SrcA sa, Dst dst, T* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_scan_reduce<T, ITEMS, SrcR>), dim3((unsigned)nb), dim3(SCAN_NT), 0, st, n, sr, partial);
    launch_scan_tail<T, ITEMS>(n, nb, sa, dst, partial, st);
    return hipGetLastError();
}

template <typename T, typename SrcR, typename SrcA, typename Dst>
inline hipError_t launch_scan2(int64_t n, SrcR sr, SrcA sa, Dst dst, T* partial, hipStream_t st) {
    int64_t nb = scan_blocks(n);
    switch (scan_items(n)) {
        case 1: return launch_scan2_n<T, 1>(n, nb, sr, sa, dst, partial, st);
        case 4: return launch_scan2_n<T, 4>(n, nb, sr, sa, dst, partial, st);
        default: return launch_scan2_n<T, SCAN_MAX_ITEMS>(n, nb, sr, sa, dst, partial, st);
    }
}

template <typename T, typename Src, typename Dst>
inline hipError_t launch_scan(int64_t n, Src src, Dst dst, T* partial, hipStream_t st) {
    int64_t nb = scan_blocks(n);
    switch (scan_items(n)) {
        case 1: return launch_scan_n<T, 1>(n, nb, src, dst, partial, st);
        case 4: return launch_scan_n<T, 4>(n, nb, src, dst, partial, st);
        default: return launch_scan_n<T, SCAN_MAX_ITEMS>(n, nb, src, dst, partial, st);
    }
}

inline size_t scan_partial_bytes(int64_t n, size_t elem) { return (size_t)(scan_blocks(n) + 1) * elem; }

// Grid for a grid-stride kernel over at most `n` items.
inline unsigned stride_grid(int64_t n, int nt, unsigned maxblocks = 256 * 16) {
    int64_t b = (n + nt - 1) / nt;
    if (b < 1) b = 1;
    if (b > (int64_t)maxblocks) b = maxblocks;
    return (unsigned)b;
}

}  // namespace rc
