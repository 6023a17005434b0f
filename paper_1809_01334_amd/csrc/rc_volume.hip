// rc_volume.hip -- ray segments of degree-R volume forests (Sec. 2.1 curved
// elements, App. A.1).  A candidate (visible leaf, pixel) crosses the leaf's
// six faces where the two planes through the pixel's ray meet the face patch:
// each face is searched as a degree-R surface (Bernstein exclusion, Krawczyk's
// test, Newton's method, a canonical polish on the tree's face polynomial, so
// that the leaves sharing a face find the same crossing).  The crossings cut
// the clip range into pieces; a piece belongs to the leaf when its midpoint
// maps back into the leaf's cube (Newton's method on the tree map, FP64), and
// adjacent pieces inside join into one interval.  Each interval is integrated
// with RK4 over equal substeps, its field points mapped back to leaf reference
// coordinates the same way, or in closed form for constant coefficients.  A
// candidate keeps its two nearest intervals, in the shell's record layout.
#include "rc_host.h"
#include "rc_volume.h"

namespace rc {
namespace {

constexpr int VOL_D1 = 16;          // deepest subdivision of a face below the leaf
constexpr int VOL_MAXVISIT = 1024;  // sub-squares visited per face at most
constexpr int VOL_MAXCROSS = 16;    // crossings kept per candidate

struct VolArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y, *z;
    const float *kappa, *eps;
    int kind;  // RC_FIELD_CONST or RC_FIELD_TRILINEAR
    VolGeom V;
    int64_t tb[7];
    int ntrees;
    const int32_t* vis_leaf;
    const int16_t* vis_cam;
    const int16_t* vis_rect;
    const int64_t* cand_offset;
    const int64_t* counts;
    const int32_t* cand_chunk;
    int64_t cap_cand;
    float4* rec;
    uint8_t* hit;
    double* sio;
};

// Crossings of the ray with face f of the leaf (axis k = f / 2 at the leaf's
// low or high end), appended to cr[] (depth along the ray, clipped).
template <int R>
__device__ inline void face_crossings(const VolArgs& a, const Cam& c, int tree, const double lo[3], double len,
                                      int f, const double w1[3], double off1, const double w2[3], double off2,
                                      double (&cr)[VOL_MAXCROSS], int& nc) {
    constexpr int N = R + 1, N2 = N * N;
    int k = f / 2, ax = (k + 1) % 3, bx = (k + 2) % 3;
    double P[3 * N2];
    vol_face_points<R>(a.V, tree, k, lo[k] + ((f & 1) ? len : 0.0), P);
    double T1[N2], T2[N2];  // over the tree's face square: the canonical polynomials
    vol_face_net<R>(a.V, P, c.o, w1, off1, T1);
    vol_face_net<R>(a.V, P, c.o, w2, off2, T2);
    double L1[N2], L2[N2];  // over the leaf's face
#pragma unroll
    for (int q = 0; q < N2; q++) {
        L1[q] = T1[q];
        L2[q] = T2[q];
    }
    double a1 = lo[ax], a2 = lo[bx];
    ho_restrict<R>(L1, a1, a1 + len, a2, a2 + len);
    ho_restrict<R>(L2, a1, a1 + len, a2, a2 + len);
    if (!(ho_may_vanish(L1) && ho_may_vanish(L2))) return;
    int d = 0;
    uint32_t i1 = 0, i2 = 0;
    for (int visit = 0; visit < VOL_MAXVISIT; visit++) {
        bool descend = false;
        double hs = ldexp(1.0, -d), u0 = (double)i1 * hs, v0 = (double)i2 * hs;
        double S1[N2], S2[N2];
#pragma unroll
        for (int q = 0; q < N2; q++) {
            S1[q] = L1[q];
            S2[q] = L2[q];
        }
        if (d > 0) {
            ho_restrict<R>(S1, u0, u0 + hs, v0, v0 + hs);
            ho_restrict<R>(S2, u0, u0 + hs, v0, v0 + hs);
        }
        if (ho_may_vanish(S1) && ho_may_vanish(S2)) {
            int kr = ho_krawczyk<R>(L1, L2, S1, S2, u0, v0, hs);
            if (kr == 2 && d < VOL_D1) {
                descend = true;
            } else if (kr != 0) {
                double u = u0 + 0.5 * hs, v = v0 + 0.5 * hs;
                if (ho_newton_local<R>(L1, L2, u, v)) {
                    // canonical polish in the tree's face coordinates
                    double t1 = a1 + u * len, t2 = a2 + v * len;
                    const double gq = 1099511627776.0;  // 2^40
                    t1 = rint(t1 * gq) / gq;
                    t2 = rint(t2 * gq) / gq;
                    bool ok = true;
#pragma unroll 1
                    for (int it = 0; it < 2 && ok; it++) {
                        double p, pu, pv, q, qu, qv;
                        ho_eval<R>(T1, t1, t2, p, pu, pv);
                        ho_eval<R>(T2, t1, t2, q, qu, qv);
                        double det = pu * qv - pv * qu;
                        ok = det != 0.0;
                        if (ok) {
                            t1 -= (qv * p - pv * q) / det;
                            t2 -= (pu * q - qu * p) / det;
                        }
                    }
                    double lu = (t1 - a1) / len, lv = (t2 - a2) / len;
                    // a crossing on the leaf's closed face, counted in the one sub-square holding it
                    if (ok && lu >= 0.0 && lu <= 1.0 && lv >= 0.0 && lv <= 1.0) {
                        int n = 1 << d;
                        int c1 = (int)fmin(lu * n, (double)(n - 1)), c2 = (int)fmin(lv * n, (double)(n - 1));
                        if (c1 == (int)i1 && c2 == (int)i2) {
                            double Z[N2], zv, zu_, zv_;
                            vol_face_net<R>(a.V, P, c.o, c.vh, 0.0, Z);
                            ho_eval<R>(Z, t1, t2, zv, zu_, zv_);
                            double s = c.ortho ? zv : zv / c.n;
                            if (s > c.smin && s < c.smax && nc < VOL_MAXCROSS) cr[nc++] = s;
                        }
                    }
                }
            }
        }
        if (descend) {
            d++;
            i1 *= 2;
            i2 *= 2;
            continue;
        }
        while (d > 0 && (i1 & 1u) && (i2 & 1u)) {
            i1 >>= 1;
            i2 >>= 1;
            d--;
        }
        if (d == 0) break;
        if (!(i1 & 1u)) {
            i1 |= 1u;
        } else {
            i1 &= ~1u;
            i2 |= 1u;
        }
    }
}

// Is the point of the ray at s inside the leaf: its reference coordinates (Newton from the leaf's centre)
// lie in the leaf's closed cube.
template <int R>
__device__ inline bool vol_inside(const VolArgs& a, int tree, const double lo[3], double len, const double rho[3],
                                  const double r[3], double s) {
    double x[3] = {rho[0] + s * r[0], rho[1] + s * r[1], rho[2] + s * r[2]};
    double xi[3] = {lo[0] + 0.5 * len, lo[1] + 0.5 * len, lo[2] + 0.5 * len};
    if (!vol_invert<R>(a.V, tree, x, xi)) return false;
    return xi[0] >= lo[0] && xi[0] <= lo[0] + len && xi[1] >= lo[1] && xi[1] <= lo[1] + len && xi[2] >= lo[2] &&
           xi[2] <= lo[2] + len;
}

// RK4 over NSUB substeps of [s_in, s_out], far end first, the field points'
// leaf coordinates from Newton's method (warm-started along the ray); NSUB =
// 0: constant coefficients in closed form.
template <int R, int NSUB>
__device__ inline float2 vol_integrate(const VolArgs& a, int64_t leaf, int tree, const double lo[3], double len,
                                       const double rho[3], const double r[3], double s_in, double s_out) {
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if constexpr (NSUB == 0) {
        return seg_const(a.kappa[leaf], a.eps[leaf], (float)((s_out - s_in) * rn));
    } else {
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
        double ds = s_out - s_in;
        double xi[3] = {lo[0] + 0.5 * len, lo[1] + 0.5 * len, lo[2] + 0.5 * len};
        // field values at the point p / (2 NSUB) of the way from the far end
        auto field_at = [&](int p, float& bv, float& gv) {
            double s = s_out - ds * ((double)p / (double)(2 * NSUB));
            double pt[3] = {rho[0] + s * r[0], rho[1] + s * r[1], rho[2] + s * r[2]};
            vol_invert<R>(a.V, tree, pt, xi);
            float u0 = (float)((xi[0] - lo[0]) / len), u1 = (float)((xi[1] - lo[1]) / len);
            float u2 = (float)((xi[2] - lo[2]) / len);
            bv = trilin(kc, u0, u1, u2);
            gv = trilin(ec, u0, u1, u2);
        };
        float hstep = (float)(ds * rn) / (float)NSUB;
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
}

template <int R, int NSUB>
__device__ inline void vol_candidate(const VolArgs& a, int64_t g, int64_t vp, const Cam& c) {
    int32_t leaf = a.vis_leaf[vp];
    Rect rc = load_rect(a.vis_rect + 4 * vp);
    int k = (int)(g - a.cand_offset[vp]);
    int i, j;
    rect_pixel(rc, k, i, j);
    int tree = 0;
    while (tree + 1 < a.ntrees && leaf >= a.tb[tree + 1]) tree++;
    const double q = 1.0 / (double)(1u << QMAX);
    double len = ldexp(1.0, -(int)a.level[leaf]);
    double lo[3] = {(double)a.x[leaf] * q, (double)a.y[leaf] * q, (double)a.z[leaf] * q};
    double w1[3], w2[3], off1, off2, rcam[3];
    ho_pixel_planes(c, i, j, w1, off1, w2, off2, rcam);
    double cr[VOL_MAXCROSS];
    int nc = 0;
#pragma unroll 1
    for (int f = 0; f < 6; f++) face_crossings<R>(a, c, tree, lo, len, f, w1, off1, w2, off2, cr, nc);
    // the clip range cut at the crossings, nearest first
    double ev[VOL_MAXCROSS + 2];
    ev[0] = c.smin;
    int ne = 1;
    for (int e = 0; e < nc; e++) {
        int b = ne++;
        for (; b > 0 && ev[b - 1] > cr[e]; b--) ev[b] = ev[b - 1];
        ev[b] = cr[e];
    }
    ev[ne++] = c.smax;
    double rho[3], r[3];
    pixel_ray(c, i, j, rho, r);
    double iv[4] = {0.0, 0.0, 0.0, 0.0};
    int ni = 0;
    bool open = false;
    double cin = 0.0, cout = 0.0;
    for (int e = 0; e + 1 < ne; e++) {
        double s0 = ev[e], s1 = ev[e + 1];
        if (!(s1 > s0)) continue;
        bool in = vol_inside<R>(a, tree, lo, len, rho, r, 0.5 * (s0 + s1));
        if (in && open && s0 == cout) {
            cout = s1;
        } else if (in) {
            if (open) {
                if (ni < 2) {
                    iv[2 * ni] = cin;
                    iv[2 * ni + 1] = cout;
                }
                ni++;
            }
            open = true;
            cin = s0;
            cout = s1;
        }
    }
    if (open) {
        if (ni < 2) {
            iv[2 * ni] = cin;
            iv[2 * ni + 1] = cout;
        }
        ni++;
    }
    float4 o[2] = {make_float4(1.0f, 0.0f, 1.0f, 0.0f), make_float4(1.0f, 0.0f, 1.0f, 0.0f)};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if (h < ni) {
            float2 ab = vol_integrate<R, NSUB>(a, leaf, tree, lo, len, rho, r, iv[2 * h], iv[2 * h + 1]);
            o[h] = make_float4((float)iv[2 * h], (float)iv[2 * h + 1], ab.x, ab.y);
        }
    }
    a.rec[2 * g] = o[0];
    a.rec[2 * g + 1] = o[1];
    if (a.hit) a.hit[g] = (uint8_t)(ni < 255 ? ni : 255);
    if (a.sio) {
#pragma unroll
        for (int h = 0; h < 4; h++) a.sio[4 * g + h] = iv[h];
    }
}

template <int R, int NSUB>
__global__ __launch_bounds__(256) void k_segments_volume(VolArgs a) {
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
        vol_candidate<R, NSUB>(a, g, v, a.cams[a.vis_cam[v]]);
    }
}

template <int R>
rc_status launch_volume(const VolArgs& a, int nsub, dim3 G, hipStream_t st) {
    switch (nsub) {
        case 0: hipLaunchKernelGGL((k_segments_volume<R, 0>), G, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_segments_volume<R, 1>), G, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_segments_volume<R, 2>), G, dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_segments_volume<R, 4>), G, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_segments_volume<R, 8>), G, dim3(256), 0, st, a); break;
        default: return RC_EUNSUPPORTED;
    }
    RC_HIP(hipGetLastError());
    return RC_OK;
}

}  // namespace

void vol_geom_init(int R, const double* pts, VolGeom& V) {
    ho_geom_init(R, nullptr, V.H);
    for (int m = 0; m <= HO_MAXR; m++) V.eta[m] = 0.0;
    V.eta[0] = 0.0;
    V.eta[R] = 1.0;
    if (R == 2) V.eta[1] = 0.5;
    if (R == 3) {
        V.eta[1] = 0.5 * (1.0 - 1.0 / sqrt(5.0));
        V.eta[2] = 0.5 * (1.0 + 1.0 / sqrt(5.0));
    }
    V.pts = pts;
}

}  // namespace rc

using namespace rc;

rc_status rc::rc_volume_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                 const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                                 const rc_tuning* tune, hipStream_t st) {
    if (fl->kind != RC_FIELD_CONST && fl->kind != RC_FIELD_TRILINEAR) return RC_EUNSUPPORTED;
    int nsub;
    if (in->method == RC_INT_ANALYTIC) {
        if (fl->kind != RC_FIELD_CONST) return RC_EUNSUPPORTED;
        nsub = 0;
    } else if (in->method == RC_INT_RK4 && in->c_rk == 0.0) {
        nsub = in->substeps;
        if (nsub != 1 && nsub != 2 && nsub != 4 && nsub != 8) return RC_EUNSUPPORTED;
    } else {
        return RC_EUNSUPPORTED;
    }
    int R = volume_degree(f);
    VolArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.z = f->z;
    a.kappa = fl->kappa;
    a.eps = fl->eps;
    a.kind = fl->kind;
    vol_geom_init(R, f->geom_table, a.V);
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
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 2048)));
    return R == 2 ? launch_volume<2>(a, nsub, G, st) : launch_volume<3>(a, nsub, G, st);
}
