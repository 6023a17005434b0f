// rc_surface_ho.hip -- ray segments of degree-R surface forests (Sec. 2.8,
// App. A.1).  A candidate (visible leaf, pixel) describes the pixel's ray by
// two planes through it; each plane's signed distance along the leaf is a
// Bernstein polynomial over the leaf square (rc_surface_ho.h).  The leaf square
// is searched depth first: sub-squares where either polynomial keeps one sign
// are dropped; on the others Krawczyk's test decides no root, one root
// (Newton's method from the centre) or undecided (split into four).  A
// converged root is polished canonically on the tree's own polynomials (snap
// to a 2^-40 grid, two Newton steps), so every leaf and sub-square that
// reaches it computes the same bits, and it counts in the one sub-square, of
// the one leaf, whose half-open extent holds it.
#include "rc_host.h"
#include "rc_surface_ho.h"

namespace rc {
namespace {

constexpr int HO_D0 = 0;   // subdivisions of the leaf square before the first test
constexpr int HO_D1 = 16;  // deepest subdivision below the leaf
// Squares visited per candidate at most: a ray lying in the surface leaves
// every square undecided, and the search stops there.
constexpr int HO_MAXVISIT = 2048;

struct HoArgs {
    const Cam* cams;
    const uint8_t* level;
    const uint32_t *x, *y;
    const float4 *As, *Is;
    HoGeom G;
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

struct HoHit {
    double s;
    float2 ab;
};

template <int R>
__device__ inline void ho_candidate(const HoArgs& a, int64_t g, int64_t vp, const Cam& c) {
    constexpr int N2 = (R + 1) * (R + 1);
    int32_t leaf = a.vis_leaf[vp];
    Rect rc = load_rect(a.vis_rect + 4 * vp);
    int k = (int)(g - a.cand_offset[vp]);
    int i, j;
    rect_pixel(rc, k, i, j);
    int tree = 0;
    while (tree + 1 < a.ntrees && leaf >= a.tb[tree + 1]) tree++;
    int lv = a.level[leaf];
    uint32_t lx = a.x[leaf], ly = a.y[leaf];
    const double inv = 1.0 / (double)(1u << QMAX);
    double len = (double)(1u << (QMAX - lv));
    double w1[3], w2[3], off1, off2, rcam[3];
    ho_pixel_planes(c, i, j, w1, off1, w2, off2, rcam);
    // the search covers the leaf's square padded by half a step of the 2^-40
    // grid that decides which leaf holds a root (tree units): a root that
    // rounds onto this leaf's edge from outside is this leaf's to find
    const double pad = 0x1p-41;
    const double a0 = (double)lx * inv - pad, a1 = ((double)lx + len) * inv + pad;
    const double b0 = (double)ly * inv - pad, b1 = ((double)ly + len) * inv + pad;
    double L1[N2], L2[N2];
    ho_net<R>(a.G, tree, c.o, w1, off1, L1);
    ho_net<R>(a.G, tree, c.o, w2, off2, L2);
    ho_restrict<R>(L1, a0, a1, b0, b1);
    ho_restrict<R>(L2, a0, a1, b0, b1);
    HoHit h0{0.0, make_float2(1.0f, 0.0f)}, h1 = h0;
    int cnt = 0;
    if (ho_may_vanish(L1) && ho_may_vanish(L2)) {
        float4 As = a.As[leaf], Is = a.Is[leaf];
        int d = 0;
        uint32_t i1 = 0, i2 = 0;
        for (int visit = 0; visit < HO_MAXVISIT; visit++) {
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
                int kr = d < HO_D0 ? 2 : ho_krawczyk<R>(L1, L2, S1, S2, u0, v0, hs);
                if (kr == 2 && d < HO_D1) {
                    descend = true;
                } else if (kr != 0) {
                    // one root in the (widened) square, or the deepest square: Newton from the centre
                    double u = u0 + 0.5 * hs, v = v0 + 0.5 * hs;
                    if (ho_newton_local<R>(L1, L2, u, v)) {
                        double t1 = a0 + u * (a1 - a0), t2 = b0 + v * (b1 - b0);
                        // canonical polish on the tree's polynomials
                        double T1[N2], T2[N2];
                        ho_net<R>(a.G, tree, c.o, w1, off1, T1);
                        ho_net<R>(a.G, tree, c.o, w2, off2, T2);
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
                        // the leaf and the square holding the root are decided on the
                        // root rounded to the same grid, which holds every leaf edge
                        double q1 = rint(t1 * gq) / gq, q2 = rint(t2 * gq) / gq;
                        double lu, lv2;
                        if (ok && q1 >= 0.0 && q1 <= 1.0 && q2 >= 0.0 && q2 <= 1.0 &&
                            surf_leaf_has(lv, lx, ly, q1, q2, lu, lv2)) {
                            // a root in a neighbouring square is that square's to count
                            int n = 1 << d;
                            double w1c = (q1 - a0) / (a1 - a0), w2c = (q2 - b0) / (b1 - b0);
                            int c1 = (int)fmin(w1c * n, (double)(n - 1)), c2 = (int)fmin(w2c * n, (double)(n - 1));
                            if (c1 == (int)i1 && c2 == (int)i2) {
                                // depth along the ray and the patch normal, in camera space
                                double jt1[3], jt2[3], pz = 0.0;
                                const double* axes[3] = {c.t, c.u, c.vh};
#pragma unroll
                                for (int m = 0; m < 3; m++) {
                                    double P[N2], pv0, p1, p2;
                                    ho_net<R>(a.G, tree, c.o, axes[m], 0.0, P);
                                    ho_eval<R>(P, t1, t2, pv0, p1, p2);
                                    jt1[m] = p1;
                                    jt2[m] = p2;
                                    if (m == 2) pz = pv0;
                                }
                                double s = c.ortho ? pz : pz / c.n;
                                if (s >= c.smin && s <= c.smax) {
                                    float2 ab = surf_model(As, Is, surf_cos(jt1, jt2, rcam), lu, lv2);
                                    HoHit hh{s, ab};
                                    if (cnt == 0) {
                                        h0 = hh;
                                    } else if (cnt == 1) {
                                        if (s < h0.s) {
                                            h1 = h0;
                                            h0 = hh;
                                        } else {
                                            h1 = hh;
                                        }
                                    } else if (s < h1.s) {
                                        if (s < h0.s) {
                                            h1 = h0;
                                            h0 = hh;
                                        } else {
                                            h1 = hh;
                                        }
                                    }
                                    cnt++;
                                }
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
    float4 o0 = make_float4(1.0f, 0.0f, 1.0f, 0.0f), o1 = o0;
    if (cnt >= 1) o0 = make_float4((float)h0.s, (float)h0.s, h0.ab.x, h0.ab.y);
    if (cnt >= 2) o1 = make_float4((float)h1.s, (float)h1.s, h1.ab.x, h1.ab.y);
    a.rec[2 * g] = o0;
    a.rec[2 * g + 1] = o1;
    if (a.hit) a.hit[g] = (uint8_t)(cnt < 255 ? cnt : 255);
    if (a.sio) {
        double s0 = cnt >= 1 ? h0.s : 0.0, s1 = cnt >= 2 ? h1.s : 0.0;
        a.sio[4 * g] = s0;
        a.sio[4 * g + 1] = s0;
        a.sio[4 * g + 2] = s1;
        a.sio[4 * g + 3] = s1;
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_segments_surface_ho(HoArgs a) {
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
            ho_candidate<R>(a, g, v, cs);
        } else {
            ho_candidate<R>(a, g, v, a.cams[cam]);
        }
    }
}

}  // namespace

// Bernstein coefficients from values at the Gauss-Lobatto nodes: the inverse of
// E[m][k] = B_k(eta_m) (Gauss-Jordan elimination with partial pivoting).
void ho_geom_init(int R, const double* pts, HoGeom& G) {
    int n = R + 1;
    double eta[HO_MAXR + 1];
    eta[0] = 0.0;
    eta[R] = 1.0;
    if (R == 2) eta[1] = 0.5;
    if (R == 3) {
        eta[1] = 0.5 * (1.0 - 1.0 / sqrt(5.0));
        eta[2] = 0.5 * (1.0 + 1.0 / sqrt(5.0));
    }
    double m[HO_MAXR + 1][2 * (HO_MAXR + 1)];
    for (int r = 0; r < n; r++)
        for (int k = 0; k < n; k++) {
            double binom = 1.0;
            for (int q = 1; q <= k; q++) binom = binom * (R - k + q) / q;
            m[r][k] = binom * pow(eta[r], k) * pow(1.0 - eta[r], R - k);
            m[r][n + k] = r == k ? 1.0 : 0.0;
        }
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
        for (int k = 0; k < 2 * n; k++) {
            double t = m[col][k];
            m[col][k] = m[piv][k];
            m[piv][k] = t;
        }
        double dv = m[col][col];
        for (int k = 0; k < 2 * n; k++) m[col][k] /= dv;
        for (int r = 0; r < n; r++)
            if (r != col) {
                double f = m[r][col];
                for (int k = 0; k < 2 * n; k++) m[r][k] -= f * m[col][k];
            }
    }
    // values = E coefficients, so coefficients = E^-1 values: nb[k][m] = E^-1[k][m]
    for (int k = 0; k < (HO_MAXR + 1) * (HO_MAXR + 1); k++) G.nb[k] = 0.0;
    for (int k = 0; k < n; k++)
        for (int q = 0; q < n; q++) G.nb[k * n + q] = m[k][n + q];
    G.pts = pts;
}

}  // namespace rc

using namespace rc;

rc_status rc::rc_surface_ho_segments(const rc_forest* f, const rc_fields* fl, const void* dcams, const rc_vforest* vf,
                                     const rc_integrator* in, float* rec_leaf, uint8_t* hit, double* sio,
                                     const rc_tuning* tune, hipStream_t st) {
    if (fl->kind != RC_FIELD_SURFACE || in->method != RC_INT_ANALYTIC) return RC_EUNSUPPORTED;
    int R = surface_degree(f);
    HoArgs a;
    a.cams = (const Cam*)dcams;
    a.level = f->level;
    a.x = f->x;
    a.y = f->y;
    a.As = (const float4*)fl->kappa;
    a.Is = (const float4*)fl->eps;
    ho_geom_init(R, f->geom_table, a.G);
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
    dim3 G(stride_grid(vf->cap_cand, 256, tuned(tune, 0, 1024))), B(256);
    if (R == 2)
        hipLaunchKernelGGL(k_segments_surface_ho<2>, G, B, 0, st, a);
    else
        hipLaunchKernelGGL(k_segments_surface_ho<3>, G, B, 0, st, a);
    RC_HIP(hipGetLastError());
    return RC_OK;
}
