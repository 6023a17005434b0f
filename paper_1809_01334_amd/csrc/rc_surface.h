// rc_surface.h -- surfaces: quadtree leaves on bilinear tree patches.
//
// A tree's patch J(t1, t2) = a + b t1 + c t2 + d t1 t2 (from its corners P00,
// P10, P01, P11) meets a ray in at most two points.  The ray is intersected
// with the whole tree patch and every hit is given to the leaf whose
// half-open parameter square holds it, which is decided exactly on the
// dyadic grid: a ray through an edge shared by leaves is counted once.  All
// predicate arithmetic is FP64 in one fixed operation order with contraction
// off, so the hits are reproducible bit for bit.
#pragma once

#include "rc_internal.h"

namespace rc {

struct SurfPatch {
    double a[3], b[3], c[3], d[3];
};

__device__ inline SurfPatch surf_patch(const double* P) {
#pragma clang fp contract(off)
    SurfPatch S;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        S.a[k] = P[k];
        S.b[k] = P[3 + k] - P[k];
        S.c[k] = P[6 + k] - P[k];
        S.d[k] = (P[9 + k] - P[3 + k]) - (P[6 + k] - P[k]);
    }
    return S;
}

__device__ inline double sdot(const double u[3], const double w[3]) {
#pragma clang fp contract(off)
    return (u[0] * w[0] + u[1] * w[1]) + u[2] * w[2];
}

__device__ inline void scross(const double u[3], const double w[3], double o[3]) {
#pragma clang fp contract(off)
    o[0] = u[1] * w[2] - u[2] * w[1];
    o[1] = u[2] * w[0] - u[0] * w[2];
    o[2] = u[0] * w[1] - u[1] * w[0];
}

// Hits (s, t1, t2) of the ray rho + s r with the patch, (t1, t2) in [0, 1]^2
// and s in [smin, smax], nearest first.  App. A.1: d1 = r x e_k (k the axis of
// smallest |r_k|) and d2 = r x d1 are normal to r; the projections
// (A_j t2 + B_j) t1 + (C_j t2 + D_j) = 0, j = 1, 2, have a common t1 where
// their determinant, a quadratic in t2, vanishes (a double root counts once);
// t1 comes from the projection with the larger coefficient of t1.
__device__ inline int surf_hits(const Cam& cm, const SurfPatch& S, const double rho[3], const double r[3],
                                double hs[2], double h1[2], double h2[2]) {
#pragma clang fp contract(off)
    int k = 0;
    if (fabs(r[1]) < fabs(r[k])) k = 1;
    if (fabs(r[2]) < fabs(r[k])) k = 2;
    double ek[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
    double d1[3], d2[3], e[3];
    scross(r, ek, d1);
    scross(r, d1, d2);
#pragma unroll
    for (int q = 0; q < 3; q++) e[q] = S.a[q] - rho[q];
    double A1 = sdot(d1, S.d), B1 = sdot(d1, S.b), C1 = sdot(d1, S.c), D1 = sdot(d1, e);
    double A2 = sdot(d2, S.d), B2 = sdot(d2, S.b), C2 = sdot(d2, S.c), D2 = sdot(d2, e);
    double qa = A1 * C2 - A2 * C1;
    double qb = (A1 * D2 - A2 * D1) + (B1 * C2 - B2 * C1);
    double qc = B1 * D2 - B2 * D1;
    double root0 = 0.0, root1 = 0.0;
    int nr = 0;
    if (qa == 0.0) {
        if (qb != 0.0) {
            root0 = -qc / qb;
            nr = 1;
        }
    } else {
        double disc = qb * qb - (4.0 * qa) * qc;
        if (disc == 0.0) {
            root0 = -qb / (2.0 * qa);
            nr = 1;
        } else if (disc > 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
            root0 = q / qa;
            root1 = qc / q;
            nr = 2;
        }
    }
    double rr = sdot(r, r);
    int nh = 0;
#pragma unroll
    for (int m = 0; m < 2; m++) {
        if (m >= nr) break;
        double t2 = m == 0 ? root0 : root1;
        double den1 = A1 * t2 + B1, den2 = A2 * t2 + B2, t1;
        if (fabs(den1) >= fabs(den2)) {
            if (den1 == 0.0) continue;
            t1 = -(C1 * t2 + D1) / den1;
        } else {
            t1 = -(C2 * t2 + D2) / den2;
        }
        if (!(t1 >= 0.0 && t1 <= 1.0 && t2 >= 0.0 && t2 <= 1.0)) continue;
        double pr[3];
#pragma unroll
        for (int q = 0; q < 3; q++) pr[q] = (((S.a[q] + S.b[q] * t1) + S.c[q] * t2) + S.d[q] * (t1 * t2)) - rho[q];
        double s = sdot(pr, r) / rr;
        if (!(s >= cm.smin && s <= cm.smax)) continue;
        if (nh == 0) {
            hs[0] = s;
            h1[0] = t1;
            h2[0] = t2;
        } else {
            hs[1] = s;
            h1[1] = t1;
            h2[1] = t2;
        }
        nh++;
    }
    if (nh == 2 && hs[1] < hs[0]) {
        double t;
        t = hs[0]; hs[0] = hs[1]; hs[1] = t;
        t = h1[0]; h1[0] = h1[1]; h1[1] = t;
        t = h2[0]; h2[0] = h2[1]; h2[1] = t;
    }
    return nh;
}

// Local coordinates (u, v) of parameter (t1, t2) in a leaf, if the leaf's
// half-open square on the finest grid holds it (the tree's far edges closed).
__device__ inline bool surf_leaf_has(int level, uint32_t x, uint32_t y, double t1, double t2, double& u, double& v) {
#pragma clang fp contract(off)
    const double S = (double)(1u << QMAX);
    double X = t1 * S, Y = t2 * S;
    double len = (double)(1u << (QMAX - level));
    double x0 = (double)x, y0 = (double)y;
    bool in1 = (X >= x0 && X < x0 + len) || (X == S && x0 + len == S);
    bool in2 = (Y >= y0 && Y < y0 + len) || (Y == S && y0 + len == S);
    u = (X - x0) / len;
    v = (Y - y0) / len;
    return in1 && in2;
}

// Pixel rectangle of a leaf: the box of its patch corners (the patch is their
// convex combination, App. A.2), widened by a relative 1e-9 for the rounding
// of the corner positions.
__device__ inline Rect surf_rect(const Cam& c, const double* P, int level, uint32_t x, uint32_t y) {
    SurfPatch S = surf_patch(P);
    const double inv = 1.0 / (double)(1u << QMAX);
    double len = (double)(1u << (QMAX - level));
    double ta[2] = {(double)x * inv, ((double)x + len) * inv};
    double tb[2] = {(double)y * inv, ((double)y + len) * inv};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double mag = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        double t1 = ta[q & 1], t2 = tb[q >> 1];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            double p = ((S.a[k] + S.b[k] * t1) + S.c[k] * t2) + S.d[k] * (t1 * t2);
            lo[k] = fmin(lo[k], p);
            hi[k] = fmax(hi[k], p);
            mag = fmax(mag, fabs(p));
        }
    }
    double m = 1e-9 * (1.0 + mag);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        lo[k] -= m;
        hi[k] += m;
    }
    return box_rect(c, lo, hi);
}

// Surface model at a hit (Sec. 2.8, eq. ABphi with eq. BIrelation): the leaf's
// corner transparency and intensity interpolated bilinearly at (u, v),
// A = A_s^(1/cos phi) with cos phi = |n . r| / (|n| |r|) for the patch normal
// n = dJ/dt1 x dJ/dt2 at the hit, B = I_s (1 - A).
__device__ inline float2 surf_model(const float4& As, const float4& Is, float cphi, double u, double v) {
    float uf = (float)u, vf = (float)v;
    float w0 = (1.0f - uf) * (1.0f - vf), w1 = uf * (1.0f - vf), w2 = (1.0f - uf) * vf, w3 = uf * vf;
    float as = w0 * As.x + w1 * As.y + w2 * As.z + w3 * As.w;
    float is = w0 * Is.x + w1 * Is.y + w2 * Is.z + w3 * Is.w;
    float A = as >= 1.0f ? 1.0f : exp2f(log2f(as) / cphi);
    return make_float2(A, is * (1.0f - A));
}

// cos phi between the ray r and the normal j1 x j2 of tangents j1, j2.
__device__ inline float surf_cos(const double j1[3], const double j2[3], const double r[3]) {
    double n[3];
    scross(j1, j2, n);
    return (float)(fabs(sdot(n, r)) / sqrt(sdot(n, n) * sdot(r, r)));
}

__device__ inline float2 surf_value(const float4& As, const float4& Is, const SurfPatch& S, const double r[3],
                                    double t1, double t2, double u, double v) {
    double j1[3], j2[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        j1[q] = S.b[q] + S.d[q] * t2;
        j2[q] = S.c[q] + S.d[q] * t1;
    }
    return surf_model(As, Is, surf_cos(j1, j2, r), u, v);
}

}  // namespace rc
