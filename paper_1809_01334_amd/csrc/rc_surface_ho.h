// rc_surface_ho.h -- degree-R surfaces: each tree maps its parameter square by
// a tensor product of degree-R Lagrange polynomials on Gauss-Lobatto nodes
// (eq. nodal, eq. tensorgeom).  The device works in Bernstein form: a
// camera-space coordinate, or any affine functional w . (p - o) + off of the
// surface point, is a tensor Bernstein polynomial whose coefficients follow
// from the functional's values at the control points (eq. camerapoints: the
// control points carry the camera transform), and its coefficients over a
// sub-square bound it there (convex hull property).
#pragma once

#include "rc_surface.h"

namespace rc {

constexpr int HO_MAXR = 3;

struct HoGeom {
    double nb[(HO_MAXR + 1) * (HO_MAXR + 1)];  // Bernstein coefficient k = sum_m nb[k (R+1) + m] * value at node m
    const double* pts;                         // (R+1)^2 control points (3 doubles) per tree, m1 fastest
};

// Host: the node-to-Bernstein matrix of degree R (2 or 3) and the control
// points (rc_surface_ho.hip).
void ho_geom_init(int R, const double* pts, HoGeom& G);

// Coefficients over the tree square of L(p) = w . (p - o) + off on tree `tree`.
template <int R>
__device__ inline void ho_net(const HoGeom& G, int tree, const double o[3], const double w[3], double off,
                              double (&c)[(R + 1) * (R + 1)]) {
    constexpr int N = R + 1;
    const double* z = G.pts + 3 * N * N * tree;
    double v[N * N], tmp[N * N];
#pragma unroll
    for (int q = 0; q < N * N; q++)
        v[q] = ((w[0] * (z[3 * q] - o[0]) + w[1] * (z[3 * q + 1] - o[1])) + w[2] * (z[3 * q + 2] - o[2])) + off;
#pragma unroll
    for (int m2 = 0; m2 < N; m2++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < N; m++) s += G.nb[k * N + m] * v[m + N * m2];
            tmp[k + N * m2] = s;
        }
#pragma unroll
    for (int k1 = 0; k1 < N; k1++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < N; m++) s += G.nb[k * N + m] * tmp[k1 + N * m];
            c[k1 + N * k] = s;
        }
}

// Restriction of a degree-R polynomial (Bernstein coefficients c over [0, 1],
// stride S apart) to [a, b]: coefficient k is the blossom at (a^(R-k), b^k).
template <int R, int S>
__device__ inline void ho_restrict1(double* c, double a, double b) {
    double out[R + 1];
#pragma unroll
    for (int k = 0; k <= R; k++) {
        double t[R + 1];
#pragma unroll
        for (int i = 0; i <= R; i++) t[i] = c[i * S];
#pragma unroll
        for (int lev = 1; lev <= R; lev++) {
            double p = lev <= k ? b : a;
#pragma unroll
            for (int i = 0; i + lev <= R; i++) t[i] = t[i] + p * (t[i + 1] - t[i]);
        }
        out[k] = t[0];
    }
#pragma unroll
    for (int i = 0; i <= R; i++) c[i * S] = out[i];
}

// Coefficients over [a1, b1] x [a2, b2] of the net c (index k1 + (R+1) k2).
template <int R>
__device__ inline void ho_restrict(double (&c)[(R + 1) * (R + 1)], double a1, double b1, double a2, double b2) {
    constexpr int N = R + 1;
#pragma unroll
    for (int k2 = 0; k2 < N; k2++) ho_restrict1<R, 1>(c + N * k2, a1, b1);
#pragma unroll
    for (int k1 = 0; k1 < N; k1++) ho_restrict1<R, N>(c + k1, a2, b2);
}

template <int R>
__device__ inline void ho_bern(double u, double (&B)[R + 1], double (&dB)[R + 1]) {
    double s = 1.0 - u;
    if constexpr (R == 2) {
        B[0] = s * s;
        B[1] = 2.0 * u * s;
        B[2] = u * u;
        dB[0] = -2.0 * s;
        dB[1] = 2.0 * (s - u);
        dB[2] = 2.0 * u;
    } else {
        B[0] = s * s * s;
        B[1] = 3.0 * u * s * s;
        B[2] = 3.0 * u * u * s;
        B[3] = u * u * u;
        dB[0] = -3.0 * s * s;
        dB[1] = 3.0 * s * s - 6.0 * u * s;
        dB[2] = 6.0 * u * s - 3.0 * u * u;
        dB[3] = 3.0 * u * u;
    }
}

// Value and partial derivatives of the net at (u, v).
template <int R>
__device__ inline void ho_eval(const double (&c)[(R + 1) * (R + 1)], double u, double v, double& f, double& fu,
                               double& fv) {
    constexpr int N = R + 1;
    double Bu[N], dBu[N], Bv[N], dBv[N];
    ho_bern<R>(u, Bu, dBu);
    ho_bern<R>(v, Bv, dBv);
    f = fu = fv = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < N; k2++) {
        double r0 = 0.0, r1 = 0.0;
#pragma unroll
        for (int k1 = 0; k1 < N; k1++) {
            r0 += c[k1 + N * k2] * Bu[k1];
            r1 += c[k1 + N * k2] * dBu[k1];
        }
        f += r0 * Bv[k2];
        fu += r1 * Bv[k2];
        fv += r0 * dBv[k2];
    }
}

// False when the coefficients share a strict sign beyond a relative 1e-10
// (no zero of the polynomial on the square).
template <int N2>
__device__ inline bool ho_may_vanish(const double (&c)[N2]) {
    double big = 0.0;
#pragma unroll
    for (int q = 0; q < N2; q++) big = fmax(big, fabs(c[q]));
    double tol = 1e-10 * big;
    bool pos = false, neg = false;
#pragma unroll
    for (int q = 0; q < N2; q++) {
        pos |= c[q] >= -tol;
        neg |= c[q] <= tol;
    }
    return pos && neg;
}

// The two planes through a pixel's ray as functionals w . (p - o) + off of
// camera-space position (t, u, vh axes): perspective n X - a Z = 0 and
// n Y - b Z = 0, orthographic X = a and Y = b, with (a, b) the pixel's offset
// ell (i - cx, j - cy) on the projection plane.
__device__ inline void ho_pixel_planes(const Cam& c, int i, int j, double w1[3], double& off1, double w2[3],
                                       double& off2, double rcam[3]) {
    double a = c.ell * ((double)i - c.cx), b = c.ell * ((double)j - c.cy);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (c.ortho) {
            w1[k] = c.t[k];
            w2[k] = c.u[k];
        } else {
            w1[k] = c.n * c.t[k] - a * c.vh[k];
            w2[k] = c.n * c.u[k] - b * c.vh[k];
        }
    }
    off1 = c.ortho ? -a : 0.0;
    off2 = c.ortho ? -b : 0.0;
    rcam[0] = c.ortho ? 0.0 : a;
    rcam[1] = c.ortho ? 0.0 : b;
    rcam[2] = c.ortho ? 1.0 : c.n;
}

// Pixel rectangle of a leaf (App. A.2): the camera-aligned box of its
// Bernstein coefficients over the leaf's square, widened by a relative 1e-9.
template <int R>
__device__ inline Rect ho_rect(const Cam& c, const HoGeom& G, int tree, int level, uint32_t x, uint32_t y) {
    constexpr int N2 = (R + 1) * (R + 1);
    const double inv = 1.0 / (double)(1u << QMAX);
    double len = (double)(1u << (QMAX - level));
    double a1 = (double)x * inv, b1 = ((double)x + len) * inv, a2 = (double)y * inv, b2 = ((double)y + len) * inv;
    double lo[3], hi[3], mag = 0.0;
    const double* axes[3] = {c.t, c.u, c.vh};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double net[N2];
        ho_net<R>(G, tree, c.o, axes[k], 0.0, net);
        ho_restrict<R>(net, a1, b1, a2, b2);
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
#pragma unroll
        for (int q = 0; q < N2; q++) {
            lo[k] = fmin(lo[k], net[q]);
            hi[k] = fmax(hi[k], net[q]);
        }
        mag = fmax(mag, fmax(fabs(lo[k]), fabs(hi[k])));
    }
    double m = 1e-9 * (1.0 + mag);
    return cam_rect(c, lo[0] - m, hi[0] + m, lo[1] - m, hi[1] + m, lo[2] - m, hi[2] + m);
}

// Krawczyk's test on the square [u0, u0 + h] x [v0, v0 + h] of the leaf,
// widened by a relative 1e-9: with F = (f1, f2) and M the inverse Jacobian at
// the centre c, K = c - M F(c) + (I - M [J]) (Q - c), [J] the Jacobian's range
// over the square from the sub-square nets S1, S2 (differences of Bernstein
// coefficients).  K disjoint from Q: no root in Q (returns 0); K inside Q:
// exactly one (returns 1); otherwise undecided (returns 2).
template <int R>
__device__ inline int ho_krawczyk(const double (&f1)[(R + 1) * (R + 1)], const double (&f2)[(R + 1) * (R + 1)],
                                  const double (&S1)[(R + 1) * (R + 1)], const double (&S2)[(R + 1) * (R + 1)],
                                  double u0, double v0, double h) {
    constexpr int N = R + 1;
    double cu = u0 + 0.5 * h, cv = v0 + 0.5 * h;
    double a, au, av, b, bu, bv;
    ho_eval<R>(f1, cu, cv, a, au, av);
    ho_eval<R>(f2, cu, cv, b, bu, bv);
    double det = au * bv - av * bu;
    if (!(det != 0.0) || !isfinite(det)) return 2;
    double m00 = bv / det, m01 = -av / det, m10 = -bu / det, m11 = au / det;
    // ranges of the four partial derivatives over the square (leaf coordinates)
    double lo[4], hi[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        lo[q] = INFINITY;
        hi[q] = -INFINITY;
    }
#pragma unroll
    for (int k2 = 0; k2 < N; k2++)
#pragma unroll
        for (int k1 = 0; k1 < N; k1++) {
            if (k1 < R) {
                double d1 = S1[k1 + 1 + N * k2] - S1[k1 + N * k2], d2 = S2[k1 + 1 + N * k2] - S2[k1 + N * k2];
                lo[0] = fmin(lo[0], d1);
                hi[0] = fmax(hi[0], d1);
                lo[2] = fmin(lo[2], d2);
                hi[2] = fmax(hi[2], d2);
            }
            if (k2 < R) {
                double d1 = S1[k1 + N * (k2 + 1)] - S1[k1 + N * k2], d2 = S2[k1 + N * (k2 + 1)] - S2[k1 + N * k2];
                lo[1] = fmin(lo[1], d1);
                hi[1] = fmax(hi[1], d1);
                lo[3] = fmin(lo[3], d2);
                hi[3] = fmax(hi[3], d2);
            }
        }
    double sc = (double)R / h;  // d/du of the sub-square polynomial is R/h times the differences
    double mid[4], rad[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        mid[q] = 0.5 * (lo[q] + hi[q]) * sc;
        rad[q] = (0.5 * (hi[q] - lo[q]) * sc) * (1.0 + 1e-9) + 1e-300;
    }
    // rows of I - M [J]: [J] = [[J00, J01], [J10, J11]] = [[d f1/du, d f1/dv], [d f2/du, d f2/dv]]
    double e00 = fabs(1.0 - (m00 * mid[0] + m01 * mid[2])) + (fabs(m00) * rad[0] + fabs(m01) * rad[2]);
    double e01 = fabs(0.0 - (m00 * mid[1] + m01 * mid[3])) + (fabs(m00) * rad[1] + fabs(m01) * rad[3]);
    double e10 = fabs(0.0 - (m10 * mid[0] + m11 * mid[2])) + (fabs(m10) * rad[0] + fabs(m11) * rad[2]);
    double e11 = fabs(1.0 - (m10 * mid[1] + m11 * mid[3])) + (fabs(m10) * rad[1] + fabs(m11) * rad[3]);
    double r = 0.5 * h * (1.0 + 1e-9);
    double k0 = cu - (m00 * a + m01 * b), k1 = cv - (m10 * a + m11 * b);
    double r0 = r * (e00 + e01), r1 = r * (e10 + e11);
    if (!(isfinite(k0) && isfinite(k1) && isfinite(r0) && isfinite(r1))) return 2;
    if (k0 + r0 < cu - r || k0 - r0 > cu + r || k1 + r1 < cv - r || k1 - r1 > cv + r) return 0;
    if (k0 - r0 > cu - r && k0 + r0 < cu + r && k1 - r1 > cv - r && k1 + r1 < cv + r) return 1;
    return 2;
}

// Newton's method on (f1, f2) = 0 with the nets over the leaf square, from (u, v).
template <int R>
__device__ inline bool ho_newton_local(const double (&f1)[(R + 1) * (R + 1)], const double (&f2)[(R + 1) * (R + 1)],
                                       double& u, double& v) {
    double prev = INFINITY;
    for (int it = 0; it < 30; it++) {
        double a, au, av, b, bu, bv;
        ho_eval<R>(f1, u, v, a, au, av);
        ho_eval<R>(f2, u, v, b, bu, bv);
        double det = au * bv - av * bu;
        if (det == 0.0) return false;
        double du = (bv * a - av * b) / det, dv = (au * b - bu * a) / det;
        u -= du;
        v -= dv;
        if (!(fabs(u) < 4.0 && fabs(v) < 4.0)) return false;
        double step = fabs(du) + fabs(dv);
        if (step < 1e-14) return true;
        // near a tangency the Jacobian is close to singular and the steps stall
        // at rounding level above 1e-14: a small step that no longer shrinks
        // has converged as far as the arithmetic allows
        if (step < 1e-8 && step > 0.25 * prev) return true;
        prev = step;
    }
    return false;
}

}  // namespace rc
