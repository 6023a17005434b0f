// rc_shell.h -- the six-tree spherical shell (equiangular cubed sphere):
// element description, canonical FP64 predicates (lenient box, ray pairing)
// and the FP64 Newton inversion of the tree map used for field points.
//
// Tree k: axis m = k / 2, sign sg = +1 (k even) or -1, frame e1 = unit(m+1),
// e2 = unit(m+2), e3 = sg unit(m); t in [0,1]^3 maps to
//   x = r (a e1 + b e2 + e3) / sqrt(1 + a^2 + b^2),
//   a = tan(pi/4 (2 t1 - 1)), b = tan(pi/4 (2 t2 - 1)), r = r0 + (r1 - r0) t3.
// Constant t1 or t2 are planes through the origin and constant t3 spheres,
// so a ray meets an element in at most two intervals.
#pragma once

#include "rc_internal.h"

namespace rc {

struct ShellElem {
    int m, m1, m2;
    double sg;
    double alo, ahi, blo, bhi, rlo, rhi;
    double tlo[3];
    int level;
    double r0, r1;
};

// geom = [r0, r1, L, tan table (2^L + 1 entries)]
__device__ inline ShellElem shell_elem(const double* geom, int k, int level, uint32_t x, uint32_t y, uint32_t z) {
#pragma clang fp contract(off)
    ShellElem e;
    e.m = k >> 1;
    e.sg = (k & 1) ? -1.0 : 1.0;
    e.m1 = (e.m + 1) % 3;
    e.m2 = (e.m + 2) % 3;
    e.r0 = geom[0];
    e.r1 = geom[1];
    int L = (int)geom[2];
    L = L < 0 ? 0 : (L > QMAX ? QMAX : L);  // table level; rc_forest_index rejects others
    const double* tab = geom + 3;
    uint32_t len = 1u << (QMAX - level);
    int sh = QMAX - L;
    e.alo = tab[x >> sh];
    e.ahi = tab[(x + len) >> sh];
    e.blo = tab[y >> sh];
    e.bhi = tab[(y + len) >> sh];
    double dr = e.r1 - e.r0;
    e.rlo = e.r0 + dr * ((double)z * QSCALE);
    e.rhi = e.r0 + dr * ((double)(z + len) * QSCALE);
    e.tlo[0] = (double)x * QSCALE;
    e.tlo[1] = (double)y * QSCALE;
    e.tlo[2] = (double)z * QSCALE;
    e.level = level;
    return e;
}

// Lenient camera-space box (App. A.2 "more lenient approximate criterion"): the
// element lies in the convex hull of rlo c_i and (rhi / mu) c_i, c_i the unit
// corner directions and mu the smallest cosine between them and their mean.
__device__ inline Rect shell_rect(const Cam& c, const ShellElem& e) {
#pragma clang fp contract(off)
    double cd[4][3];
    double av[2] = {e.alo, e.ahi}, bv[2] = {e.blo, e.bhi};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        double a = av[q & 1], b = bv[q >> 1];
        double nrm = sqrt((1.0 + a * a) + b * b);
        double v[3];
        v[e.m1] = a / nrm;
        v[e.m2] = b / nrm;
        v[e.m] = e.sg / nrm;
        cd[q][0] = v[0];
        cd[q][1] = v[1];
        cd[q][2] = v[2];
    }
    double mean[3];
#pragma unroll
    for (int k = 0; k < 3; k++) mean[k] = ((cd[0][k] + cd[1][k]) + cd[2][k]) + cd[3][k];
    double ml = sqrt((mean[0] * mean[0] + mean[1] * mean[1]) + mean[2] * mean[2]);
#pragma unroll
    for (int k = 0; k < 3; k++) mean[k] = mean[k] / ml;
    double mu = 1.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        double d = (cd[q][0] * mean[0] + cd[q][1] * mean[1]) + cd[q][2] * mean[2];
        if (d < mu) mu = d;
    }
    double sin_ = e.rlo * (1.0 - 1e-12), sout = e.rhi * (1.0 + 1e-12) / mu;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double* axes[3] = {c.t, c.u, c.vh};
#pragma unroll
    for (int q = 0; q < 8; q++) {
        double sc = (q < 4) ? sin_ : sout;
        double p[3];
#pragma unroll
        for (int k = 0; k < 3; k++) p[k] = sc * cd[q & 3][k] - c.o[k];
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const double* a = axes[ax];
            double v = (a[0] * p[0] + a[1] * p[1]) + a[2] * p[2];
            if (v < lo[ax]) lo[ax] = v;
            if (v > hi[ax]) hi[ax] = v;
        }
    }
    Rect r{1, 0, 1, 0};
    double z0 = lo[2], z1 = hi[2];
    if (z1 < c.n || z0 > c.zfar) return r;
    double zc0 = z0 < c.n ? c.n : z0;
    double zc1 = z1 > c.zfar ? c.zfar : z1;
    Rect q;
    axis_pixels(c, lo[0], hi[0], zc0, zc1, c.cx, c.w, q.i0, q.i1);
    axis_pixels(c, lo[1], hi[1], zc0, zc1, c.cy, c.h, q.j0, q.j1);
    if (q.empty()) return r;
    return q;
}

// Plane of constant a (tangent axis mt) through the origin: P(v) = v[mt] - a (sg v[m]).
// lower: the element keeps P >= 0, else P < 0.  Returns false on a miss.
__device__ inline bool shell_plane(const ShellElem& e, int mt, double a, bool lower, const double rho[3],
                                   const double r[3], double& sa, double& sb) {
#pragma clang fp contract(off)
    double Pr = r[mt] - a * (e.sg * r[e.m]);
    double Pp = rho[mt] - a * (e.sg * rho[e.m]);
    if (Pr != 0.0) {
        double sx = -(Pp / Pr);
        bool ge = lower ? (Pr > 0.0) : (Pr < 0.0);
        if (ge) {
            if (sx > sa) sa = sx;
        } else {
            if (sx < sb) sb = sx;
        }
        return true;
    }
    return lower ? (Pp >= 0.0) : (Pp < 0.0);
}

// Parameters where |rho + s r| = R, |.|^2 = A s^2 + 2 B s + C (stable roots).
__device__ inline bool shell_sphere(double A, double B, double C, double R, double& lo, double& hi) {
#pragma clang fp contract(off)
    double c = C - R * R;
    double D = B * B - A * c;
    if (!(D > 0.0)) return false;
    double sq = sqrt(D);
    double q = (B >= 0.0) ? -(B + sq) : (sq - B);
    double s1 = q / A, s2 = c / q;
    lo = s1 < s2 ? s1 : s2;
    hi = s1 < s2 ? s2 : s1;
    return true;
}

// Hit intervals (at most two) of a ray with an element, clipped to [smin, smax].
__device__ inline int shell_pair(const Cam& c, const ShellElem& e, const double rho[3], const double r[3],
                                 double iv[4]) {
#pragma clang fp contract(off)
    double sa = c.smin, sb = c.smax;
    if (!shell_plane(e, e.m1, e.alo, true, rho, r, sa, sb)) return 0;
    if (!shell_plane(e, e.m1, e.ahi, false, rho, r, sa, sb)) return 0;
    if (!shell_plane(e, e.m2, e.blo, true, rho, r, sa, sb)) return 0;
    if (!shell_plane(e, e.m2, e.bhi, false, rho, r, sa, sb)) return 0;
    if (!(sb > sa)) return 0;
    double A = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    double B = (rho[0] * r[0] + rho[1] * r[1]) + rho[2] * r[2];
    double C = (rho[0] * rho[0] + rho[1] * rho[1]) + rho[2] * rho[2];
    double o0, o1, i0, i1;
    if (!shell_sphere(A, B, C, e.rhi, o0, o1)) return 0;
    if (o0 > sa) sa = o0;
    if (o1 < sb) sb = o1;
    if (!(sb > sa)) return 0;
    if (!shell_sphere(A, B, C, e.rlo, i0, i1)) {
        iv[0] = sa;
        iv[1] = sb;
        return 1;
    }
    int n = 0;
    double b0 = i0 < sb ? i0 : sb;
    if (b0 > sa) {
        iv[0] = sa;
        iv[1] = b0;
        n = 1;
    }
    double a1 = i1 > sa ? i1 : sa;
    if (sb > a1) {
        iv[2 * n] = a1;
        iv[2 * n + 1] = sb;
        n++;
    }
    return n;
}

// Newton inversion of the tree map in FP64: reference t (in/out, warm start)
// for the real point x, in the tree frame X = (x[m1], x[m2], sg x[m]) where the
// map reads X = (r / rho) (a, b, 1).  Converged to a residual of 1e-13 or after
// 8 steps.
__device__ inline void shell_newton(const ShellElem& e, const double x[3], double t[3]) {
    const double qpi = 0.78539816339744830962;  // pi / 4
    const double hpi = 1.57079632679489661923;  // pi / 2
    double X1 = x[e.m1], X2 = x[e.m2], X3 = e.sg * x[e.m];
    double dr = e.r1 - e.r0;
    for (int it = 0; it < 8; it++) {
        double a = tan(qpi * (2.0 * t[0] - 1.0));
        double b = tan(qpi * (2.0 * t[1] - 1.0));
        double r = e.r0 + dr * t[2];
        double rho2 = 1.0 + a * a + b * b;
        double rho = sqrt(rho2);
        double f = r / rho;
        double F1 = f * a - X1, F2 = f * b - X2, F3 = f - X3;
        if (fmax(fabs(F1), fmax(fabs(F2), fabs(F3))) <= 1e-13) break;
        double r3 = r / (rho2 * rho);
        double da = hpi * (1.0 + a * a), db = hpi * (1.0 + b * b);
        // Jacobian columns d/dt1, d/dt2, d/dt3
        double J11 = r3 * (1.0 + b * b) * da, J21 = -r3 * a * b * da, J31 = -r3 * a * da;
        double J12 = -r3 * a * b * db, J22 = r3 * (1.0 + a * a) * db, J32 = -r3 * b * db;
        double J13 = a / rho * dr, J23 = b / rho * dr, J33 = dr / rho;
        double det = J11 * (J22 * J33 - J23 * J32) - J12 * (J21 * J33 - J23 * J31) + J13 * (J21 * J32 - J22 * J31);
        double id = 1.0 / det;
        double d1 = (F1 * (J22 * J33 - J23 * J32) - J12 * (F2 * J33 - J23 * F3) + J13 * (F2 * J32 - J22 * F3)) * id;
        double d2 = (J11 * (F2 * J33 - J23 * F3) - F1 * (J21 * J33 - J23 * J31) + J13 * (J21 * F3 - F2 * J31)) * id;
        double d3 = (J11 * (J22 * F3 - F2 * J32) - J12 * (J21 * F3 - F2 * J31) + F1 * (J21 * J32 - J22 * J31)) * id;
        t[0] -= d1;
        t[1] -= d2;
        t[2] -= d3;
    }
}

}  // namespace rc
