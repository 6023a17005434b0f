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

// Component k (0..2, known only at run time) of a 3-vector, by selects so the
// vector stays in registers.
__device__ inline double pick(const double v[3], int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

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
        double va = a / nrm, vb = b / nrm, vc = e.sg / nrm;
#pragma unroll
        for (int k = 0; k < 3; k++) cd[q][k] = k == e.m1 ? va : (k == e.m2 ? vb : vc);
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
    double Pr = pick(r, mt) - a * (e.sg * pick(r, e.m));
    double Pp = pick(rho, mt) - a * (e.sg * pick(rho, e.m));
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
        if (n == 0) {
            iv[0] = a1;
            iv[1] = sb;
        } else {
            iv[2] = a1;
            iv[3] = sb;
        }
        n++;
    }
    return n;
}

// Inversion of the tree map in FP64.  The map sends rays from the centre to
// rays, so j_k(t) = x splits into tan(theta1(t1)) = X1 / X3,
// tan(theta2(t2)) = X2 / X3 and r(t3) = |x| in the tree frame
// X = (x[m1], x[m2], sg x[m]), with theta(t) = pi/4 (2 t - 1).  The angular
// equations are solved by Newton's method on theta, warm-started along the
// ray; the radial one is linear.

// tan(d) for |d| <= 0.1 from its Taylor series (coefficients from the
// Bernoulli numbers); the first omitted term is below 2e-18.
__device__ inline double tan_small(double d) {
    double z = d * d;
    double p = 929569.0 / 638512875.0;
    p = fma(p, z, 21844.0 / 6081075.0);
    p = fma(p, z, 1382.0 / 155925.0);
    p = fma(p, z, 62.0 / 2835.0);
    p = fma(p, z, 17.0 / 315.0);
    p = fma(p, z, 2.0 / 15.0);
    p = fma(p, z, 1.0 / 3.0);
    return fma(d * z, p, d);
}

// tan(d) for |d| <= 0.8: halve until |d| <= 0.1, then double back with
// tan(2 x) = 2 tan(x) / (1 - tan(x)^2).
__device__ inline double tan_step(double d) {
    int k = 0;
    while (fabs(d) > 0.1 && k < 3) {
        d *= 0.5;
        k++;
    }
    double t = tan_small(d);
    for (int i = 0; i < k; i++) t = (t + t) / fma(-t, t, 1.0);
    return t;
}

// Newton for theta with tan(theta) = A from the pair (theta, T = tan(theta)):
// theta += d, d = -(T - A) / (1 + T^2) limited to |d| <= 0.5 (the tree spans
// pi/2 in theta), and T advanced by the addition theorem.  Stops at
// |T - A| <= 1e-13.
__device__ inline void angle_newton(double A, double& th, double& T) {
    for (int it = 0; it < 24; it++) {
        double res = T - A;
        if (fabs(res) <= 1e-13) break;
        double d = -res / fma(T, T, 1.0);
        d = fmin(fmax(d, -0.5), 0.5);
        th += d;
        double tau = tan_step(d);
        T = (T + tau) / fma(-T, tau, 1.0);
    }
}

// Leaf reference coordinates of the real point x (three floats in [0, 1] up
// to rounding), updating the angle state (th1, T1), (th2, T2).
struct ShellRef {
    double th_lo1, th_lo2, k_ang, k_rad, r0, tlo3;
    double th1, T1, th2, T2;
};

__device__ inline ShellRef shell_ref_init(const ShellElem& e) {
    const double hpi = 1.57079632679489661923;  // pi / 2
    const double qpi = 0.78539816339744830962;  // pi / 4
    ShellRef s;
    double scale = ldexp(1.0, e.level);
    s.th_lo1 = hpi * e.tlo[0] - qpi;
    s.th_lo2 = hpi * e.tlo[1] - qpi;
    s.k_ang = scale / hpi;
    s.k_rad = scale / (e.r1 - e.r0);
    s.r0 = e.r0;
    s.tlo3 = e.tlo[2] * scale;
    s.th1 = s.th_lo1;  // start at the element's low corner, where tan is the table value
    s.T1 = e.alo;
    s.th2 = s.th_lo2;
    s.T2 = e.blo;
    return s;
}

__device__ inline void shell_ref_point(const ShellElem& e, ShellRef& s, const double x[3], float xi[3]) {
    double X1 = pick(x, e.m1), X2 = pick(x, e.m2), X3 = e.sg * pick(x, e.m);
    angle_newton(X1 / X3, s.th1, s.T1);
    angle_newton(X2 / X3, s.th2, s.T2);
    double rr = sqrt(fma(X1, X1, fma(X2, X2, X3 * X3)));
    xi[0] = (float)((s.th1 - s.th_lo1) * s.k_ang);
    xi[1] = (float)((s.th2 - s.th_lo2) * s.k_ang);
    xi[2] = (float)(fma(rr - s.r0, s.k_rad, -s.tlo3));
}

}  // namespace rc
