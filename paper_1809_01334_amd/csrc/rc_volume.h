// rc_volume.h -- degree-R volume trees: each tree maps its reference cube to
// space by a tensor product of degree-R Lagrange polynomials on the
// Gauss-Lobatto nodes (eq. nodal, eq. tensorgeom); the control points are the
// map's values at the node triples, m1 fastest.  A leaf is a sub-cube of the
// reference cube; its faces are degree-R patches (the map with one reference
// coordinate held fixed), searched for ray crossings with the Bernstein and
// Krawczyk machinery of the surfaces (App. A.1); its pixel rectangle comes
// from the Bernstein coefficients over the leaf (App. A.2).
#pragma once

#include "rc_surface_ho.h"

namespace rc {

struct VolGeom {
    HoGeom H;                    // the node-to-Bernstein matrix (H.pts unused)
    double eta[HO_MAXR + 1];     // Gauss-Lobatto nodes
    const double* pts;           // (R+1)^3 control points of 3 doubles per tree
};

// Host: nodes and node-to-Bernstein matrix of degree R (rc_volume.hip).
void vol_geom_init(int R, const double* pts, VolGeom& V);

// Lagrange basis on the nodes at t, and its derivative.
template <int R>
__device__ inline void vol_lagrange(const VolGeom& V, double t, double (&L)[R + 1], double (&dL)[R + 1]) {
#pragma unroll
    for (int m = 0; m <= R; m++) {
        double p = 1.0, dp = 0.0;
#pragma unroll
        for (int l = 0; l <= R; l++) {
            if (l == m) continue;
            double inv = 1.0 / (V.eta[m] - V.eta[l]);
            double f = (t - V.eta[l]) * inv;
            dp = dp * f + p * inv;
            p *= f;
        }
        L[m] = p;
        dL[m] = dp;
    }
}

// X(xi) of tree `tree` and its Jacobian J[k][a] = dX_k / dxi_a.
template <int R>
__device__ inline void vol_point(const VolGeom& V, int tree, const double xi[3], double X[3], double J[3][3]) {
    constexpr int N = R + 1;
    const double* z = V.pts + 3 * N * N * N * tree;
    double L[3][N], dL[3][N];
#pragma unroll
    for (int a = 0; a < 3; a++) vol_lagrange<R>(V, xi[a], L[a], dL[a]);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        X[k] = 0.0;
        J[k][0] = J[k][1] = J[k][2] = 0.0;
    }
#pragma unroll 1
    for (int m3 = 0; m3 < N; m3++)
#pragma unroll
        for (int m2 = 0; m2 < N; m2++)
#pragma unroll
            for (int m1 = 0; m1 < N; m1++) {
                const double* zc = z + 3 * (m1 + N * (m2 + N * m3));
                double w = L[0][m1] * L[1][m2] * L[2][m3];
                double w0 = dL[0][m1] * L[1][m2] * L[2][m3];
                double w1 = L[0][m1] * dL[1][m2] * L[2][m3];
                double w2 = L[0][m1] * L[1][m2] * dL[2][m3];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    double zk = zc[k];
                    X[k] += w * zk;
                    J[k][0] += w0 * zk;
                    J[k][1] += w1 * zk;
                    J[k][2] += w2 * zk;
                }
            }
}

// Reference coordinates of the real-space point x: Newton's method from the
// start xi (replaced by the result); true when the step falls below 1e-13.
template <int R>
__device__ inline bool vol_invert(const VolGeom& V, int tree, const double x[3], double xi[3]) {
    for (int it = 0; it < 40; it++) {
        double X[3], J[3][3];
        vol_point<R>(V, tree, xi, X, J);
        double e0 = X[0] - x[0], e1 = X[1] - x[1], e2 = X[2] - x[2];
        // J^-1 e by the adjugate
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        double c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        double c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        double c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        double c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        double c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        double det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
        if (!(det != 0.0) || !isfinite(det)) return false;
        double inv = 1.0 / det;
        double s0 = (c00 * e0 + c01 * e1 + c02 * e2) * inv;
        double s1 = (c10 * e0 + c11 * e1 + c12 * e2) * inv;
        double s2 = (c20 * e0 + c21 * e1 + c22 * e2) * inv;
        xi[0] -= s0;
        xi[1] -= s1;
        xi[2] -= s2;
        if (!(fabs(xi[0]) < 4.0 && fabs(xi[1]) < 4.0 && fabs(xi[2]) < 4.0)) return false;
        if (fabs(s0) + fabs(s1) + fabs(s2) < 1e-13) return true;
    }
    return false;
}

// Control points of the tree's face patch at reference coordinate xi_k = c:
// the patch in (xi_a, xi_b), a = k + 1, b = k + 2 (mod 3), interpolates the
// map on that plane exactly: P[m1 + N m2] = sum over m_k of z l_{m_k}(c).
template <int R>
__device__ inline void vol_face_points(const VolGeom& V, int tree, int k, double c,
                                       double (&P)[3 * (R + 1) * (R + 1)]) {
    constexpr int N = R + 1;
    const double* z = V.pts + 3 * N * N * N * tree;
    double L[N], dL[N];
    vol_lagrange<R>(V, c, L, dL);
    int a = (k + 1) % 3, b = (k + 2) % 3;
#pragma unroll
    for (int m2 = 0; m2 < N; m2++)
#pragma unroll
        for (int m1 = 0; m1 < N; m1++) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int mk = 0; mk < N; mk++) {
                int m[3];
                m[k] = mk;
                m[a] = m1;
                m[b] = m2;
                const double* zc = z + 3 * (m[0] + N * (m[1] + N * m[2]));
                s0 += L[mk] * zc[0];
                s1 += L[mk] * zc[1];
                s2 += L[mk] * zc[2];
            }
            P[3 * (m1 + N * m2)] = s0;
            P[3 * (m1 + N * m2) + 1] = s1;
            P[3 * (m1 + N * m2) + 2] = s2;
        }
}

// Bernstein coefficients over the face square of L(p) = w . (p - o) + off on
// a face patch with control points P.
template <int R>
__device__ inline void vol_face_net(const VolGeom& V, const double (&P)[3 * (R + 1) * (R + 1)], const double o[3],
                                    const double w[3], double off, double (&c)[(R + 1) * (R + 1)]) {
    constexpr int N = R + 1;
    double v[N * N], tmp[N * N];
#pragma unroll
    for (int q = 0; q < N * N; q++)
        v[q] = ((w[0] * (P[3 * q] - o[0]) + w[1] * (P[3 * q + 1] - o[1])) + w[2] * (P[3 * q + 2] - o[2])) + off;
#pragma unroll
    for (int m2 = 0; m2 < N; m2++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < N; m++) s += V.H.nb[k * N + m] * v[m + N * m2];
            tmp[k + N * m2] = s;
        }
#pragma unroll
    for (int k1 = 0; k1 < N; k1++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < N; m++) s += V.H.nb[k * N + m] * tmp[k1 + N * m];
            c[k1 + N * k] = s;
        }
}

// Pixel rectangle of a leaf (App. A.2): the camera-aligned box of the
// Bernstein coefficients of the map over the leaf's cube, widened by a
// relative 1e-9.
template <int R>
__device__ inline Rect vol_rect(const Cam& c, const VolGeom& V, int tree, int level, uint32_t x, uint32_t y,
                                uint32_t z) {
    constexpr int N = R + 1, N3 = N * N * N;
    const double inv = 1.0 / (double)(1u << QMAX);
    double len = (double)(1u << (QMAX - level));
    double lo_[3] = {(double)x * inv, (double)y * inv, (double)z * inv};
    double hi_[3] = {((double)x + len) * inv, ((double)y + len) * inv, ((double)z + len) * inv};
    const double* zp = V.pts + 3 * N3 * tree;
    const double* axes[3] = {c.t, c.u, c.vh};
    double lo[3], hi[3], mag = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double* w = axes[k];
        double net[N3];
#pragma unroll
        for (int q = 0; q < N3; q++)
            net[q] = (w[0] * (zp[3 * q] - c.o[0]) + w[1] * (zp[3 * q + 1] - c.o[1])) + w[2] * (zp[3 * q + 2] - c.o[2]);
        // node values to Bernstein coefficients, one axis at a time
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const int st = ax == 0 ? 1 : (ax == 1 ? N : N * N);
            double t[N3];
#pragma unroll
            for (int q = 0; q < N3; q++) {
                int jj = (q / st) % N;
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < N; m++) s += V.H.nb[jj * N + m] * net[q + (m - jj) * st];
                t[q] = s;
            }
#pragma unroll
            for (int q = 0; q < N3; q++) net[q] = t[q];
        }
        // restricted to the leaf's cube, one axis at a time over all its lines
#pragma unroll
        for (int i2 = 0; i2 < N; i2++)
#pragma unroll
            for (int i1 = 0; i1 < N; i1++) ho_restrict1<R, 1>(net + N * (i1 + N * i2), lo_[0], hi_[0]);
#pragma unroll
        for (int i2 = 0; i2 < N; i2++)
#pragma unroll
            for (int i1 = 0; i1 < N; i1++) ho_restrict1<R, N>(net + i1 + N * N * i2, lo_[1], hi_[1]);
#pragma unroll
        for (int i2 = 0; i2 < N; i2++)
#pragma unroll
            for (int i1 = 0; i1 < N; i1++) ho_restrict1<R, N * N>(net + i1 + N * i2, lo_[2], hi_[2]);
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
#pragma unroll
        for (int q = 0; q < N3; q++) {
            lo[k] = fmin(lo[k], net[q]);
            hi[k] = fmax(hi[k], net[q]);
        }
        mag = fmax(mag, fmax(fabs(lo[k]), fabs(hi[k])));
    }
    double m = 1e-9 * (1.0 + mag);
    return cam_rect(c, lo[0] - m, hi[0] + m, lo[1] - m, hi[1] + m, lo[2] - m, hi[2] + m);
}

}  // namespace rc
