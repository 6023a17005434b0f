// rc_steps.h -- one FP32 step of the Gauss and Simpson integrators (Sec. 2.7)
// over a piece of a segment, from (A, B) = (1, 0), and the reverse of the RK4,
// Gauss and Simpson steps; the forward (rc_integrators.hip) and the adjoint's
// recomputation (rc_backward.hip, and the recursion's adjoint in
// rc_integrators.hip) evaluate the same formulas.
#pragma once

#include <hip/hip_runtime.h>

namespace rc {

// Implicit Gauss, two stages, from (1, 0): eq. gaussAB with eq. gaussABab.
__device__ inline float2 gauss2_step(float b0, float b1, float g0, float g1, float h) {
    const float r3_12 = 0.14433756729740643f;  // sqrt(3) / 12
    float a1 = h * (b0 + b1) * 0.25f;
    float a2 = h * h * b0 * b1 * (1.0f / 12.0f);
    float c1 = h * (g0 + g1) * 0.5f;
    float c2 = h * h * (b0 * g1 - b1 * g0) * r3_12;
    float den = 1.0f + a1 + a2;
    return make_float2((1.0f - a1 + a2) / den, (c1 + c2) / den);
}

// Simpson quadrature of the closed form: eq. simpson, weights 1/6, 4/6, 1/6
// at the far end, the middle and the near end.
__device__ inline float2 simpson_step(float b0, float b1, float b2, float g0, float g1, float g2, float h) {
    float A = expf(-h * (b0 + 4.0f * b1 + b2) * (1.0f / 6.0f));
    float B = h * (A * g0 + 4.0f * sqrtf(A) * g1 + g2) * (1.0f / 6.0f);
    return make_float2(A, B);
}

// Reverse of rk4_step: adds the adjoints of (b0, bm, b1, g0, gm, g1) given
// those of the step's (A, B).
__device__ inline void rk4_step_bwd(float b0, float bm, float b1, float g0, float gm, float h, float Abar, float Bbar,
                                    float& db0, float& dbm, float& db1, float& dg0, float& dgm, float& dg1) {
    (void)g0;
    float hh = 0.5f * h;
    // forward intermediates
    float A1 = fmaf(-hh, b0, 1.0f);
    float A2 = fmaf(-hh * bm, A1, 1.0f);
    float A3 = fmaf(-h * bm, A2, 1.0f);
    float B1 = hh * g0;
    float f1 = fmaf(-bm, B1, gm);
    float B2 = hh * f1;
    float f2 = fmaf(-bm, B2, gm);
    float B3 = h * f2;
    // A = 1 - (h/6) (b0 + 2 bm (A1 + A2) + b1 A3)
    float sa = -h * (1.0f / 6.0f) * Abar;
    db0 += sa;
    dbm += 2.0f * (A1 + A2) * sa;
    float A1b = 2.0f * bm * sa, A2b = 2.0f * bm * sa;
    db1 += A3 * sa;
    float A3b = b1 * sa;
    // B = (h/6) (g0 + 2 (f1 + f2) + f3)
    float sb = h * (1.0f / 6.0f) * Bbar;
    dg0 += sb;
    float f1b = 2.0f * sb, f2b = 2.0f * sb, f3b = sb;
    // f3 = g1 - b1 B3
    dg1 += f3b;
    db1 -= B3 * f3b;
    float B3b = -b1 * f3b;
    f2b += h * B3b;  // B3 = h f2
    // f2 = gm - bm B2
    dgm += f2b;
    dbm -= B2 * f2b;
    float B2b = -bm * f2b;
    f1b += hh * B2b;  // B2 = hh f1
    // f1 = gm - bm B1
    dgm += f1b;
    dbm -= B1 * f1b;
    float B1b = -bm * f1b;
    dg0 += hh * B1b;  // B1 = hh g0
    // A3 = 1 - h bm A2
    dbm -= h * A2 * A3b;
    A2b -= h * bm * A3b;
    // A2 = 1 - hh bm A1
    dbm -= hh * A1 * A2b;
    A1b -= hh * bm * A2b;
    // A1 = 1 - hh b0
    db0 -= hh * A1b;
}

// Reverse of the two-stage implicit Gauss step (eq. gaussAB with eq.
// gaussABab, as evaluated by the forward): adds the adjoints of (b0, b1, g0,
// g1), the stage values at 1/2 -+ sqrt(3)/6 of the piece from its far end,
// given those of the step's (A, B).
__device__ inline void gauss2_step_bwd(float b0, float b1, float g0, float g1, float h, float Abar, float Bbar,
                                       float& db0, float& db1, float& dg0, float& dg1) {
    const float r3_12 = 0.14433756729740643f;  // sqrt(3) / 12
    float a1 = h * (b0 + b1) * 0.25f;
    float a2 = h * h * b0 * b1 * (1.0f / 12.0f);
    float c1 = h * (g0 + g1) * 0.5f;
    float c2 = h * h * (b0 * g1 - b1 * g0) * r3_12;
    float rd = 1.0f / (1.0f + a1 + a2);
    float A = (1.0f - a1 + a2) * rd, B = (c1 + c2) * rd;
    // A = (1 - a1 + a2) / den, B = (c1 + c2) / den, den = 1 + a1 + a2
    float a1b = (-(1.0f + A) * Abar - B * Bbar) * rd;
    float a2b = ((1.0f - A) * Abar - B * Bbar) * rd;
    float cb = Bbar * rd;
    float s1 = h * 0.25f * a1b, s2 = h * h * (1.0f / 12.0f) * a2b;
    float t = h * 0.5f * cb, u = h * h * r3_12 * cb;
    db0 += s1 + s2 * b1 + u * g1;
    db1 += s1 + s2 * b0 - u * g0;
    dg0 += t - u * b1;
    dg1 += t + u * b0;
}

// Reverse of the Simpson step of the closed form (eq. simpson): stage values
// at the far end, the middle and the near end of the piece.  B depends on the
// exponent through A and sqrt(A) = exp(half the exponent), so no division.
__device__ inline void simpson_step_bwd(float b0, float b1, float b2, float g0, float g1, float g2, float h,
                                        float Abar, float Bbar, float& db0, float& db1, float& db2, float& dg0,
                                        float& dg1, float& dg2) {
    float h6 = h * (1.0f / 6.0f);
    float A = expf(-h * (b0 + 4.0f * b1 + b2) * (1.0f / 6.0f));
    float sA = sqrtf(A);
    dg0 += h6 * A * Bbar;
    dg1 += 4.0f * h6 * sA * Bbar;
    dg2 += h6 * Bbar;
    // d/d(b0 + 4 b1 + b2): A' = -h6 A, sqrt(A)' = -h6 sqrt(A) / 2
    float sb = -h6 * (A * Abar + h6 * Bbar * (A * g0 + 2.0f * sA * g1));
    db0 += sb;
    db1 += 4.0f * sb;
    db2 += sb;
}

}  // namespace rc
