// rc_steps.h -- one FP32 step of the Gauss and Simpson integrators (Sec. 2.7)
// over a piece of a segment, from (A, B) = (1, 0); the forward (rc_integrators.hip)
// and the adjoint's recomputation (rc_backward.hip) evaluate the same formulas.
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

}  // namespace rc
