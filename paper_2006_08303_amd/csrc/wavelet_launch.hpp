// Host-side entry points of the wavelet (x) DCT prior (wavelet.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace cip {

// Forward 2D transform of `planes` planes of x (N1 x N2), `levels` levels:
// coefficients to coef (Mallat layout), tmp is staging of the same size.
hipError_t wavelet_forward(const float* x, float* coef, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st);
// Inverse: coef (destroyed) -> x; tmp is staging.
hipError_t wavelet_inverse(float* coef, float* x, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st);
// Band DCT, soft threshold, dual update and back (see wavelet.hpp), S <= 8;
// rs: when given, two residual partial sums per work-group
// (wavelet_state_groups of them).
hipError_t wavelet_state(float* coef, float* v, const float* cs, int S, int N1, int N2,
                         float kappa, int first, hipStream_t st, float* rs = nullptr);
int wavelet_state_groups(int N1, int N2);
// After a penalty change: v re-expressed for the new threshold (u scaled by
// sc) and coef = C_S^T (t - u') for the inverse transform.
hipError_t wavelet_emit(float* coef, float* v, const float* cs, int S, int N1, int N2,
                        float kappa, float sc, hipStream_t st);

}  // namespace cip
