// Wavelet (x) DCT analysis prior (Section V-A's Kronecker basis): the 2D
// Symmlet-8 wavelet transform of every plane followed by the orthonormal
// DCT-II along the planes, T = C_S (x) W_2D, orthonormal (T^T T = I).
//
// W_2D is the periodized orthonormal DWT in Mallat's pyramid: level l
// transforms the top-left R x C corner (R = N1 / 2^l, C = N2 / 2^l) along
// both axes, one axis at a time; along an axis of length n,
//   a[k] = sum_t h[t] x[(2k + t) mod n],  d[k] = sum_t g[t] x[(2k + t) mod n],
// with g[t] = (-1)^t h[15 - t], stored as [a | d]. The inverse is the
// transpose: x[2m + e] = sum_j a[(m - j) mod n/2] h[e + 2j]
//                                + d[(m - j) mod n/2] g[e + 2j].
// The transform runs out of place, one launch per axis and level, between
// a coefficient buffer and a staging buffer; the band DCT, the soft
// threshold and the dual update (v-form state, as in the other analysis
// priors) are one pointwise kernel over the coefficients.
#pragma once
#include <hip/hip_runtime.h>

namespace cip {

// Symmlet-8 scaling filter (least-asymmetric orthonormal Daubechies
// wavelet with 8 vanishing moments), in FP32.
__device__ constexpr float kSym8[16] = {
    -0.0033824159510061256f, -0.0005421323317911481f, 0.03169508781149298f,
    0.007607487324917605f,   -0.1432942383508097f,    -0.061273359067658524f,
    0.4813596512583722f,     0.7771857517005235f,     0.3644418948353314f,
    -0.05194583810770904f,   -0.027219029917056003f,  0.049137179673607506f,
    0.003808752013890615f,   -0.01495225833704823f,   -0.0003029205147213668f,
    0.0018899503327594609f};

__device__ __forceinline__ float sym8_g(int t) {   // wavelet filter
  return (t & 1) ? -kSym8[15 - t] : kSym8[15 - t];
}

// Forward level along the rows (contiguous axis) of the R x C corner of
// every plane (leading dimension N2, plane stride N1 N2): in -> out.
// Thread (p, r, k), k < C / 2, forms a[k] and d[k].
__global__ void k_dwt_rows(const float* __restrict__ in, float* __restrict__ out, int planes,
                           int N1, int N2, int R, int C) {
  const int h = C >> 1;
  const size_t n = (size_t)planes * R * h;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int k = (int)(idx % h);
  const int r = (int)((idx / h) % R);
  const int p = (int)(idx / ((size_t)h * R));
  const float* row = in + ((size_t)p * N1 + r) * N2;
  float a = 0.f, d = 0.f;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const float v = row[(2 * k + t) % C];
    a = fmaf(kSym8[t], v, a);
    d = fmaf(sym8_g(t), v, d);
  }
  float* o = out + ((size_t)p * N1 + r) * N2;
  o[k] = a;
  o[h + k] = d;
}

// Forward level along the columns of the R x C corner: thread (p, k, c),
// k < R / 2 (consecutive threads take consecutive columns).
__global__ void k_dwt_cols(const float* __restrict__ in, float* __restrict__ out, int planes,
                           int N1, int N2, int R, int C) {
  const int h = R >> 1;
  const size_t n = (size_t)planes * h * C;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int c = (int)(idx % C);
  const int k = (int)((idx / C) % h);
  const int p = (int)(idx / ((size_t)C * h));
  const float* col = in + (size_t)p * N1 * N2 + c;
  float a = 0.f, d = 0.f;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const float v = col[(size_t)((2 * k + t) % R) * N2];
    a = fmaf(kSym8[t], v, a);
    d = fmaf(sym8_g(t), v, d);
  }
  float* o = out + (size_t)p * N1 * N2 + c;
  o[(size_t)k * N2] = a;
  o[(size_t)(h + k) * N2] = d;
}

// Inverse level along the rows: thread (p, r, m), m < C / 2, forms x[2m]
// and x[2m + 1] from a = in[0 .. C/2) and d = in[C/2 .. C).
__global__ void k_idwt_rows(const float* __restrict__ in, float* __restrict__ out, int planes,
                            int N1, int N2, int R, int C) {
  const int h = C >> 1;
  const size_t n = (size_t)planes * R * h;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int m = (int)(idx % h);
  const int r = (int)((idx / h) % R);
  const int p = (int)(idx / ((size_t)h * R));
  const float* row = in + ((size_t)p * N1 + r) * N2;
  float x0 = 0.f, x1 = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = ((m - j) % h + h) % h;
    const float a = row[k], d = row[h + k];
    x0 = fmaf(kSym8[2 * j], a, fmaf(sym8_g(2 * j), d, x0));
    x1 = fmaf(kSym8[2 * j + 1], a, fmaf(sym8_g(2 * j + 1), d, x1));
  }
  float* o = out + ((size_t)p * N1 + r) * N2;
  o[2 * m] = x0;
  o[2 * m + 1] = x1;
}

// Inverse level along the columns: thread (p, m, c), m < R / 2.
__global__ void k_idwt_cols(const float* __restrict__ in, float* __restrict__ out, int planes,
                            int N1, int N2, int R, int C) {
  const int h = R >> 1;
  const size_t n = (size_t)planes * h * C;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int c = (int)(idx % C);
  const int m = (int)((idx / C) % h);
  const int p = (int)(idx / ((size_t)C * h));
  const float* col = in + (size_t)p * N1 * N2 + c;
  float x0 = 0.f, x1 = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = ((m - j) % h + h) % h;
    const float a = col[(size_t)k * N2], d = col[(size_t)(h + k) * N2];
    x0 = fmaf(kSym8[2 * j], a, fmaf(sym8_g(2 * j), d, x0));
    x1 = fmaf(kSym8[2 * j + 1], a, fmaf(sym8_g(2 * j + 1), d, x1));
  }
  float* o = out + (size_t)p * N1 * N2 + c;
  o[(size_t)(2 * m) * N2] = x0;
  o[(size_t)(2 * m + 1) * N2] = x1;
}

// Band DCT, soft threshold and dual update at every coefficient position
// (S planes): c' = C_S c, v <- c' + clip(v) (v = 0 on the first
// iteration), w = t - u = 2 soft(v) - v, coef <- C_S^T w (in place).
// cs: C_S row-major (S x S); v: the state, [S][N1][N2].
template <int S>
__global__ void k_wdct_state(float* __restrict__ coef, float* __restrict__ v,
                             const float* __restrict__ cs, size_t plane, float kappa, int first) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  float c[S], w[S];
#pragma unroll
  for (int s = 0; s < S; ++s) c[s] = coef[s * plane + i];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) acc = fmaf(cs[k * S + s], c[s], acc);
    const float vo = first ? 0.f : v[k * plane + i];
    const float vn = acc + fminf(fmaxf(vo, -kappa), kappa);
    v[k * plane + i] = vn;
    const float t = vn > kappa ? vn - kappa : (vn < -kappa ? vn + kappa : 0.f);
    w[k] = 2.f * t - vn;
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < S; ++k) acc = fmaf(cs[k * S + s], w[k], acc);
    coef[s * plane + i] = acc;
  }
}

}  // namespace cip
