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
// One launch per level does both axes through an LDS tile. The detail
// bands go to the coefficient buffer and the low-low band of a level to one
// of two staging areas (quadrants of a staging buffer), which the next level
// reads; the inverse mirrors this. The band DCT, the soft threshold and the
// dual update (v-form state, as in the other analysis priors) are one
// pointwise kernel over the coefficients.
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

// i mod n for i in [-n, n + 78) without an integer division (levels whose
// side is below a tile's reach wrap several times)
__device__ __forceinline__ int wrap_idx(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

// i mod n; `once` (uniform) states that i lies in [-n, 2n), where one
// conditional correction is enough
__device__ __forceinline__ int wrap_fast(int i, int n, bool once) {
  if (once) return i < 0 ? i + n : (i >= n ? i - n : i);
  return wrap_idx(i, n);
}

// One forward level on the R x C corner (both axes fused through LDS). A
// work-group produces the coefficients k1 in [K1, K1 + T), k2 in
// [K2, K2 + T) of the four bands of one plane from the (2T + 14)^2 input
// samples they read (indices mod R and mod C): the transform along the rows
// first (a | d along the columns), then along the columns (a ; d along the
// rows). The low-low band goes to ll (another buffer, or the coefficient
// corner at the last level), the three others to coef. src and ll have the
// coefficient array's layout (leading dimension N2, plane stride N1 N2).
// DWT_T output coefficients per tile and axis (32, or 16 on the small
// levels, whose grids would otherwise not fill the GPU); DWT_IN input
// samples per tile and axis.
template <int DWT_T>
__global__ void __launch_bounds__(256)
k_dwt2(const float* __restrict__ src, float* __restrict__ ll, float* __restrict__ coef, int N1,
       int N2, int R, int C) {
  constexpr int DWT_IN = 2 * DWT_T + 14;
  __shared__ float X[DWT_IN][DWT_IN + 1];
  __shared__ float RA[DWT_IN][DWT_T + 1], RD[DWT_IN][DWT_T + 1];
  const int h1 = R >> 1, h2 = C >> 1;
  const int K1 = blockIdx.y * DWT_T, K2 = blockIdx.x * DWT_T;
  const size_t po = (size_t)blockIdx.z * N1 * N2;
  const float* in = src + po;
  // thread (ph, v) loads column v of the input tile, rows ph, ph + LP, ...
  // (the column index is wrapped once, rows by one correction where the
  // level is at least a tile's reach); every load is issued, at a clamped
  // valid position, before the LDS stores, which skip the clamped ones
  constexpr int LP = 256 / DWT_IN, NJ = (DWT_IN + LP - 1) / LP;
  const int ph = threadIdx.x / DWT_IN, v = threadIdx.x % DWT_IN;
  const bool act = ph < LP;
  const int phc = act ? ph : LP - 1;
  const bool once = R >= DWT_IN && C >= DWT_IN;
  const int gc = wrap_fast(2 * K2 + v, C, once);
  float val[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int u = min(phc + LP * j, DWT_IN - 1);
    const int gr = wrap_fast(2 * K1 + u, R, once);
    val[j] = in[(unsigned)gr * (unsigned)N2 + (unsigned)gc];
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int u = ph + LP * j;
    if (act && u < DWT_IN) X[u][v] = val[j];
  }
  __syncthreads();
  // along the rows: outputs k = 2j, 2j + 1 of row u from one window of 18
  // samples (consecutive lanes take consecutive rows: odd LDS pitch)
  for (int e = threadIdx.x; e < DWT_IN * (DWT_T / 2); e += 256) {
    const int u = e % DWT_IN, j = e / DWT_IN;
    float w[18];
#pragma unroll
    for (int t = 0; t < 18; ++t) w[t] = X[u][4 * j + t];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      float a = 0.f, d = 0.f;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        a = fmaf(kSym8[t], w[2 * o + t], a);
        d = fmaf(sym8_g(t), w[2 * o + t], d);
      }
      RA[u][2 * j + o] = a;
      RD[u][2 * j + o] = d;
    }
  }
  __syncthreads();
  // along the columns: outputs i = 2m, 2m + 1 of column k from one window of
  // 18 rows of RA and RD
  for (int e = threadIdx.x; e < (DWT_T / 2) * DWT_T; e += 256) {
    const int m = e / DWT_T, k = e % DWT_T;
    const int k2 = K2 + k;
    float ra[18], rd[18];
#pragma unroll
    for (int t = 0; t < 18; ++t) {
      ra[t] = RA[4 * m + t][k];
      rd[t] = RD[4 * m + t][k];
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const int k1 = K1 + 2 * m + o;
      float aa = 0.f, ad = 0.f, da = 0.f, dd = 0.f;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        aa = fmaf(kSym8[t], ra[2 * o + t], aa);
        ad = fmaf(kSym8[t], rd[2 * o + t], ad);
        da = fmaf(sym8_g(t), ra[2 * o + t], da);
        dd = fmaf(sym8_g(t), rd[2 * o + t], dd);
      }
      if (k1 < h1 && k2 < h2) {
        ll[po + (size_t)k1 * N2 + k2] = aa;
        coef[po + (size_t)k1 * N2 + h2 + k2] = ad;
        coef[po + (size_t)(h1 + k1) * N2 + k2] = da;
        coef[po + (size_t)(h1 + k1) * N2 + h2 + k2] = dd;
      }
    }
  }
}

// One inverse level: the R x C corner from its four bands (low-low at ll,
// the others in coef), written to dst. A work-group produces the samples
// 2 m + e, m in [M, M + T) along both axes, from the band coefficients
// (m - j) mod (R/2, C/2), j < 8 (T + 7 per axis): inverse along the rows
// first, then along the columns.
template <int DWT_T>
__global__ void __launch_bounds__(256)
k_idwt2(const float* __restrict__ ll, const float* __restrict__ coef, float* __restrict__ dst,
        int N1, int N2, int R, int C) {
  constexpr int IDWT_IN = DWT_T + 7;
  __shared__ float B[4][IDWT_IN][IDWT_IN + 1];
  __shared__ float YL[IDWT_IN][2 * DWT_T + 1], YH[IDWT_IN][2 * DWT_T + 1];
  const int h1 = R >> 1, h2 = C >> 1;
  const int M1 = blockIdx.y * DWT_T, M2 = blockIdx.x * DWT_T;
  const size_t po = (size_t)blockIdx.z * N1 * N2;
  // band b: 0 low-low, 1 low rows / high columns, 2 high rows / low columns, 3 high-high
  // The four bands' tiles are one array of 4 IDWT_IN rows (band-rows br =
  // b IDWT_IN + u); thread (ph, v) loads column v of band-rows ph, ph + LP,
  // ... As in the forward level, every load is issued at a clamped valid
  // position before the LDS stores.
  constexpr int NBR = 4 * IDWT_IN, LP = 256 / IDWT_IN, NJ = (NBR + LP - 1) / LP;
  const int ph = threadIdx.x / IDWT_IN, v = threadIdx.x % IDWT_IN;
  const bool act = ph < LP;
  const int phc = act ? ph : LP - 1;
  const bool once = h1 >= IDWT_IN && h2 >= IDWT_IN;
  const int k2 = wrap_fast(M2 - 7 + v, h2, once);
  const float* llp = ll + po;
  const float* cfp = coef + po;
  float val[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int br = min(phc + LP * j, NBR - 1);
    const int b = br / IDWT_IN, u = br % IDWT_IN;
    const int k1 = wrap_fast(M1 - 7 + u, h1, once);
    const unsigned off = (unsigned)(k1 + (b >> 1) * h1) * (unsigned)N2 + (unsigned)(k2 + (b & 1) * h2);
    val[j] = (b == 0 ? llp : cfp)[off];
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int br = ph + LP * j;
    if (act && br < NBR) B[br / IDWT_IN][br % IDWT_IN][v] = val[j];
  }
  __syncthreads();
  // along the rows: Y[u][2 m + e] for the low and the high row families
  for (int e = threadIdx.x; e < IDWT_IN * DWT_T; e += 256) {
    const int u = e / DWT_T, m = e % DWT_T;
    float l0 = 0.f, l1 = 0.f, g0 = 0.f, g1 = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int v = m - j + 7;
      const float a = B[0][u][v], d = B[1][u][v], a2 = B[2][u][v], d2 = B[3][u][v];
      l0 = fmaf(kSym8[2 * j], a, fmaf(sym8_g(2 * j), d, l0));
      l1 = fmaf(kSym8[2 * j + 1], a, fmaf(sym8_g(2 * j + 1), d, l1));
      g0 = fmaf(kSym8[2 * j], a2, fmaf(sym8_g(2 * j), d2, g0));
      g1 = fmaf(kSym8[2 * j + 1], a2, fmaf(sym8_g(2 * j + 1), d2, g1));
    }
    YL[u][2 * m] = l0;
    YL[u][2 * m + 1] = l1;
    YH[u][2 * m] = g0;
    YH[u][2 * m + 1] = g1;
  }
  __syncthreads();
  // along the columns: out[2 m + e][n]
  float* out = dst + po;
  for (int e = threadIdx.x; e < DWT_T * 2 * DWT_T; e += 256) {
    const int m = e / (2 * DWT_T), n = e % (2 * DWT_T);
    if (M1 + m >= h1 || M2 + (n >> 1) >= h2) continue;
    float x0 = 0.f, x1 = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int u = m - j + 7;
      const float a = YL[u][n], d = YH[u][n];
      x0 = fmaf(kSym8[2 * j], a, fmaf(sym8_g(2 * j), d, x0));
      x1 = fmaf(kSym8[2 * j + 1], a, fmaf(sym8_g(2 * j + 1), d, x1));
    }
    const size_t col = (size_t)2 * M2 + n;
    out[(size_t)(2 * (M1 + m)) * N2 + col] = x0;
    out[(size_t)(2 * (M1 + m) + 1) * N2 + col] = x1;
  }
}

// Band DCT, soft threshold and dual update at every coefficient position
// (S planes): c' = C_S c, v <- c' + clip(v) (v = 0 on the first
// iteration), w = t - u = 2 soft(v) - v, coef <- C_S^T w (in place).
// cs: C_S row-major (S x S); v: the state, [S][N1][N2]. When rs is given
// (adaptive penalty, Section IV-C) every work-group of 256 positions writes
//   rs[2 b] = sum (c' - t)^2 = sum (clip(v_new) - clip(v_old))^2 and
//   rs[2 b + 1] = sum (t - t_prev)^2 = sum (soft(v_new) - soft(v_old))^2
// (v_old = 0 on the first iteration), summed in a fixed order.
template <int S>
__global__ void __launch_bounds__(256)
k_wdct_state(float* __restrict__ coef, float* __restrict__ v, const float* __restrict__ cs,
             size_t plane, float kappa, int first, float* __restrict__ rs) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  float r2 = 0.f, s2 = 0.f;
  if (i < plane) {
    float c[S], w[S], vp[S];
    // every load before the first store of the state (the planes of v are
    // not known to be distinct to the compiler)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      c[s] = coef[s * plane + i];
      vp[s] = first ? 0.f : v[s * plane + i];
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      float acc = 0.f;
#pragma unroll
      for (int s = 0; s < S; ++s) acc = fmaf(cs[k * S + s], c[s], acc);
      const float vo = vp[k];
      const float vn = acc + fminf(fmaxf(vo, -kappa), kappa);
      v[k * plane + i] = vn;
      const float t = vn > kappa ? vn - kappa : (vn < -kappa ? vn + kappa : 0.f);
      w[k] = 2.f * t - vn;
      if (rs) {
        const float to = vo > kappa ? vo - kappa : (vo < -kappa ? vo + kappa : 0.f);
        const float d = fminf(fmaxf(vn, -kappa), kappa) - fminf(fmaxf(vo, -kappa), kappa);
        r2 += d * d;
        s2 += (t - to) * (t - to);
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < S; ++k) acc = fmaf(cs[k * S + s], w[k], acc);
      coef[s * plane + i] = acc;
    }
  }
  if (rs) {
    __shared__ float red[2][4];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      r2 += __shfl_xor(r2, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = r2;
      red[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      rs[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      rs[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
  }
}

// After a penalty change (adaptive solve): with t = soft(v, kappa),
// u = clip(v, kappa) of the updated state, v <- t + sc u (sc = rho / rho',
// the v-form for kappa' = lambda / rho') and coef <- C_S^T (t - sc u), the
// input of the inverse transform for the next x-update.
template <int S>
__global__ void __launch_bounds__(256)
k_wdct_emit(float* __restrict__ coef, float* __restrict__ v, const float* __restrict__ cs,
            size_t plane, float kappa, float sc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  float w[S], vp[S];
#pragma unroll
  for (int k = 0; k < S; ++k) vp[k] = v[k * plane + i];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float vo = vp[k];
    const float t = vo > kappa ? vo - kappa : (vo < -kappa ? vo + kappa : 0.f);
    const float u = sc * fminf(fmaxf(vo, -kappa), kappa);
    v[k * plane + i] = t + u;
    w[k] = t - u;
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
