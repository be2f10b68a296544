// Residual and iterate-change norms for the adaptive penalty and the stopping
// rule of Section IV-C (Eq. paramS), analysis priors. A norm pass runs before
// the row pass of a checked iteration l, reads the column-pass output of that
// iteration (x^l) and the current state v (v-form: t^(l-1) = soft(v, k),
// u^(l-1) = clip(v, k), k = lambda / rho; zero before the first row pass) and
// accumulates, without writing any solver state,
//   sums[0] = sum (w - t^l)^2          (primal residual r^2, w = T x^l)
//   sums[1] = sum (t^l - t^(l-1))^2    (s^2 / rho^2)
//   sums[2] = sum (x^l - x^(l-1))^2    (when xprev is given)
//   sums[3] = sum (x^(l-1))^2
// with t^l = soft(w + u^(l-1), k). Each work-group writes its four partial
// sums to sums[4 b]; the host adds them in double precision. x^l is also
// written to xcur when given (the iterate the next check compares with). For
// the DCT prior the rows seen here are C1 x (column transform already
// applied), whose norms equal those of x (C1 orthonormal).
#pragma once
#include "kernels.hpp"

namespace cip {

constexpr int next_pow2(int n) { return n <= 1 ? 1 : 2 * next_pow2((n + 1) / 2); }

// Sum four per-thread values over the work-group (tree in LDS, fixed order);
// thread i < 4 writes total i to out[i]. red: 4 * NTP floats of free LDS,
// NTP a power of two >= blockDim.x. Starts with a barrier.
template <int NTP>
__device__ __forceinline__ void block_sum4(const float (&a)[4], float* red, float* __restrict__ out) {
  const int tid = threadIdx.x, n = blockDim.x;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) red[i * NTP + tid] = a[i];
  for (int j = tid + n; j < NTP; j += n)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[i * NTP + j] = 0.f;
  __syncthreads();
  for (int h = NTP / 2; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[i * NTP + tid] += red[i * NTP + tid + h];
    __syncthreads();
  }
  if (tid < 4) out[tid] = red[tid * NTP];
}

// Isotropic TV priors (T = I), after the t-update of iteration l: with
// t^l = f - u^l (f = x^l + u^(l-1), u^l the updated dual), the work-group of
// `count` consecutive values (RT rows of one plane) sums (x^l - t^l)^2,
// (t^l - t^(l-1))^2 (t^(l-1) = 0 when first), and (x^l - x^(l-1))^2 and
// (x^(l-1))^2 when xprev is given, to sums[4 b]; when keep, t^l replaces
// t^(l-1) in tprev (read first, element by element).
__global__ void __launch_bounds__(256)
k_itv_norm(const float* __restrict__ f, const float* __restrict__ u, const float* __restrict__ x,
           float* __restrict__ tprev, const float* __restrict__ xprev, int count, int first,
           int keep, float* __restrict__ sums) {
  __shared__ float red[4 * 256];
  const size_t base = (size_t)blockIdx.x * count;
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  for (int i = threadIdx.x; i < count; i += 256) {
    const size_t k = base + i;
    const float xv = x[k], tv = f[k] - u[k];
    const float tp = first ? 0.f : tprev[k];
    a[0] += (xv - tv) * (xv - tv);
    a[1] += (tv - tp) * (tv - tp);
    if (xprev) {
      const float pv = xprev[k];
      a[2] += (xv - pv) * (xv - pv);
      a[3] += pv * pv;
    }
    if (keep) tprev[k] = tv;
  }
  block_sum4<256>(a, red, sums + 4 * blockIdx.x);
}

// One constraint element: w = (T x)_i, p = current state value.
__device__ __forceinline__ void residual_terms(float w, float p, float kappa, float (&acc)[4]) {
  const float tp = soft_f(p, kappa);
  const float tn = soft_f(w + clip_f(p, kappa), kappa);
  acc[0] += (w - tn) * (w - tn);
  acc[1] += (tn - tp) * (tn - tp);
}

// DCT prior: same tiling as k_admm_row_dct (one work-group per plane and row
// tile, PAIRS row pairs).
template <int N2>
__global__ void __launch_bounds__(PAIRS * (N2 / ppt_row<N2>()))
k_norm_dct(const cx<float>* __restrict__ Yin, const float* __restrict__ vstate, int N1,
           const cx<float>* __restrict__ twg, const cx<float>* __restrict__ ewg, float kappa,
           int first, float* __restrict__ xcur, const float* __restrict__ xprev,
           float* __restrict__ sums) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  constexpr int NTP = next_pow2(PAIRS * T);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  cx<float>* ew = tw + N2;
  float* lds = reinterpret_cast<float*>(smem_raw) + 4 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int s = blockIdx.x / tiles, row0 = (blockIdx.x % tiles) * RT;
  const int ra = row0 + 2 * g;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  lds_load_table(tw, twg, N2);
  lds_load_table(ew, ewg, N2);
  tile_to_staging(Yin + rt_tile_base(s, row0, N1, H2), stg, H2 * RT);
  __syncthreads();
  cx<float> v[PPT];
  staging_to_pair<N2, PPT>(v, stg, g, t);
  __syncthreads();
  fft_group<N2, PPT, -1>(v, cb, t, tw);
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const size_t oa = ((size_t)s * N1 + ra) * N2, ob = oa + N2;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = t + T * q;
    const float xa = v[q].x, xb = v[q].y;
    if (xprev) {
      const float pa = xprev[oa + n], pb = xprev[ob + n];
      acc[2] += (xa - pa) * (xa - pa) + (xb - pb) * (xb - pb);
      acc[3] += pa * pa + pb * pb;
    }
    if (xcur) {
      xcur[oa + n] = xa;
      xcur[ob + n] = xb;
    }
  }
  dct_fwd_group<N2, PPT, false>(v, cb, t, tw, ew);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int k = t + T * q;
    residual_terms(v[q].x, first ? 0.f : vstate[oa + k], kappa, acc);
    residual_terms(v[q].y, first ? 0.f : vstate[ob + k], kappa, acc);
  }
  block_sum4<NTP>(acc, lds, sums + 4 * blockIdx.x);
}

// TV priors (BAND: TV3D): same tiling as the TV row passes; the band term of
// plane s needs x of plane s + 1, read from xall ([S][N1][N2], x of every
// plane from the same spectra, written by k_row_c2r before this pass).
template <int N2, bool BAND>
__global__ void __launch_bounds__((PAIRS + 1) * (N2 / ppt_row<N2>()))
k_norm_tv(const cx<float>* __restrict__ Yin, const float* __restrict__ vin, int S, int N1,
          const cx<float>* __restrict__ twg, float kappa, int first, float* __restrict__ xcur,
          const float* __restrict__ xprev, float* __restrict__ sums,
          const float* __restrict__ xall) {
  using G = TvGeo<N2>;
  constexpr int NTP = next_pow2((int)G::NT);
  constexpr int PERO = (RT * N2 + (int)G::NT - 1) / (int)G::NT;   // own elements per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / G::T, t = threadIdx.x % G::T;
  const int tiles = N1 / RT;
  const int s = blockIdx.x / tiles, row0 = (blockIdx.x % tiles) * RT;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  const unsigned plane = (unsigned)N1 * N2, cstride = (unsigned)S * plane;
  lds_load_table(tw, twg, N2);
  tv_stage_rows<N2>(Yin, stg, s, row0, N1);
  tv_inverse_rows<N2>(stg, cb, tw, lds, g, t);
  const float* X = lds;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float xo[PERO];
#pragma unroll
  for (int it = 0; it < PERO; ++it) {
    const unsigned e = threadIdx.x + it * G::NT;
    xo[it] = 0.f;
    if (e < (unsigned)(RT * N2)) {
      const unsigned lr = 1 + e / N2, n2 = e % N2;   // local row (0 = halo row above)
      const unsigned o = s * plane + (unsigned)(row0 - 1 + (int)lr) * N2 + n2;
      const float x0 = X[lr * N2 + n2];
      xo[it] = x0;
      if (xprev) {
        const float p = ld_off(xprev, o);
        acc[2] += (x0 - p) * (x0 - p);
        acc[3] += p * p;
      }
      if (xcur) st_off(xcur, o, x0);
      const float wv = X[(lr + 1) * N2 + n2] - x0;
      const float wh = X[lr * N2 + (n2 + 1 == N2 ? 0 : n2 + 1)] - x0;
      residual_terms(wv, first ? 0.f : ld_off(vin, o), kappa, acc);
      residual_terms(wh, first ? 0.f : ld_off(vin, cstride + o), kappa, acc);
    }
  }
  if (BAND && s + 1 < S) {
    const float* xn = xall + (size_t)(s + 1) * plane;
#pragma unroll
    for (int it = 0; it < PERO; ++it) {
      const unsigned e = threadIdx.x + it * G::NT;
      if (e < (unsigned)(RT * N2)) {
        const unsigned o = (unsigned)row0 * N2 + e;   // own element e of the tile
        const float wb = ld_off(xn, o) - xo[it];
        residual_terms(wb, first ? 0.f : ld_off(vin, 2 * cstride + s * plane + o), kappa, acc);
      }
    }
  }
  block_sum4<NTP>(acc, lds, sums + 4 * blockIdx.x);
}

// Iterate change of the stopping rule for solvers that hold x in space
// (synthesis priors): per work-group partial sums sums[2 b] = sum (x - xp)^2,
// sums[2 b + 1] = sum xp^2 (when have_prev), then xp = x. Grid-stride over n
// values, fixed summation order; 256 threads per work-group.
__global__ void __launch_bounds__(256)
k_xchange(const float* __restrict__ x, float* __restrict__ xp, float* __restrict__ sums, size_t n,
          int have_prev) {
  __shared__ float red[2][4];
  float a = 0.f, b = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float xv = x[i];
    if (have_prev) {
      const float pv = xp[i];
      a += (xv - pv) * (xv - pv);
      b += pv * pv;
    }
    xp[i] = xv;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    sums[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// out[0] = sum in[2 i], out[1] = sum in[2 i + 1] over i < npairs, in FP64 and
// a fixed order; one work-group of 256 threads.
__global__ void __launch_bounds__(256)
k_sum_pairs(const float* __restrict__ in, size_t npairs, double* __restrict__ out) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (size_t i = threadIdx.x; i < npairs; i += 256) {
    a += (double)in[2 * i];
    b += (double)in[2 * i + 1];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    out[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// State of a threshold split re-expressed for a new penalty (v-form, as in
// the analysis row passes): t = soft(v, kappa) stays, the scaled dual
// u = clip(v, kappa) becomes sc u with sc = rho / rho'; v' = t + sc u.
__global__ void k_rescale_state(float* __restrict__ v, size_t n, float kappa, float sc) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float vv = v[i];
    v[i] = soft_f(vv, kappa) + sc * clip_f(vv, kappa);
  }
}

}  // namespace cip
