// Device kernels of the ADMM hot path (Section IV of Dogan & Oktem).
//
// Data layouts in HBM (complex values are interleaved re/im):
//   real planes      [P][N1][N2]                  (x, y, kernels, ADMM state)
//   row-spectrum RT  [P][N1/RT][H2][RT] complex   (H2 = N2/2 + 1): output of a
//                    row pass (real-to-complex along N2); a tile of RT rows is
//                    contiguous, so a row pass reads/writes whole tiles and a
//                    column pass reads RT consecutive rows of one column at a
//                    time.
//   spectrum FL      [E][H2][N1] complex          per-frequency tables, one
//                    column (fixed k2) contiguous over k1.
// Transforms are unnormalised in both directions; 1/(N1 N2) is folded into
// the per-frequency tables.
#pragma once
#include "fft.hpp"

namespace cip {

constexpr int RT = 8;          // rows per row tile
constexpr int PAIRS = RT / 2;  // row pairs per row-pass work-group

// Points per thread of the length-N transforms in row passes and column
// passes (a group of N / PPT threads carries one transform).
#ifndef CIP_PPT_ROW_1024
#define CIP_PPT_ROW_1024 16
#endif
#ifndef CIP_PPT_COL_1024
#define CIP_PPT_COL_1024 16
#endif
// Lengths with a factor 3 (3 * 2^k) use 12 points per thread, so that the
// radix-3 butterfly lies in the first, in-register stage; the later stages
// then use radices 4 and 2 (divisors of 12).
constexpr int ppt_default(int N) { return N % 3 == 0 ? 12 : (N >= 16 ? 16 : N); }
constexpr int ppt_row_n(int N) { return N == 1024 ? CIP_PPT_ROW_1024 : ppt_default(N); }
constexpr int ppt_col_n(int N) { return N == 1024 ? CIP_PPT_COL_1024 : ppt_default(N); }
template <int N> constexpr int ppt_row() { return ppt_row_n(N); }
template <int N> constexpr int ppt_col() { return ppt_col_n(N); }

__device__ __forceinline__ size_t rt_tile_base(int p, int n1, int N1, int H2) {
  return (((size_t)p * (N1 / RT) + (n1 / RT)) * H2) * RT;
}
__device__ __forceinline__ size_t rt_idx(int p, int n1, int k2, int N1, int H2) {
  return rt_tile_base(p, n1, N1, H2) + (size_t)k2 * RT + (n1 % RT);
}
__device__ __forceinline__ size_t fl_idx(int e, int k1, int k2, int N1, int H2) {
  return ((size_t)e * H2 + k2) * N1 + k1;
}

// Work-group index remap so that consecutive logical indices run on the same
// XCD: the hardware deals work-groups round-robin over the 8 XCDs, each with
// its own L2, while neighbouring columns / row tiles share cache lines.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  constexpr int NX = 8;
  const int per = (n + NX - 1) / NX;
  const int tall = n % NX == 0 ? NX : n % NX;
  const int x = b % NX, i = b / NX;
  return x < tall ? x * per + i : tall * per + (x - tall) * (per - 1) + i;
}

// Complex LDS arrays are interleaved (one 8- or 16-byte access per value)
// and padded with pad().
template <typename Re> __device__ __forceinline__ cx<Re> ldc(const cx<Re>* b, int i) {
  return b[pad(i)];
}
template <typename Re> __device__ __forceinline__ void stc(cx<Re>* b, int i, cx<Re> v) {
  b[pad(i)] = v;
}

// ---------------------------------------------------------------- LDS helpers
// Padding for the row-tile staging arrays ([k2][RT] order, stride RT floats).
__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }
constexpr int pad8_len(int n) { return n + (n >> 3) + 1; }

// Global -> LDS copies of the whole work-group with U loads of every thread
// in flight before their LDS stores (a plain strided loop waits for each
// load in turn): idx(i) gives the source and staging index of element i.
template <int U, typename T, typename Src, typename Dst>
__device__ __forceinline__ void batched_to_lds(int n, Src src, Dst dst) {
  const int step = blockDim.x;
  int i = threadIdx.x;
  for (; i + (U - 1) * step < n; i += U * step) {
    T r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = src(i + u * step);
#pragma unroll
    for (int u = 0; u < U; ++u) dst(i + u * step, r[u]);
  }
  for (; i < n; i += step) dst(i, src(i));
}

// Copy n complex values from global memory into LDS (whole work-group).
template <typename Re>
__device__ __forceinline__ void lds_load_table(cx<Re>* dst, const cx<Re>* __restrict__ src, int n) {
  batched_to_lds<4, cx<Re>>(
      n, [&](int i) { return src[i]; }, [&](int i, const cx<Re>& v) { dst[i] = v; });
}

// Floats of LDS used by a row-pass work-group of NG row pairs (staging holds
// the work-group's 2 NG rows of the tile).
template <int N2, typename Re> constexpr int row_work_floats(int ng, bool staged) {
  int fft = ng * 2 * padded_len(N2);
  int stg = staged ? 2 * pad8_len((N2 / 2 + 1) * 2 * ng) : 0;
  return fft > stg ? fft : stg;
}

// Load one RT row tile (H2 x RT complex, contiguous) into the padded staging
// array (complex, padded with pad8).
__device__ __forceinline__ void tile_to_staging(const cx<float>* __restrict__ src, cx<float>* stg,
                                                int n) {
  batched_to_lds<8, cx<float>>(
      n, [&](int i) { return src[i]; }, [&](int i, const cx<float>& v) { stg[pad8(i)] = v; });
}
__device__ __forceinline__ void staging_to_tile(cx<float>* __restrict__ dst, const cx<float>* stg,
                                                int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = stg[pad8(i)];
}

// Part of a tile: rows r0 .. r0 + SW - 1 of each of the H2 columns
// (staging [k2][SW]); with SW = RT these are the plain tile copies above.
template <int SW>
__device__ __forceinline__ void subtile_to_staging(const cx<float>* __restrict__ tile, cx<float>* stg,
                                                   int h2, int r0) {
  batched_to_lds<8, cx<float>>(
      h2 * SW, [&](int i) { return tile[(i / SW) * RT + r0 + i % SW]; },
      [&](int i, const cx<float>& v) { stg[pad8(i)] = v; });
}
template <int SW>
__device__ __forceinline__ void staging_to_subtile(cx<float>* __restrict__ tile, const cx<float>* stg,
                                                   int h2, int r0) {
  for (int i = threadIdx.x; i < h2 * SW; i += blockDim.x)
    tile[(i / SW) * RT + r0 + i % SW] = stg[pad8(i)];
}

// From the staged half spectra of rows a = 2g, b = 2g + 1 of the tile, build
// the full spectrum Z[k] = A[k] + i B[k] (Hermitian extension of A and B), in
// the group register order (slot q holds k = t + T q).
template <int N2, int PPT, int SW = RT>
__device__ __forceinline__ void staging_to_pair(cx<float>* v, const cx<float>* stg, int g,
                                                int t) {
  constexpr int T = N2 / PPT;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = k <= N2 / 2 ? k : N2 - k;
    float sg = k <= N2 / 2 ? 1.f : -1.f;
    int i = kk * SW + 2 * g;
    cx<float> A = stg[pad8(i)], B = stg[pad8(i + 1)];
    A.y *= sg;
    B.y *= sg;
    v[q] = cx<float>{A.x - B.y, A.y + B.x};
  }
}

// Split the spectrum Z of a packed pair (z = a + i b) into the half spectra
// A[k] = (Z[k] + conj Z[N-k]) / 2, B[k] = (Z[k] - conj Z[N-k]) / 2i,
// k = 0..N/2, and write them to the staging arrays as rows 2g, 2g + 1. `v`
// holds Z in group register order on entry. The group scratch cb may
// alias the staging arrays.
template <int N2, int PPT, int SW = RT, bool WS = false>
__device__ __forceinline__ void pair_to_staging(cx<float>* v, cx<float>* cb, cx<float>* stg, int g,
                                                int t) {
  constexpr int T = N2 / PPT;
  constexpr int QH = (N2 / 2) / T + 1;   // slots that can hold k <= N/2
  // (called right after fft_group, which ends with a barrier)
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
  group_sync<T, WS>();
  cx<float> A[QH], B[QH];
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    int k = t + T * q;
    if (k <= N2 / 2) {
      cx<float> Z = ldc(cb, k);
      cx<float> Zc = conjx(ldc(cb, k == 0 ? 0 : N2 - k));
      cx<float> s = Z + Zc, d = Z - Zc;
      A[q] = cx<float>{0.5f * s.x, 0.5f * s.y};
      B[q] = cx<float>{0.5f * d.y, -0.5f * d.x};
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    int k = t + T * q;
    if (k <= N2 / 2) {
      int i = k * SW + 2 * g;
      stg[pad8(i)] = A[q];
      stg[pad8(i + 1)] = B[q];
    }
  }
}

// ---------------------------------------------------------------- DCT via FFT
// Orthonormal DCT-II of a complex sequence (real and imaginary parts
// transformed independently), computed with one N-point FFT of the
// even/odd-reordered sequence and a post-twiddle (Makhoul's method):
//   X[k] = a_k Re(E[k] Va[k]) + i a_k Re(E[k] Vb[k]),  E[k] = exp(-i pi k / 2N),
//   a_0 = sqrt(1/N), a_k = sqrt(2/N), Va / Vb the spectra of the reordered
//   real / imaginary parts (separated from one complex FFT).
// `ew` is the LDS table E[0..N).
// LEAD: synchronise before the first LDS write (not needed right after
// fft_group, which ends with a barrier after its last LDS read).
template <int N, int PPT, bool LEAD = true, bool WS = false>
__device__ __forceinline__ void dct_fwd_group(cx<float>* reg, cx<float>* cb, int t,
                                              const cx<float>* tw, const cx<float>* ew) {
  constexpr int T = N / PPT;
  const float a0 = __builtin_sqrtf(1.0f / N), a1 = __builtin_sqrtf(2.0f / N);
  if constexpr (LEAD) group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int n = t + T * q;
    int p = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
    stc(cb, p, reg[q]);
  }
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) reg[q] = ldc(cb, t + T * q);
  fft_group<N, PPT, +1, float, WS>(reg, cb, t, tw);
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, reg[q]);
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = k == 0 ? 0 : N - k;
    cx<float> V = ldc(cb, k);
    cx<float> Vc = conjx(ldc(cb, kk));
    cx<float> s = V + Vc, d = V - Vc;
    // Va = s / 2, Vb = d / 2i = (d.y, -d.x) / 2; fold the 1/2 into alpha
    cx<float> e = ew[k];
    float al = 0.5f * (k == 0 ? a0 : a1);
    reg[q] = cx<float>{al * (e.x * s.x - e.y * s.y), al * (e.x * d.y + e.y * d.x)};
  }
}

// Inverse (DCT-III, orthonormal) of a complex coefficient sequence Y:
//   V[k] = conj(E[k]) / N * (Y[k] / a_k - i Y[N-k] / a_{N-k}),  V[0] = Y[0] / (N a_0),
// then an inverse FFT and the inverse even/odd reordering.
template <int N, int PPT, bool LEAD = true, bool WS = false>
__device__ __forceinline__ void dct_inv_group(cx<float>* reg, cx<float>* cb, int t,
                                              const cx<float>* tw, const cx<float>* ew) {
  constexpr int T = N / PPT;
  const float ia0 = __builtin_sqrtf((float)N) / N, ia1 = __builtin_sqrtf(0.5f * N) / N;
  if constexpr (LEAD) group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, reg[q]);
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    cx<float> Yk = ldc(cb, k);
    cx<float> a;
    if (k == 0) {
      a = cx<float>{Yk.x * ia0, Yk.y * ia0};
    } else {
      cx<float> Yn = ldc(cb, N - k);
      a = cx<float>{(Yk.x + Yn.y) * ia1, (Yk.y - Yn.x) * ia1};   // Yk - i Yn
    }
    cx<float> e = ew[k];
    reg[q] = cmulc(a, e);   // a * conj(E[k])
  }
  fft_group<N, PPT, -1, float, WS>(reg, cb, t, tw);
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int m = t + T * q;
    int pos = (m < N / 2) ? 2 * m : 2 * N - 2 * m - 1;
    stc(cb, pos, reg[q]);
  }
  group_sync<T, WS>();
#pragma unroll
  for (int q = 0; q < PPT; ++q) reg[q] = ldc(cb, t + T * q);
}


// ---------------------------------------------------------------- row passes
// Two real rows a, b are carried by one complex FFT (z = a + i b). LDS layout
// of every row kernel: [twiddles N2 complex][work region].

// Real-to-complex FFT of every row: in [P][N1][N2] -> out RT [P][N1/RT][H2][RT].
// STAGED (float): one work-group per (plane, row tile), coalesced tile store.
// Otherwise (double, plan time): one work-group per (plane, row pair).
template <int N2, typename Re, bool STAGED>
__global__ void k_row_r2c(const Re* __restrict__ in, cx<Re>* __restrict__ out, int N1,
                          const cx<Re>* __restrict__ twg) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<Re>* tw = reinterpret_cast<cx<Re>*>(smem_raw);
  Re* lds = reinterpret_cast<Re*>(smem_raw) + 2 * N2;
  lds_load_table(tw, twg, N2);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  int p, row0;
  if (STAGED) {
    const int tiles = N1 / RT;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    p = b / tiles;
    row0 = (b % tiles) * RT;
  } else {
    const int pairs = N1 / 2;
    p = blockIdx.x / pairs;
    row0 = (blockIdx.x % pairs) * 2;
  }
  const int ra = row0 + 2 * g;
  cx<Re>* cb = reinterpret_cast<cx<Re>*>(lds) + g * padded_len(N2);
  const Re* xa = in + ((size_t)p * N1 + ra) * N2;
  const Re* xb = xa + N2;
  cx<Re> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int n = t + T * q;
    v[q] = cx<Re>{xa[n], xb[n]};
  }
  __syncthreads();   // twiddle table ready
  fft_group<N2, PPT, +1>(v, cb, t, tw);
  if constexpr (STAGED) {
    cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
    pair_to_staging<N2, PPT>(v, cb, stg, g, t);
    __syncthreads();
    staging_to_tile(out + rt_tile_base(p, row0, N1, H2), stg, H2 * RT);
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
    group_sync<T>();
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int k = t + T * q;
      if (k <= N2 / 2) {
        cx<Re> Z = ldc(cb, k);
        cx<Re> Zc = conjx(ldc(cb, k == 0 ? 0 : N2 - k));
        cx<Re> s = Z + Zc, d = Z - Zc;
        out[rt_idx(p, ra, k, N1, H2)] = cx<Re>{Re(0.5) * s.x, Re(0.5) * s.y};
        out[rt_idx(p, ra + 1, k, N1, H2)] = cx<Re>{Re(0.5) * d.y, Re(-0.5) * d.x};
      }
    }
  }
}

// Complex-to-real inverse FFT of every row: RT [P][..] -> out [P][N1][N2],
// scaled by `scale`. One work-group per (plane, row tile).
template <int N2>
__global__ void k_row_c2r(const cx<float>* __restrict__ in, float* __restrict__ out, int N1,
                          float scale, const cx<float>* __restrict__ twg) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int p = b / tiles, row0 = (b % tiles) * RT;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  lds_load_table(tw, twg, N2);
  tile_to_staging(in + rt_tile_base(p, row0, N1, H2), stg, H2 * RT);
  __syncthreads();
  cx<float> v[PPT];
  staging_to_pair<N2, PPT>(v, stg, g, t);
  __syncthreads();   // staging aliases the group scratch
  fft_group<N2, PPT, -1>(v, cb, t, tw);
  float* xa = out + ((size_t)p * N1 + row0 + 2 * g) * N2;
  float* xb = xa + N2;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int n = t + T * q;
    xa[n] = v[q].x * scale;
    xb[n] = v[q].y * scale;
  }
}

// ---------------------------------------------------------------- column passes
enum ColOp { OP_FWD = 0, OP_ADJ = 1, OP_XHAT0 = 2, OP_SPEC = 3 };

// Column FFT of Pin planes of a row spectrum (one work-group per column k2),
// a per-frequency linear map Pin -> Pout, then either an inverse column FFT
// to an RT output (OP_FWD, OP_ADJ) or a store to an FL table (OP_XHAT0,
// OP_SPEC).
//   OP_FWD  : out_k = sum_s Lam[k][s] in_s              (Lam FL [K*S])
//   OP_ADJ  : out_s = sum_k conj(Lam[k][s]) in_k
//   OP_XHAT0: out_s = sum_k M[s][k] in_k                 (M FL [S*K])
//   OP_SPEC : out_0 = in_0, stored at FL plane `spec_plane`
// LDS: [twiddles N1 complex][PM planes x 2 x padded N1].
template <int N1, typename Re, int OP>
__global__ void k_col_op(const cx<Re>* __restrict__ in, void* __restrict__ outv, int Pin, int Pout,
                         int H2, const cx<Re>* __restrict__ twg, const cx<Re>* __restrict__ mat,
                         int spec_plane) {
  constexpr int PPT = ppt_col<N1>();
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<Re>* tw = reinterpret_cast<cx<Re>*>(smem_raw);
  Re* lds = reinterpret_cast<Re*>(smem_raw) + 2 * N1;
  const int k2 = xcd_remap(blockIdx.x, gridDim.x);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  cx<Re>* cb = reinterpret_cast<cx<Re>*>(lds) + g * PL;
  lds_load_table(tw, twg, N1);
  cx<Re> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q)
    v[q] = g < Pin ? in[rt_idx(g, t + T * q, k2, N1, H2)] : cx<Re>{Re(0), Re(0)};
  __syncthreads();
  fft_group<N1, PPT, +1>(v, cb, t, tw);
  const size_t F = (size_t)N1 * H2;
  if constexpr (OP == OP_SPEC) {
    cx<Re>* out = reinterpret_cast<cx<Re>*>(outv);
    if (g == 0) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) out[fl_idx(spec_plane, t + T * q, k2, N1, H2)] = v[q];
    }
    return;
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
    __syncthreads();
    // per-frequency map; each thread owns whole frequencies (the plane loops
    // run to the static maximum of 8 with guards, so that xin stays in
    // registers)
    for (int k1 = threadIdx.x; k1 < N1; k1 += blockDim.x) {
      cx<Re> xin[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        xin[j] = j < Pin ? ldc(reinterpret_cast<const cx<Re>*>(lds) + j * PL, k1)
                         : cx<Re>{Re(0), Re(0)};
      const size_t f = (size_t)k2 * N1 + k1;
      for (int o = 0; o < Pout; ++o) {
        cx<Re> acc = {Re(0), Re(0)};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j >= Pin) break;
          cx<Re> m;
          if (OP == OP_ADJ) m = conjx(mat[(size_t)(j * Pout + o) * F + f]);
          else m = mat[(size_t)(o * Pin + j) * F + f];
          acc = acc + cmul(m, xin[j]);
        }
        if (OP == OP_XHAT0) {
          reinterpret_cast<cx<Re>*>(outv)[(size_t)o * F + f] = acc;
        } else {
          stc(reinterpret_cast<cx<Re>*>(lds) + o * PL, k1, acc);
        }
      }
    }
    if constexpr (OP == OP_XHAT0) return;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) v[q] = ldc(cb, t + T * q);
    fft_group<N1, PPT, -1>(v, cb, t, tw);
    cx<Re>* out = reinterpret_cast<cx<Re>*>(outv);
    if (g < Pout) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) out[rt_idx(g, t + T * q, k2, N1, H2)] = v[q];
    }
  }
}

// ---------------------------------------------------------------- ADMM state
// State per constraint component: v = T x^l + u^{l-1}. From v the pair (t, u)
// of Algorithm 1 is t = soft(v, kappa), u = clip(v, kappa) (kappa = lambda /
// rho), so t - u = 2 soft(v) - v and the next v = T x^{l+1} + clip(v).
__device__ __forceinline__ float soft_f(float v, float k) {
  return v > k ? v - k : (v < -k ? v + k : 0.f);
}
__device__ __forceinline__ float clip_f(float v, float k) { return fminf(fmaxf(v, -k), k); }

enum RowMode { ROW_FIRST = 0, ROW_FULL = 1, ROW_FINAL = 2 };

// Row pass of one ADMM iteration (DCT prior), one work-group per (plane, NP
// row pairs of a row tile), PPT_ points per thread in the row transforms (the
// twiddle table must be the one built for PPT_): inverse row FFT of the column-pass output (x^l in the column-DCT /
// row-frequency domain) -> row DCT gives w = T x^l -> prox + dual update of v
// -> inverse row DCT of t - u -> forward row FFT -> RT output for the next
// column pass. ROW_FINAL stops after the inverse row FFT and writes x.
// LDS: [twiddles N2][DCT table E N2][work region].
template <int N2, int NP, int PPT_ = ppt_row<N2>()>
__global__ void __launch_bounds__(NP * (N2 / PPT_), 2)
k_admm_row_dct(const cx<float>* __restrict__ Yin, cx<float>* __restrict__ Gout,
               float* __restrict__ vstate, int N1, const cx<float>* __restrict__ twg,
               const cx<float>* __restrict__ ewg, float kappa, int mode,
               float* __restrict__ xout, float sc) {
  constexpr int PPT = PPT_;
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  constexpr int SW = 2 * NP;         // tile rows of this work-group
  constexpr int PARTS = RT / SW;     // work-groups per tile
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  cx<float>* ew = tw + N2;
  float* lds = reinterpret_cast<float*>(smem_raw) + 4 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int s = b / (tiles * PARTS), rem = b % (tiles * PARTS);
  const int row0 = (rem / PARTS) * RT, r0 = (rem % PARTS) * SW;
  const int ra = row0 + r0 + 2 * g;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  // Every global load of the prologue is issued before the first LDS store:
  // the twiddle and DCT tables, the rows of the tile, and the state of rows
  // a, b (its latency also overlaps the two transforms below).
  constexpr int NT = NP * T;                          // threads
  constexpr int NTAB = (N2 + NT - 1) / NT;            // table values per thread
  constexpr int NSTG = (H2 * SW + NT - 1) / NT;       // tile values per thread
  const cx<float>* tile = Yin + rt_tile_base(s, row0, N1, H2);
  cx<float> rtw[NTAB], rew[NTAB], rst[NSTG];
#pragma unroll
  for (int k = 0; k < NTAB; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < N2) {
      rtw[k] = twg[i];
      if (mode != ROW_FINAL) rew[k] = ewg[i];
    }
  }
#pragma unroll
  for (int k = 0; k < NSTG; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < H2 * SW) rst[k] = tile[(i / SW) * RT + r0 + i % SW];
  }
  float* va = vstate + ((size_t)s * N1 + ra) * N2;
  float* vb = va + N2;
  float oa[PPT], ob[PPT];
  if (mode == ROW_FULL) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      oa[q] = va[t + T * q];
      ob[q] = vb[t + T * q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) oa[q] = ob[q] = 0.f;
  }
#pragma unroll
  for (int k = 0; k < NTAB; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < N2) {
      tw[i] = rtw[k];
      if (mode != ROW_FINAL) ew[i] = rew[k];
    }
  }
#pragma unroll
  for (int k = 0; k < NSTG; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < H2 * SW) stg[pad8(i)] = rst[k];
  }
  __syncthreads();
  cx<float> v[PPT];
  staging_to_pair<N2, PPT, SW>(v, stg, g, t);
  __syncthreads();   // staging aliases the group scratch
  fft_group<N2, PPT, -1, float, true>(v, cb, t, tw);
  if (mode == ROW_FINAL) {
    float* xa = xout + ((size_t)s * N1 + ra) * N2;
    float* xb = xa + N2;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int n = t + T * q;
      xa[n] = v[q].x;
      xb[n] = v[q].y;
    }
    return;
  }
  dct_fwd_group<N2, PPT, false, true>(v, cb, t, tw, ew);
  if (sc == 1.f) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int k = t + T * q;
      float na = v[q].x + clip_f(oa[q], kappa);
      float nb = v[q].y + clip_f(ob[q], kappa);
      va[k] = na;
      vb[k] = nb;
      v[q] = cx<float>{2.f * soft_f(na, kappa) - na, 2.f * soft_f(nb, kappa) - nb};
    }
  } else {
    // penalty change after this iteration: u is rescaled by sc = rho / rho'
    // and the state is re-expressed for rho' (v' = t + sc u)
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int k = t + T * q;
      const float na = v[q].x + clip_f(oa[q], kappa);
      const float nb = v[q].y + clip_f(ob[q], kappa);
      const float ta = soft_f(na, kappa), tb = soft_f(nb, kappa);
      const float ua = sc * (na - ta), ub = sc * (nb - tb);
      va[k] = ta + ua;
      vb[k] = tb + ub;
      v[q] = cx<float>{ta - ua, tb - ub};
    }
  }
  dct_inv_group<N2, PPT, true, true>(v, cb, t, tw, ew);
  fft_group<N2, PPT, +1, float, true>(v, cb, t, tw);
  pair_to_staging<N2, PPT, SW, true>(v, cb, stg, g, t);
  __syncthreads();
  staging_to_subtile<SW>(Gout + rt_tile_base(s, row0, N1, H2), stg, H2, r0);
}

// Row pass of one ADMM iteration for the anisotropic TV prior on every plane
// (T = [D_v; D_h], circular forward differences along n1 and n2). One
// work-group per (plane, tile of RT rows), with one halo row on each side:
//   1. inverse row FFT of rows r0-1 .. r0+RT (column-pass output) -> x rows;
//   2. w_v = x[n1+1] - x[n1], w_h = x[n2+1] - x[n2]; state update
//      v_new = w + clip(v_old) for the RT own rows (both components) and the
//      halo row r0-1 (vertical component, recomputed, not stored);
//      q = t - u = 2 soft(v_new) - v_new;
//   3. g = T^T q = (q_v[n1-1] - q_v[n1]) + (q_h[n2-1] - q_h[n2]) for own rows;
//   4. forward row FFT of g -> RT output.
// The state is double-buffered (vin -> vout) because neighbouring tiles read
// the halo row of vin. Layout of each buffer: [component][S][N1][N2],
// component 0 = vertical (n1) difference, 1 = horizontal (n2) difference
// (2 = band difference for TV3D).
// LDS: [twiddles N2][work: max(NP + 1 group scratches, staging (2 NP + 2) x
// H2, q arrays)], 76 KB at N2 = 1024 with NP = 4 (two work-groups per CU),
// 45 KB with NP = 2 (three).
template <int N2, int NP = PAIRS> constexpr int tv_work_floats() {
  constexpr int H2 = N2 / 2 + 1;
  constexpr int SW = 2 * NP;
  constexpr int fft = (NP + 1) * 2 * padded_len(N2);
  constexpr int stg = 2 * pad8_len(H2 * (SW + 2));
  constexpr int xr = (SW + 2) * N2;
  constexpr int qq = (2 * SW + 1) * N2;   // QV (SW + 1 rows) and QH (SW rows)
  constexpr int a = fft > stg ? fft : stg;
  constexpr int b = xr > qq ? xr : qq;
  return a > b ? a : b;
}

// Global float access at a 32-bit element offset from a uniform base (the
// address is the base plus a zero-extended byte offset, one VGPR per
// address). Valid while 4 * off < 2^32.
__device__ __forceinline__ float ld_off(const float* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (off << 2));
}
__device__ __forceinline__ void st_off(float* __restrict__ base, unsigned off, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (off << 2)) = v;
}

// Steps shared by the TV row passes (TV2D and TV3D), for plane s and the SW =
// 2 NP own rows starting at rb (rows r0 .. r0 + SW - 1 of the RT-row tile at
// row0, rb = row0 + r0). Group g < NP owns rows rb + 2g, rb + 2g + 1 (local
// rows 1 + 2g, 2 + 2g of the LDS row block, whose row 0 is the halo row
// rb - 1); group NP only transforms the halo pair.
template <int N2, int PPT_ = ppt_row<N2>(), int NP_ = PAIRS> struct TvGeo {
  static constexpr int PPT = PPT_;
  static constexpr int NP = NP_;
  static constexpr int SW = 2 * NP;
  static constexpr int T = N2 / PPT;
  static constexpr int H2 = N2 / 2 + 1;
  static constexpr int NR = SW + 2;                // rows in LDS: halo, SW own rows, halo
  static constexpr unsigned NT = (NP + 1) * T;     // threads per work-group
  static constexpr int NE = (SW + 1) * N2;         // state elements: halo row + own rows
  static constexpr int PER = (NE + NT - 1) / NT;
};

// Stage rows rb-1 .. rb+SW of plane s ([k2][NR] order), rb = row0 + r0; own
// rows come from the tile at row0, the two halo rows from wherever they lie.
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__device__ __forceinline__ void tv_stage_rows(const cx<float>* __restrict__ Yin, cx<float>* stg,
                                              int s, int row0, int N1, int r0 = 0) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int H2 = G::H2, NR = G::NR, SW = G::SW;
  const cx<float>* tile = Yin + rt_tile_base(s, row0, N1, H2);
  batched_to_lds<8, cx<float>>(
      H2 * SW, [&](int i) { return tile[(i / SW) * RT + r0 + i % SW]; },
      [&](int i, const cx<float>& v) { stg[pad8((i / SW) * NR + i % SW + 1)] = v; });
  const int rb = row0 + r0;
  const int lo = (rb - 1 + N1) % N1, hi = (rb + SW) % N1;
  batched_to_lds<4, cx<float>>(
      2 * H2, [&](int i) { return Yin[rt_idx(s, i / H2 ? hi : lo, i % H2, N1, H2)]; },
      [&](int i, const cx<float>& v) { stg[pad8((i % H2) * NR + (i / H2 ? NR - 1 : 0))] = v; });
}

// Load the vertical / horizontal state this thread updates in tv_spatial
// (issued early so that the latency overlaps the transforms).
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__device__ __forceinline__ void tv_prefetch(const float* __restrict__ vin,
                                            float (&pov)[TvGeo<N2, PPT_, NP>::PER],
                                            float (&poh)[TvGeo<N2, PPT_, NP>::PER], unsigned s,
                                            int row0, int N1, unsigned cstride, int first) {
  using G = TvGeo<N2, PPT_, NP>;
  const unsigned plane = (unsigned)N1 * N2;
#pragma unroll
  for (int it = 0; it < G::PER; ++it) {
    const unsigned e = threadIdx.x + it * G::NT;
    pov[it] = 0.f;
    poh[it] = 0.f;
    if (e < (unsigned)G::NE && !first) {
      const unsigned lr = e / N2, n2 = e % N2;
      const unsigned n1 = (row0 == 0 && lr == 0) ? (unsigned)N1 - 1 : (unsigned)(row0 - 1) + lr;
      const unsigned o = s * plane + n1 * N2 + n2;
      pov[it] = ld_off(vin, o);
      if (lr > 0) poh[it] = ld_off(vin, cstride + o);
    }
  }
}

// Inverse row FFTs of the staged rows (two rows per group); x rows -> X =
// lds [NR][N2]. Begins after the staging writes and ends with a barrier.
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__device__ __forceinline__ void tv_inverse_rows(const cx<float>* stg, cx<float>* cb,
                                                const cx<float>* tw, float* X, int g, int t) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int PPT = G::PPT, T = G::T, NR = G::NR;
  __syncthreads();
  cx<float> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = k <= N2 / 2 ? k : N2 - k;
    float sg = k <= N2 / 2 ? 1.f : -1.f;
    int i = kk * NR + 2 * g;
    cx<float> A = stg[pad8(i)], B = stg[pad8(i + 1)];
    A.y *= sg;
    B.y *= sg;
    v[q] = cx<float>{A.x - B.y, A.y + B.x};
  }
  __syncthreads();
  fft_group<N2, PPT, -1>(v, cb, t, tw);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    X[(2 * g) * N2 + t + T * q] = v[q].x;
    X[(2 * g + 1) * N2 + t + T * q] = v[q].y;
  }
  __syncthreads();
}

// From X: state update of the vertical / horizontal components for the halo
// row (vertical only, not stored) and the own rows, q = 2 soft(v) - v, and
// the spatial part of T^T q for the own rows into v (two rows per group,
// zero for group NP). Overwrites X; ends with a barrier.
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__device__ __forceinline__ void tv_spatial(float* lds, const float (&pov)[TvGeo<N2, PPT_, NP>::PER],
                                           const float (&poh)[TvGeo<N2, PPT_, NP>::PER],
                                           float* __restrict__ vout, unsigned s, int row0, int N1,
                                           unsigned cstride, float kappa, float sc, int g, int t,
                                           cx<float> (&v)[PPT_]) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int PPT = G::PPT, T = G::T, PER = G::PER;
  const unsigned plane = (unsigned)N1 * N2;
  const float* X = lds;
  float qv[PER], qh[PER];
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const unsigned e = threadIdx.x + it * G::NT;
    if (e < (unsigned)G::NE) {
      const unsigned lr = e / N2, n2 = e % N2;   // lr 0 = halo row r0-1
      const unsigned n1 = (row0 == 0 && lr == 0) ? (unsigned)N1 - 1 : (unsigned)(row0 - 1) + lr;
      const float x0 = X[e];
      const float wv = X[e + N2] - x0;
      const unsigned o = s * plane + n1 * N2 + n2;
      const float nv = wv + clip_f(pov[it], kappa);
      float sv = nv;   // state written (re-expressed for rho' when sc != 1)
      if (sc == 1.f) {
        qv[it] = 2.f * soft_f(nv, kappa) - nv;
      } else {
        const float tv = soft_f(nv, kappa), uv = sc * (nv - tv);
        qv[it] = tv - uv;
        sv = tv + uv;
      }
      if (lr > 0) {
        const float wh = X[lr * N2 + (n2 + 1 == N2 ? 0 : n2 + 1)] - x0;
        const float nh = wh + clip_f(poh[it], kappa);
        float sh = nh;
        if (sc == 1.f) {
          qh[it] = 2.f * soft_f(nh, kappa) - nh;
        } else {
          const float th = soft_f(nh, kappa), uh = sc * (nh - th);
          qh[it] = th - uh;
          sh = th + uh;
        }
        st_off(vout, o, sv);
        st_off(vout, cstride + o, sh);
      }
    }
  }
  __syncthreads();
  // QV [SW + 1][N2] (row 0 = halo); QH holds local rows 1 .. SW, stored
  // right after QV (QH[e] for e >= N2 lands in [(SW + 1) N2, (2 SW + 1) N2)),
  // so that the work region stays below half of the CU's LDS and two
  // work-groups fit on a CU
  float* QV = lds;
  float* QH = lds + G::SW * N2;
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const unsigned e = threadIdx.x + it * G::NT;
    if (e < (unsigned)G::NE) {
      QV[e] = qv[it];
      if (e >= (unsigned)N2) QH[e] = qh[it];
    }
  }
  __syncthreads();
  const bool active = g < NP;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n2 = t + T * q;
    const int nm = n2 == 0 ? N2 - 1 : n2 - 1;
    float ga = 0.f, gb = 0.f;
    if (active) {
      const int la = 1 + 2 * g, lb = la + 1;
      ga = (QH[la * N2 + nm] - QH[la * N2 + n2]) + (QV[(la - 1) * N2 + n2] - QV[la * N2 + n2]);
      gb = (QH[lb * N2 + nm] - QH[lb * N2 + n2]) + (QV[(lb - 1) * N2 + n2] - QV[lb * N2 + n2]);
    }
    v[q] = cx<float>{ga, gb};
  }
  __syncthreads();
}

// Forward row FFT of v (two rows per group), split into the half spectra of
// the two rows, staged and written as rows r0 .. r0 + SW - 1 of the RT tile
// at `tile`.
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__device__ __forceinline__ void tv_forward_rows(cx<float> (&v)[PPT_], float* lds,
                                                cx<float>* cb, const cx<float>* tw,
                                                cx<float>* __restrict__ tile, int g, int t,
                                                int r0 = 0) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int PPT = G::PPT, T = G::T, H2 = G::H2, SW = G::SW;
  fft_group<N2, PPT, +1>(v, cb, t, tw);
  cx<float>* ostg = reinterpret_cast<cx<float>*>(lds);
  {
    constexpr int QH2 = (N2 / 2) / T + 1;
#pragma unroll
    for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
    __syncthreads();
    cx<float> A[QH2], B[QH2];
#pragma unroll
    for (int q = 0; q < QH2; ++q) {
      int k = t + T * q;
      if (k <= N2 / 2) {
        cx<float> Z = ldc(cb, k);
        cx<float> Zc = conjx(ldc(cb, k == 0 ? 0 : N2 - k));
        cx<float> sm = Z + Zc, d = Z - Zc;
        A[q] = cx<float>{0.5f * sm.x, 0.5f * sm.y};
        B[q] = cx<float>{0.5f * d.y, -0.5f * d.x};
      }
    }
    __syncthreads();
    if (g < NP) {
#pragma unroll
      for (int q = 0; q < QH2; ++q) {
        int k = t + T * q;
        if (k <= N2 / 2) {
          int i = k * SW + 2 * g;
          ostg[pad8(i)] = A[q];
          ostg[pad8(i + 1)] = B[q];
        }
      }
    }
  }
  __syncthreads();
  staging_to_subtile<SW>(tile, ostg, H2, r0);
}

// NP own row pairs per work-group (4: whole RT-row tiles; 2: half tiles,
// twice the work-groups, which spreads a 1024^2 x 3 problem evenly over the
// compute units at the cost of more halo rows).
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__global__ void __launch_bounds__((NP + 1) * (N2 / PPT_))
k_admm_row_tv(const cx<float>* __restrict__ Yin, cx<float>* __restrict__ Gout,
              const float* __restrict__ vin, float* __restrict__ vout, int S, int N1,
              const cx<float>* __restrict__ twg, float kappa, int first, float sc) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int PARTS = RT / G::SW;   // work-groups per RT-row tile
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / G::T, t = threadIdx.x % G::T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int s = b / (tiles * PARTS), rem = b % (tiles * PARTS);
  const int row0 = (rem / PARTS) * RT, r0 = (rem % PARTS) * G::SW;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  const unsigned cstride = (unsigned)S * N1 * N2;   // component stride within a buffer
  lds_load_table(tw, twg, N2);
  tv_stage_rows<N2, PPT_, NP>(Yin, stg, s, row0, N1, r0);
  float pov[G::PER], poh[G::PER];
  tv_prefetch<N2, PPT_, NP>(vin, pov, poh, s, row0 + r0, N1, cstride, first);
  tv_inverse_rows<N2, PPT_, NP>(stg, cb, tw, lds, g, t);
  cx<float> v[G::PPT];
  tv_spatial<N2, PPT_, NP>(lds, pov, poh, vout, s, row0 + r0, N1, cstride, kappa, sc, g, t, v);
  tv_forward_rows<N2, PPT_, NP>(v, lds, cb, tw, Gout + rt_tile_base(s, row0, N1, G::H2), g, t,
                                r0);
}

// Row pass of the TV3D prior: T adds the band difference w_b[s] = x[s+1] -
// x[s] (s < S - 1; none after the last plane), whose adjoint adds
// q_b[s-1] - q_b[s] to g of plane s. x of every plane is first brought to
// image space once by k_row_c2r (xin [S][N1][N2]); one work-group per (plane
// s, row tile) as for TV2D stages rows rb-1 .. rb+SW of plane s from xin and
// reads the own rows of planes s -/+ 1 from it directly, so no neighbouring
// plane is transformed again. q_b[s] is computed identically by the
// work-groups of planes s and s + 1 (same inputs, same arithmetic); only the
// former stores the band state of plane s.
// State buffer layout [3][S][N1][N2] (vertical, horizontal, band).
template <int N2, int PPT_ = ppt_row<N2>(), int NP = PAIRS>
__global__ void __launch_bounds__((NP + 1) * (N2 / PPT_))
k_admm_row_tv3(const float* __restrict__ xin, cx<float>* __restrict__ Gout,
                const float* __restrict__ vin, float* __restrict__ vout, int S, int N1,
                const cx<float>* __restrict__ twg, float kappa, int first, float sc) {
  using G = TvGeo<N2, PPT_, NP>;
  constexpr int PPT = G::PPT, T = G::T, NR = G::NR;
  constexpr int PARTS = RT / G::SW;   // work-groups per RT-row tile
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int s = b / (tiles * PARTS), rem = b % (tiles * PARTS);
  const int row0 = (rem / PARTS) * RT, r0 = (rem % PARTS) * G::SW, rb = row0 + r0;
  const unsigned plane = (unsigned)N1 * N2;
  const unsigned cstride = (unsigned)S * plane;
  const bool active = g < NP;
  const unsigned oa = (unsigned)(rb + 2 * g) * N2 + t;
  const float* Xa = lds + (1 + 2 * g) * N2 + t;
  const float* Xb = Xa + N2;
  lds_load_table(tw, twg, N2);
  // X rows 0 .. NR-1 are the image rows rb-1 .. rb+SW of plane s (circular)
  const float* xs = xin + (size_t)s * plane;
  batched_to_lds<8, float>(
      NR * N2,
      [&](int e) {
        int gr = rb - 1 + e / N2;
        gr += gr < 0 ? N1 : (gr >= N1 ? -N1 : 0);
        return xs[(size_t)gr * N2 + e % N2];
      },
      [&](int e, const float& v) { lds[e] = v; });
  float pov[G::PER], poh[G::PER];
  tv_prefetch<N2, PPT_, NP>(vin, pov, poh, s, rb, N1, cstride, first);
  __syncthreads();
  float xa[PPT], xb[PPT];   // x of plane s, own elements
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    xa[q] = active ? Xa[T * q] : 0.f;
    xb[q] = active ? Xb[T * q] : 0.f;
  }
  cx<float> v[PPT];
  tv_spatial<N2, PPT_, NP>(lds, pov, poh, vout, s, rb, N1, cstride, kappa, sc, g, t, v);
  // band terms: first + q_b[s-1] (from plane s-1), then - q_b[s] (plane s+1)
  for (int d = 0; d < 2; ++d) {
    const int sn = d == 0 ? s - 1 : s + 1;   // neighbouring plane
    if (sn < 0 || sn >= S || !active) continue;
    const unsigned bo = 2 * cstride + (unsigned)(d == 0 ? s - 1 : s) * plane + oa;
    const float* xn = xin + (size_t)sn * plane + oa;
    float na_[PPT], nb_[PPT], pa_[PPT], pb_[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      na_[q] = xn[T * q];
      nb_[q] = xn[N2 + T * q];
      pa_[q] = first ? 0.f : ld_off(vin, bo + T * q);
      pb_[q] = first ? 0.f : ld_off(vin, bo + N2 + T * q);
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const float wa = d == 0 ? xa[q] - na_[q] : na_[q] - xa[q];
      const float wb = d == 0 ? xb[q] - nb_[q] : nb_[q] - xb[q];
      const float na = wa + clip_f(pa_[q], kappa);
      const float nb = wb + clip_f(pb_[q], kappa);
      float qa, qb, sa = na, sb = nb;
      if (sc == 1.f) {
        qa = 2.f * soft_f(na, kappa) - na;
        qb = 2.f * soft_f(nb, kappa) - nb;
      } else {
        const float ta = soft_f(na, kappa), ua = sc * (na - ta);
        const float tb = soft_f(nb, kappa), ub = sc * (nb - tb);
        qa = ta - ua;
        qb = tb - ub;
        sa = ta + ua;
        sb = tb + ub;
      }
      if (d == 0) {
        v[q] = cx<float>{v[q].x + qa, v[q].y + qb};
      } else {
        st_off(vout, bo + T * q, sa);
        st_off(vout, bo + N2 + T * q, sb);
        v[q] = cx<float>{v[q].x - qa, v[q].y - qb};
      }
    }
  }
  tv_forward_rows<N2, PPT_, NP>(v, lds, reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2),
                                tw, Gout + rt_tile_base(s, row0, N1, G::H2), g, t, r0);
}

__device__ __forceinline__ int pair_index(int i, int j, int S) {  // i < j
  return i * S - i * (i + 1) / 2 + (j - i - 1);
}

// Mix the S planes of a column pass work-group at every element with the
// band matrix C (S x S, row-major): plane g receives sum_j C[g][j] v_j
// (TRANS: sum_j C[j][g] v_j). Group g holds plane g's elements t + T q in
// v; buf is the LDS array of S padded planes. Barriers before and after.
template <int N1, int PPT, int S, bool TRANS>
__device__ __forceinline__ void band_mix(cx<float>* v, cx<float>* buf, const float* __restrict__ C,
                                         int g, int t) {
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(buf + g * PL, t + T * q, v[q]);
  __syncthreads();
  float c[S];
#pragma unroll
  for (int j = 0; j < S; ++j) c[j] = TRANS ? C[j * S + g] : C[g * S + j];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const cx<float> w = ldc(buf + j * PL, t + T * q);
      acc.x += c[j] * w.x;
      acc.y += c[j] * w.y;
    }
    v[q] = acc;
  }
  __syncthreads();
}

// Column pass of one ADMM iteration, one work-group per column k2 holding all
// S planes: [inverse column DCT] -> column FFT -> per-frequency solve
//   X(w) = xh0(w) + A(w) g(w)    (A = rho Psi^+ / (N1 N2), packed Hermitian)
// -> inverse column FFT -> [column DCT] -> RT output.
// DCT = true for the DCT priors (T acts on both axes), false for TV priors;
// band != NULL (3D DCT): the band DCT C_S is applied across the planes after
// the column DCT of the output and its transpose before the inverse column
// DCT of the input (it commutes with the per-plane transforms).
// The solve tables (x_hat0, the diagonal and the S - 1 off-diagonal entries
// of plane g's Psi^+ row) go through a software pipeline of col_depth()
// frequencies: the first loads are issued with the input loads and ride
// under the column transforms, and solving frequency q issues the loads of
// frequency q + depth. A prefetch of all PPT frequencies costs about 2 S PPT
// registers and lowers the number of resident waves (measured: 34.6 us with
// it, 28.0 us reading each frequency's tables inside the solve, K = S = 3).
// LDS: [twiddles N1][DCT table E N1, when it fits][S x padded N1 complex];
// when the E table does not fit (N1 = 2048 with many planes) it is read
// from global memory.
constexpr int LDS_BYTES_MAX = 160 * 1024;
template <int N1, int S> constexpr bool col_e_in_lds() {
  return (4 * N1 + S * 2 * padded_len(N1)) * 4 <= LDS_BYTES_MAX;
}
template <int N1, bool DCT, int S> constexpr int col_lds_floats() {
  return 2 * N1 + (DCT && col_e_in_lds<N1, S>() ? 2 * N1 : 0) + S * 2 * padded_len(N1);
}

// Solve tables of one frequency for plane g.
template <int S> struct ColTab {
  cx<float> xh;
  float dg;
  cx<float> a[S > 1 ? S - 1 : 1];
};
// Frequencies in flight in the table pipeline (0: each frequency's tables
// are loaded where they are used). Measured at 1024^2, K = S = 3: 28.4 us
// with depth 0, 26.5 with 1, 26.2 with 2 or 4, 33.8 with 8 (the prologue
// loads then delay the first transform).
#ifndef CIP_COL_DEPTH
#define CIP_COL_DEPTH 2
#endif
template <int S, int PPT> constexpr int col_depth() {
  return CIP_COL_DEPTH < PPT ? CIP_COL_DEPTH : PPT;
}
template <int S>
__device__ __forceinline__ void col_tab_load(ColTab<S>& c, const cx<float>* __restrict__ xh0,
                                             const float* __restrict__ Adiag,
                                             const cx<float>* __restrict__ Aoff, size_t gi,
                                             const size_t (&arow)[S > 1 ? S - 1 : 1], size_t fi) {
  c.xh = xh0[gi];
  c.dg = Adiag[gi];
#pragma unroll
  for (int jj = 0; jj < S - 1; ++jj) c.a[jj] = Aoff[arow[jj] + fi];
}

// Pair mode of the column pass. The row transforms of real rows are real at
// k2 = 0 and k2 = N2/2, so those two columns travel as one complex column
// z = a + i b (one work-group instead of two: H2 - 1 = N2/2 work-groups in
// all, two per compute unit at N2 = 1024, none left over). After the column
// transform Z = A + i B with A, B the (Hermitian) spectra of a and b:
//   A[m] = (Z[m] + conj Z[N-m]) / 2,   B[m] = (Z[m] - conj Z[N-m]) / (2i).
// The solved spectra XA (column 0 tables) and XB (column N2/2 tables) are
// Hermitian too, so only m <= N/2 of each is solved: the thread holding
// frequency m < N/2 solves XA[m], the one holding m >= N/2 solves XB[N-m],
// and XB[0], XA[N/2] (needed by the thread holding m = 0 and m = N/2, t = 0)
// are solved by every thread alike.
// Each thread then takes the missing half from its partner (the thread
// holding N - m, through LDS) and forms Z'[m] = XA[m] + i XB[m], whose
// inverse column transform is xa + i xb.
// In: Z of every plane in LDS (planes p at lds + p PL). Out: v[q] = Z'[t + T q].
// Ends after the barrier that follows its LDS reads.
template <int N1, int PPT, int S, int D>
__device__ __forceinline__ void col_pair_solve(cx<float>* v, const cx<float>* Z, int g, int t,
                                               size_t F, size_t fb, const cx<float>* __restrict__ xh0,
                                               const float* __restrict__ Adiag,
                                               const cx<float>* __restrict__ Aoff,
                                               const size_t (&arow)[S > 1 ? S - 1 : 1],
                                               const float (&asgn)[S > 1 ? S - 1 : 1],
                                               cx<float>* cb, ColTab<S> (&tb)[D > 0 ? D : 1]) {
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  // table index of slot q: slot q < PPT/2 holds m < N/2 (XA[m], column 0
  // tables); slot q >= PPT/2 holds m >= N/2 (XB[N - m], column N2/2 tables;
  // at m = N/2 that is XB[N/2]). tb holds the tables of slots 0 .. D-1
  // (loaded with the input), as for the other columns.
  auto fidx = [&](int q) -> size_t {
    const int m = t + T * q;
    return 2 * q < PPT ? (size_t)m : fb + (size_t)(m == 0 ? 0 : N1 - m);
  };
  // one solve from separated inputs: HALF_A picks (Z[m] + conj Z[r]) / 2,
  // otherwise (Z[m] - conj Z[r]) / (2i)
  auto solve = [&](const ColTab<S>& c, int m, int r, bool half_a) {
    auto sep = [&](int p) {
      const cx<float> a = ldc(Z + p * PL, m), b = ldc(Z + p * PL, r);
      if (half_a) return cx<float>{0.5f * (a.x + b.x), 0.5f * (a.y - b.y)};
      return cx<float>{0.5f * (a.y + b.y), -0.5f * (a.x - b.x)};
    };
    const cx<float> u = sep(g);
    cx<float> acc = {c.xh.x + c.dg * u.x, c.xh.y + c.dg * u.y};
#pragma unroll
    for (int jj = 0; jj < S - 1; ++jj) {
      const int j = jj < g ? jj : jj + 1;
      cx<float> a = c.a[jj];
      a.y *= asgn[jj];
      acc = acc + cmul(a, sep(j));
    }
    return acc;
  };
  // XB[0] and XA[N/2], needed by thread 0: computed by every lane alike
  // (uniform addresses)
  ColTab<S> e0, eh;
  col_tab_load<S>(e0, xh0, Adiag, Aoff, (size_t)g * F + fb, arow, fb);
  col_tab_load<S>(eh, xh0, Adiag, Aoff, (size_t)g * F + N1 / 2, arow, (size_t)(N1 / 2));
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int m = t + T * q;
    const int mr = m == 0 ? 0 : N1 - m;
    ColTab<S> c;
    if constexpr (D == 0) {
      col_tab_load<S>(c, xh0, Adiag, Aoff, (size_t)g * F + fidx(q), arow, fidx(q));
    } else {
      c = tb[q % D];
      if (q + D < PPT)
        col_tab_load<S>(tb[q % D], xh0, Adiag, Aoff, (size_t)g * F + fidx(q + D), arow,
                        fidx(q + D));
    }
    if (2 * q < PPT) v[q] = solve(c, m, mr, true);   // XA[m]
    else v[q] = solve(c, mr, m, false);               // XB[N - m]
    __builtin_amdgcn_sched_barrier(0);
  }
  const cx<float> xb0 = solve(e0, 0, 0, false);
  const cx<float> xah = solve(eh, N1 / 2, N1 / 2, true);
  __syncthreads();   // every plane's Z was read
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int m = t + T * q;
    const cx<float> P = ldc(cb, m == 0 ? 0 : N1 - m);
  cx<float> xa, xb;
    if (q == 0 && t == 0) {
      xa = v[q];
      xb = xb0;
    } else if (2 * q == PPT && t == 0) {
      xa = xah;
      xb = v[q];
    } else if (2 * q < PPT) {
      xa = v[q];
      xb = P;
    } else {
      xa = conjx(P);
      xb = conjx(v[q]);
    }
    v[q] = cx<float>{xa.x - xb.y, xa.y + xb.x};
  }
  __syncthreads();   // partners' values were read before cb is reused
}

// Body of the column pass for column k2 (PAIR: columns 0 and N2/2 together).
template <int N1, bool DCT, int S, bool PAIR>
__device__ __forceinline__ void col_body(const cx<float>* __restrict__ Gin,
                                         cx<float>* __restrict__ Yout, int H2,
                                         const float* __restrict__ Adiag,
                                         const cx<float>* __restrict__ Aoff,
                                         const cx<float>* __restrict__ xh0,
                                         const cx<float>* __restrict__ twg,
                                         const cx<float>* __restrict__ ewg,
                                         const float* __restrict__ band, int zero_in, int dct_out,
                                         int k2) {
  constexpr int PPT = ppt_col<N1>();
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  constexpr bool ELDS = DCT && col_e_in_lds<N1, S>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  cx<float>* ewl = tw + N1;
  const cx<float>* ew = ELDS ? ewl : ewg;
  float* lds = reinterpret_cast<float*>(smem_raw) + (ELDS ? 4 : 2) * N1;
  const int kn = H2 - 1;
  // plane index; uniform across a wavefront when a group spans whole waves
  const int g = (T % 64 == 0) ? __builtin_amdgcn_readfirstlane(threadIdx.x / T)
                              : (int)(threadIdx.x / T);
  const int t = threadIdx.x % T;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * PL;
  const size_t F = (size_t)N1 * H2;
  const size_t f0 = (size_t)k2 * N1 + t;
  // offset of A[g][j] (packed upper triangle) and the sign of its imaginary
  // part (conjugate below the diagonal), per j != g
  size_t arow[S > 1 ? S - 1 : 1];
  float asgn[S > 1 ? S - 1 : 1];
#pragma unroll
  for (int jj = 0; jj < S - 1; ++jj) {
    const int j = jj < g ? jj : jj + 1;
    arow[jj] = (size_t)(g < j ? pair_index(g, j, S) : pair_index(j, g, S)) * F;
    asgn[jj] = g < j ? 1.f : -1.f;
  }
  constexpr int D = col_depth<S, PPT>();
  lds_load_table(tw, twg, N1);
  if (ELDS) lds_load_table(ewl, ewg, N1);
  cx<float> v[PPT];
  ColTab<S> tb[D > 0 ? D : 1];
  if (!zero_in) {
    if constexpr (PAIR) {
      // columns 0 and N2/2 of a real row transform are real: z = a + i b
#pragma unroll
      for (int q = 0; q < PPT; ++q)
        v[q] = cx<float>{Gin[rt_idx(g, t + T * q, 0, N1, H2)].x,
                         Gin[rt_idx(g, t + T * q, kn, N1, H2)].x};
    } else {
#pragma unroll
      for (int q = 0; q < PPT; ++q) v[q] = Gin[rt_idx(g, t + T * q, k2, N1, H2)];
    }
    // (in pair mode the first D slots also use the column 0 tables)
#pragma unroll
    for (int q = 0; q < D; ++q)
      col_tab_load<S>(tb[q], xh0, Adiag, Aoff, (size_t)g * F + f0 + T * q, arow, f0 + T * q);
  }
  __syncthreads();
  if (!zero_in) {
    if constexpr (DCT) {
      if (band) band_mix<N1, PPT, S, true>(v, reinterpret_cast<cx<float>*>(lds), band, g, t);
      dct_inv_group<N1, PPT, false, true>(v, cb, t, tw, ew);
    }
    fft_group<N1, PPT, +1, float, true>(v, cb, t, tw);
#pragma unroll
    for (int q = 0; q < PPT; ++q) stc(cb, t + T * q, v[q]);
    __syncthreads();
    if constexpr (PAIR) {
      static_assert(2 * D <= PPT, "pair mode: the prefetched slots must hold m < N/2");
      col_pair_solve<N1, PPT, S, D>(v, reinterpret_cast<const cx<float>*>(lds), g, t, F,
                                    (size_t)kn * N1, xh0, Adiag, Aoff, arow, asgn, cb, tb);
    } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int k1 = t + T * q;
      ColTab<S> c;
      if constexpr (D == 0) {
        col_tab_load<S>(c, xh0, Adiag, Aoff, (size_t)g * F + f0 + T * q, arow, f0 + T * q);
      } else {
        c = tb[q % D];
        if (q + D < PPT)
          col_tab_load<S>(tb[q % D], xh0, Adiag, Aoff, (size_t)g * F + f0 + T * (q + D), arow,
                          f0 + T * (q + D));
      }
      cx<float> gg = ldc(cb, k1);
      cx<float> acc = {c.xh.x + c.dg * gg.x, c.xh.y + c.dg * gg.y};
#pragma unroll
      for (int jj = 0; jj < S - 1; ++jj) {
        const int j = jj < g ? jj : jj + 1;
        cx<float> a = c.a[jj];
        a.y *= asgn[jj];
        acc = acc + cmul(a, ldc(reinterpret_cast<const cx<float>*>(lds) + j * PL, k1));
      }
      v[q] = acc;
      // keep the pipeline depth as written (otherwise the scheduler hoists
      // every table load and runs out of registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();   // every plane's scratch was read by the solve
    }
  } else if constexpr (PAIR) {
    const size_t fb = (size_t)kn * N1;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const cx<float> xa = xh0[(size_t)g * F + f0 + T * q];
      const cx<float> xb = xh0[(size_t)g * F + fb + t + T * q];
      v[q] = cx<float>{xa.x - xb.y, xa.y + xb.x};
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) v[q] = xh0[(size_t)g * F + f0 + T * q];
  }
  fft_group<N1, PPT, -1, float, true>(v, cb, t, tw);
  if constexpr (DCT) {
    if (dct_out) {
      dct_fwd_group<N1, PPT, false, true>(v, cb, t, tw, ew);
      if (band) band_mix<N1, PPT, S, false>(v, reinterpret_cast<cx<float>*>(lds), band, g, t);
    }
  }
  if constexpr (PAIR) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      Yout[rt_idx(g, t + T * q, 0, N1, H2)] = cx<float>{v[q].x, 0.f};
      Yout[rt_idx(g, t + T * q, kn, N1, H2)] = cx<float>{v[q].y, 0.f};
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) Yout[rt_idx(g, t + T * q, k2, N1, H2)] = v[q];
  }
}

// One work-group per column k2 < N2/2 (H2 - 1 work-groups); the one given
// k2 = 0 also carries the Nyquist column (col_pair_solve). The two bodies are
// separate instances so that neither's register allocation sees the other.
template <int N1, bool DCT, int S>
__global__ void __launch_bounds__(S * (N1 / ppt_col<N1>()))
k_admm_col(const cx<float>* __restrict__ Gin, cx<float>* __restrict__ Yout, int H2,
           const float* __restrict__ Adiag, const cx<float>* __restrict__ Aoff,
           const cx<float>* __restrict__ xh0, const cx<float>* __restrict__ twg,
           const cx<float>* __restrict__ ewg, const float* __restrict__ band, int zero_in,
           int dct_out) {
  const int k2 = xcd_remap(blockIdx.x, gridDim.x);
  if (k2 == 0)
    col_body<N1, DCT, S, true>(Gin, Yout, H2, Adiag, Aoff, xh0, twg, ewg, band, zero_in, dct_out,
                               0);
  else
    col_body<N1, DCT, S, false>(Gin, Yout, H2, Adiag, Aoff, xh0, twg, ewg, band, zero_in, dct_out,
                                k2);
}

}  // namespace cip
