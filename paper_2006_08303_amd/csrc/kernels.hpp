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

template <int N> constexpr int ppt_for() { return N >= 16 ? 16 : N; }

__device__ __forceinline__ size_t rt_tile_base(int p, int n1, int N1, int H2) {
  return (((size_t)p * (N1 / RT) + (n1 / RT)) * H2) * RT;
}
__device__ __forceinline__ size_t rt_idx(int p, int n1, int k2, int N1, int H2) {
  return rt_tile_base(p, n1, N1, H2) + (size_t)k2 * RT + (n1 % RT);
}
__device__ __forceinline__ size_t fl_idx(int e, int k1, int k2, int N1, int H2) {
  return ((size_t)e * H2 + k2) * N1 + k1;
}

template <typename Re> __device__ __forceinline__ cx<Re> ldc(const Re* re, const Re* im, int i) {
  return cx<Re>{re[pad(i)], im[pad(i)]};
}
template <typename Re> __device__ __forceinline__ void stc(Re* re, Re* im, int i, cx<Re> v) {
  re[pad(i)] = v.x;
  im[pad(i)] = v.y;
}

// ---------------------------------------------------------------- DCT via FFT
// Orthonormal DCT-II of a complex sequence (real and imaginary parts
// transformed independently), computed with one N-point FFT of the
// even/odd-reordered sequence and a post-twiddle (Makhoul's method).
//   fw[k] = a_k exp(-i pi k / 2N),  a_0 = sqrt(1/N), a_k = sqrt(2/N).
template <int N, int PPT>
__device__ __forceinline__ void dct_fwd_group(cx<float>* reg, float* re, float* im, int t,
                                              const cx<float>* __restrict__ tw,
                                              const cx<float>* __restrict__ fw) {
  constexpr int T = N / PPT;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int n = t + T * q;
    int p = (n & 1) ? (N - 1 - (n >> 1)) : (n >> 1);
    stc(re, im, p, reg[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) reg[q] = ldc(re, im, t + T * q);
  fft_group<N, PPT, +1>(reg, re, im, t, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, reg[q]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = (N - k) & (N - 1);
    cx<float> V = ldc(re, im, k);
    cx<float> Vc = conjx(ldc(re, im, kk));
    cx<float> s = V + Vc, d = V - Vc;
    cx<float> Va = {0.5f * s.x, 0.5f * s.y};
    cx<float> Vb = {0.5f * d.y, -0.5f * d.x};   // (V - conj V[N-k]) / 2i
    cx<float> c = fw[k];
    reg[q] = cx<float>{c.x * Va.x - c.y * Va.y, c.x * Vb.x - c.y * Vb.y};
  }
}

// Inverse (DCT-III, orthonormal) of a complex coefficient sequence:
//   V[k] = iv[k] (Y[k] ia[k] - i Y[N-k] ia[N-k]),  V[0] = iv[0] Y[0] ia[0],
//   iv[k] = exp(i pi k / 2N) / N, ia[k] = 1 / a_k,
// then an inverse FFT and the inverse even/odd reordering.
template <int N, int PPT>
__device__ __forceinline__ void dct_inv_group(cx<float>* reg, float* re, float* im, int t,
                                              const cx<float>* __restrict__ tw,
                                              const cx<float>* __restrict__ iv,
                                              const float* __restrict__ ia) {
  constexpr int T = N / PPT;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, reg[q]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    cx<float> Yk = ldc(re, im, k);
    float sk = ia[k];
    cx<float> a = {Yk.x * sk, Yk.y * sk};
    if (k != 0) {
      int kk = N - k;
      cx<float> Yn = ldc(re, im, kk);
      float sn = ia[kk];
      a.x += Yn.y * sn;    // - i * Yn
      a.y -= Yn.x * sn;
    }
    reg[q] = cmul(iv[k], a);
  }
  fft_group<N, PPT, -1>(reg, re, im, t, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int m = t + T * q;
    int pos = (m < N / 2) ? 2 * m : 2 * N - 2 * m - 1;
    stc(re, im, pos, reg[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) reg[q] = ldc(re, im, t + T * q);
}

// Exact float -> double promotion of one plane (plan time).
__global__ void k_promote(const float* __restrict__ src, double* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------- row passes
// Two real rows a, b are carried by one complex FFT (z = a + i b).

// Real-to-complex FFT of every row: in [P][N1][N2] -> out RT [P][N1/RT][H2][RT].
// One work-group per (plane, pair of rows) when STAGED = false (any type), or
// per (plane, row tile) with a coalesced tile store when STAGED = true.
template <int N2, typename Re, bool STAGED>
__global__ void k_row_r2c(const Re* __restrict__ in, cx<Re>* __restrict__ out, int N1,
                          const cx<Re>* __restrict__ tw) {
  constexpr int PPT = ppt_for<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  constexpr int NG = STAGED ? PAIRS : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Re* lds = reinterpret_cast<Re*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  int p, row0;  // plane and first row handled by this work-group
  if (STAGED) {
    const int tiles = N1 / RT;
    p = blockIdx.x / tiles;
    row0 = (blockIdx.x % tiles) * RT;
  } else {
    const int pairs = N1 / 2;
    p = blockIdx.x / pairs;
    row0 = (blockIdx.x % pairs) * 2;
  }
  const int ra = row0 + 2 * g;
  Re* re = lds + g * 2 * padded_len(N2);
  Re* im = re + padded_len(N2);
  const Re* xa = in + ((size_t)p * N1 + ra) * N2;
  const Re* xb = xa + N2;
  cx<Re> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int n = t + T * q;
    v[q] = cx<Re>{xa[n], xb[n]};
  }
  fft_group<N2, PPT, +1>(v, re, im, t, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, v[q]);
  __syncthreads();
  cx<Re> A[PPT], B[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    if (k <= N2 / 2) {
      cx<Re> Z = ldc(re, im, k);
      cx<Re> Zc = conjx(ldc(re, im, (N2 - k) & (N2 - 1)));
      cx<Re> s = Z + Zc, d = Z - Zc;
      A[q] = cx<Re>{Re(0.5) * s.x, Re(0.5) * s.y};
      B[q] = cx<Re>{Re(0.5) * d.y, Re(-0.5) * d.x};
    }
  }
  if constexpr (STAGED) {
    __syncthreads();
    Re* st = lds;   // [H2][RT] complex, aliases the FFT scratch
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int k = t + T * q;
      if (k <= N2 / 2) {
        int ia = (k * RT + 2 * g) * 2;
        st[ia] = A[q].x;
        st[ia + 1] = A[q].y;
        st[ia + 2] = B[q].x;
        st[ia + 3] = B[q].y;
      }
    }
    __syncthreads();
    cx<Re>* dst = out + rt_tile_base(p, row0, N1, H2);
    for (int i = threadIdx.x; i < H2 * RT; i += blockDim.x) dst[i] = cx<Re>{st[2 * i], st[2 * i + 1]};
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int k = t + T * q;
      if (k <= N2 / 2) {
        out[rt_idx(p, ra, k, N1, H2)] = A[q];
        out[rt_idx(p, ra + 1, k, N1, H2)] = B[q];
      }
    }
  }
}

// Complex-to-real inverse FFT of every row: RT [P][..] -> out [P][N1][N2],
// scaled by `scale`. One work-group per (plane, row tile).
template <int N2>
__global__ void k_row_c2r(const cx<float>* __restrict__ in, float* __restrict__ out, int N1,
                          float scale, const cx<float>* __restrict__ tw) {
  constexpr int PPT = ppt_for<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int p = blockIdx.x / tiles, row0 = (blockIdx.x % tiles) * RT;
  float* re = lds + g * 2 * padded_len(N2);
  float* im = re + padded_len(N2);
  float* st = lds;
  const cx<float>* src = in + rt_tile_base(p, row0, N1, H2);
  for (int i = threadIdx.x; i < H2 * RT; i += blockDim.x) {
    cx<float> z = src[i];
    st[2 * i] = z.x;
    st[2 * i + 1] = z.y;
  }
  __syncthreads();
  cx<float> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = k <= N2 / 2 ? k : N2 - k;
    float sg = k <= N2 / 2 ? 1.f : -1.f;
    int ia = (kk * RT + 2 * g) * 2;
    cx<float> A = {st[ia], sg * st[ia + 1]};
    cx<float> B = {st[ia + 2], sg * st[ia + 3]};
    v[q] = cx<float>{A.x - B.y, A.y + B.x};
  }
  fft_group<N2, PPT, -1>(v, re, im, t, tw);
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
template <int N1, typename Re, int OP>
__global__ void k_col_op(const cx<Re>* __restrict__ in, void* __restrict__ outv, int Pin, int Pout,
                         int H2, const cx<Re>* __restrict__ tw, const cx<Re>* __restrict__ mat,
                         int spec_plane) {
  constexpr int PPT = ppt_for<N1>();
  constexpr int T = N1 / PPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Re* lds = reinterpret_cast<Re*>(smem_raw);
  const int k2 = blockIdx.x;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int PM = blockDim.x / T;
  constexpr int PL = padded_len(N1);
  Re* re = lds + g * 2 * PL;
  Re* im = re + PL;
  cx<Re> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q)
    v[q] = g < Pin ? in[rt_idx(g, t + T * q, k2, N1, H2)] : cx<Re>{Re(0), Re(0)};
  fft_group<N1, PPT, +1>(v, re, im, t, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, v[q]);
  __syncthreads();
  const size_t F = (size_t)N1 * H2;
  if constexpr (OP == OP_SPEC) {
    cx<Re>* out = reinterpret_cast<cx<Re>*>(outv);
    if (g == 0) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) out[fl_idx(spec_plane, t + T * q, k2, N1, H2)] = v[q];
    }
    return;
  } else {
    // per-frequency map; each thread owns whole frequencies
    for (int k1 = threadIdx.x; k1 < N1; k1 += blockDim.x) {
      cx<Re> xin[8];
      for (int j = 0; j < Pin; ++j) xin[j] = ldc(lds + j * 2 * PL, lds + j * 2 * PL + PL, k1);
      const size_t f = (size_t)k2 * N1 + k1;
      for (int o = 0; o < Pout; ++o) {
        cx<Re> acc = {Re(0), Re(0)};
        for (int j = 0; j < Pin; ++j) {
          cx<Re> m;
          if (OP == OP_FWD) m = mat[(size_t)(o * Pin + j) * F + f];
          else if (OP == OP_ADJ) m = conjx(mat[(size_t)(j * Pout + o) * F + f]);
          else m = mat[(size_t)(o * Pin + j) * F + f];
          acc = acc + cmul(m, xin[j]);
        }
        if (OP == OP_XHAT0) {
          reinterpret_cast<cx<Re>*>(outv)[(size_t)o * F + f] = acc;
        } else {
          stc(lds + o * 2 * PL, lds + o * 2 * PL + PL, k1, acc);
        }
      }
    }
    if constexpr (OP == OP_XHAT0) return;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) v[q] = ldc(re, im, t + T * q);
    fft_group<N1, PPT, -1>(v, re, im, t, tw);
    cx<Re>* out = reinterpret_cast<cx<Re>*>(outv);
    if (g < Pout) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) out[rt_idx(g, t + T * q, k2, N1, H2)] = v[q];
    }
    (void)PM;
  }
}

// ---------------------------------------------------------------- ADMM, DCT prior
// State: v = T x^l + u^{l-1} per DCT coefficient (one float per voxel). From
// v the pair (t, u) of Algorithm 1 is t = soft(v, kappa), u = clip(v, kappa),
// so t - u = 2 soft(v) - v and the next v = T x^{l+1} + clip(v).
__device__ __forceinline__ float soft_f(float v, float k) {
  return v > k ? v - k : (v < -k ? v + k : 0.f);
}
__device__ __forceinline__ float clip_f(float v, float k) { return fminf(fmaxf(v, -k), k); }

enum RowMode { ROW_FIRST = 0, ROW_FULL = 1, ROW_FINAL = 2 };

// Row pass of one ADMM iteration (DCT prior), one work-group per (plane, row
// tile): inverse row FFT of the column-pass output (x^l in the column-DCT /
// row-frequency domain) -> row DCT gives w = T x^l -> prox + dual update of v
// -> inverse row DCT of t - u -> forward row FFT -> RT output for the next
// column pass. ROW_FINAL stops after the inverse row FFT and writes x.
template <int N2>
__global__ void __launch_bounds__(PAIRS * (N2 / ppt_for<N2>()))
k_admm_row_dct(const cx<float>* __restrict__ Yin, cx<float>* __restrict__ Gout,
               float* __restrict__ vstate, int N1, const cx<float>* __restrict__ tw,
               const cx<float>* __restrict__ fw, const cx<float>* __restrict__ iv,
               const float* __restrict__ ia, float kappa, int mode, float* __restrict__ xout) {
  constexpr int PPT = ppt_for<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int s = blockIdx.x / tiles, row0 = (blockIdx.x % tiles) * RT;
  float* re = lds + g * 2 * padded_len(N2);
  float* im = re + padded_len(N2);
  float* st = lds;
  const cx<float>* src = Yin + rt_tile_base(s, row0, N1, H2);
  for (int i = threadIdx.x; i < H2 * RT; i += blockDim.x) {
    cx<float> z = src[i];
    st[2 * i] = z.x;
    st[2 * i + 1] = z.y;
  }
  __syncthreads();
  cx<float> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    int kk = k <= N2 / 2 ? k : N2 - k;
    float sg = k <= N2 / 2 ? 1.f : -1.f;
    int ia2 = (kk * RT + 2 * g) * 2;
    cx<float> A = {st[ia2], sg * st[ia2 + 1]};
    cx<float> B = {st[ia2 + 2], sg * st[ia2 + 3]};
    v[q] = cx<float>{A.x - B.y, A.y + B.x};
  }
  fft_group<N2, PPT, -1>(v, re, im, t, tw);
  const int ra = row0 + 2 * g;
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
  dct_fwd_group<N2, PPT>(v, re, im, t, tw, fw);
  float* va = vstate + ((size_t)s * N1 + ra) * N2;
  float* vb = va + N2;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    float oa = 0.f, ob = 0.f;
    if (mode != ROW_FIRST) {
      oa = va[k];
      ob = vb[k];
    }
    float na = v[q].x + clip_f(oa, kappa);
    float nb = v[q].y + clip_f(ob, kappa);
    va[k] = na;
    vb[k] = nb;
    v[q] = cx<float>{2.f * soft_f(na, kappa) - na, 2.f * soft_f(nb, kappa) - nb};
  }
  dct_inv_group<N2, PPT>(v, re, im, t, tw, iv, ia);
  fft_group<N2, PPT, +1>(v, re, im, t, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, v[q]);
  __syncthreads();
  cx<float> A[PPT], B[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    if (k <= N2 / 2) {
      cx<float> Z = ldc(re, im, k);
      cx<float> Zc = conjx(ldc(re, im, (N2 - k) & (N2 - 1)));
      cx<float> sm = Z + Zc, d = Z - Zc;
      A[q] = cx<float>{0.5f * sm.x, 0.5f * sm.y};
      B[q] = cx<float>{0.5f * d.y, -0.5f * d.x};
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k = t + T * q;
    if (k <= N2 / 2) {
      int i2 = (k * RT + 2 * g) * 2;
      st[i2] = A[q].x;
      st[i2 + 1] = A[q].y;
      st[i2 + 2] = B[q].x;
      st[i2 + 3] = B[q].y;
    }
  }
  __syncthreads();
  cx<float>* dst = Gout + rt_tile_base(s, row0, N1, H2);
  for (int i = threadIdx.x; i < H2 * RT; i += blockDim.x) dst[i] = cx<float>{st[2 * i], st[2 * i + 1]};
}

__device__ __forceinline__ int pair_index(int i, int j, int S) {  // i < j
  return i * S - i * (i + 1) / 2 + (j - i - 1);
}

// Column pass of one ADMM iteration, one work-group per column k2 holding all
// S planes: [inverse column DCT] -> column FFT -> per-frequency solve
//   X(w) = xh0(w) + A(w) g(w)    (A = rho Psi^+ / (N1 N2), packed Hermitian)
// -> inverse column FFT -> [column DCT] -> RT output.
// DCT = true for the DCT prior (T acts on both axes), false for TV priors.
template <int N1, bool DCT>
__global__ void __launch_bounds__(8 * (N1 / ppt_for<N1>()))
k_admm_col(const cx<float>* __restrict__ Gin, cx<float>* __restrict__ Yout, int S, int H2,
           const float* __restrict__ Adiag, const cx<float>* __restrict__ Aoff,
           const cx<float>* __restrict__ xh0, const cx<float>* __restrict__ tw,
           const cx<float>* __restrict__ fw, const cx<float>* __restrict__ iv,
           const float* __restrict__ ia, int zero_in, int dct_out) {
  constexpr int PPT = ppt_for<N1>();
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* lds = reinterpret_cast<float*>(smem_raw);
  const int k2 = blockIdx.x;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  float* re = lds + g * 2 * PL;
  float* im = re + PL;
  cx<float> v[PPT];
  if (!zero_in) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) v[q] = Gin[rt_idx(g, t + T * q, k2, N1, H2)];
    if constexpr (DCT) dct_inv_group<N1, PPT>(v, re, im, t, tw, iv, ia);
    fft_group<N1, PPT, +1>(v, re, im, t, tw);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PPT; ++q) stc(re, im, t + T * q, v[q]);
    __syncthreads();
  }
  const size_t F = (size_t)N1 * H2;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    int k1 = t + T * q;
    size_t f = (size_t)k2 * N1 + k1;
    cx<float> acc = xh0[(size_t)g * F + f];
    if (!zero_in) {
      float d = Adiag[(size_t)g * F + f];
      cx<float> gg = ldc(re, im, k1);
      acc.x += d * gg.x;
      acc.y += d * gg.y;
      for (int j = 0; j < S; ++j) {
        if (j == g) continue;
        cx<float> a = (g < j) ? Aoff[(size_t)pair_index(g, j, S) * F + f]
                              : conjx(Aoff[(size_t)pair_index(j, g, S) * F + f]);
        acc = acc + cmul(a, ldc(lds + j * 2 * PL, lds + j * 2 * PL + PL, k1));
      }
    }
    v[q] = acc;
  }
  fft_group<N1, PPT, -1>(v, re, im, t, tw);
  if constexpr (DCT) {
    if (dct_out) dct_fwd_group<N1, PPT>(v, re, im, t, tw, fw);
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) Yout[rt_idx(g, t + T * q, k2, N1, H2)] = v[q];
}

}  // namespace cip
