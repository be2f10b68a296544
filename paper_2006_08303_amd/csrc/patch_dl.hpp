// Online update of the patch dictionary (Section IV-B, patch-based
// dictionary update): one step of the dictionary ADMM per outer iteration,
// taken after the sparse-code update with the image x and the codes Z:
//   D = (X Z^T + sigma (G - E)) (Z Z^T + sigma I)^-1     Eq. sold_patch
//   G = (D + E) / ||D + E||_F                              Eq. ADMM1
//   E = E + D - G                                          Eq. subh
// (E is the scaled dual of the penalty sigma/2 ||D - G + E||^2 of Eqs. ADMM0
// and ADMM1, so it moves by the split residual D - G; the sign printed with
// Eq. subh makes E double every step and the solve diverge)
// with X = [P_1 x | ... | P_J x] (n x J, n = 64 S) and Z (A x J). The next x-
// and code updates use G: its BF16 copy and M1 = G^T (rho I + G G^T)^-1.
//
// Z Z^T + sigma I is ill-conditioned at the paper's sigma = 1 (its largest
// eigenvalue grows with the patch count: about 1e6 relative to sigma at
// 1024^2), so the D-step runs in FP64 on the FP32 operands x and Z:
//   k_pdl_gemm64   X Z^T and Z Z^T on FP64 MFMA (v_mfma_f64_16x16x4), the
//                  products of FP32 operands exact, FP64 accumulation, split
//                  over the patches, every split written to its own slice
//                  (no atomics);
//   k_pdl_reduce64 fixed-order sum of the slices, + sigma (G - E) and sigma I;
//   k_pdl_chol64   Cholesky factor of Z Z^T + sigma I (order A <= 256),
//                  blocked right-looking in one work-group: 16-column panels
//                  factored by one wave in registers (readlane broadcasts, no
//                  barriers), trailing updates by all waves in 8 x 8
//                  register tiles from the panel in LDS;
//   k_pdl_trsolve64  rows of B M^-1 = B L^-T L^-1 in FP64, one row per wave,
//                  L read from global memory (L2) a few columns ahead;
//   k_pdl_project  the Frobenius projection (FP64 norm) and the dual update
//                  from the FP64 D; G and E kept in FP32.
// M1 = G^T (rho I + G G^T)^-1 (well conditioned for the unit-norm G and the
// rho of the code split) stays FP32: k_pdl_gram, k_pdl_chol (FP32, one
// work-group, the matrix in registers, 8 x 8 per thread, pivot columns
// broadcast through LDS) and k_pdl_trsolve (L packed in LDS), with the BF16
// copy of M1 as output.
#pragma once
#include "patch.hpp"

namespace cip {

constexpr int PDL_MAXM = 256;    // largest system order (A or n = 64 S)
constexpr int PDL_KSTEP = 32;    // patches per LDS stage of k_pdl_gemm

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Split-K products W Z^T with W = [X; Z] ((n + A) x J) in FP64. Work-group
// (rb, cb, ks) computes the 64 x 64 block (rb, cb) over the patches
// [ks * chunk, (ks + 1) * chunk) and writes it to part[ks] ((n + A) x A,
// row-major). Rows rb < S are the patch rows of plane s = rb (row
// 64 s + 8 a + b, patch j = pi J2 + pj: pixel x[s][4 pi + a][4 pj + b],
// circular); blocks of Z Z^T above the diagonal are skipped. Each stage of
// 32 patches is staged in LDS as FP64 (the FP32 values convert exactly);
// wave (wr, wc) computes the 32 x 32 quarter (wr, wc) as 2 x 2 tiles of
// v_mfma_f64_16x16x4 (lane l: A[l % 16][l / 16], B[l / 16][l % 16]; result
// register r: D[l / 16 + 4 r][l % 16]).
// Requires chunk % 32 == 0, J % chunk == 0, J2 a power of two.
constexpr int PDL_LS64 = PDL_KSTEP + 1;   // LDS row stride (doubles)

__global__ void __launch_bounds__(256)
k_pdl_gemm64(const float* __restrict__ x, const float* __restrict__ zf, double* __restrict__ part,
             PatchGeo G, int S, int NA, int chunk) {
  __shared__ double As[64][PDL_LS64], Bs[64][PDL_LS64];
  const int rb = blockIdx.x, cb = blockIdx.y, ks = blockIdx.z;
  if (rb >= S && cb > rb - S) return;
  const int rows = 64 * S + NA;
  const size_t J = (size_t)G.J1 * G.J2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 8;   // staging: row, 8 patches
  const int pa = lr >> 3, pb = lr & 7;
  const int jsh = __builtin_ctz((unsigned)G.J2);
  const float* zb = zf + (size_t)(64 * cb + lr) * J;
  const float* za = zf + (size_t)(64 * (rb >= S ? rb - S : 0) + lr) * J;
  const float* xs = x + (size_t)(rb < S ? rb : 0) * G.N1 * G.N2;
  f64x4 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = f64x4{0.0, 0.0, 0.0, 0.0};
  // the next stage's operands are loaded into registers while the current
  // stage runs on the MFMA units
  auto load = [&](size_t j0, float (&av)[8], float (&bv)[8]) {
    const float4* bp = reinterpret_cast<const float4*>(zb + j0 + lk);
    const float4 b0 = bp[0], b1 = bp[1];
    bv[0] = b0.x; bv[1] = b0.y; bv[2] = b0.z; bv[3] = b0.w;
    bv[4] = b1.x; bv[5] = b1.y; bv[6] = b1.z; bv[7] = b1.w;
    if (rb >= S) {
      const float4* ap = reinterpret_cast<const float4*>(za + j0 + lk);
      const float4 a0 = ap[0], a1 = ap[1];
      av[0] = a0.x; av[1] = a0.y; av[2] = a0.z; av[3] = a0.w;
      av[4] = a1.x; av[5] = a1.y; av[6] = a1.z; av[7] = a1.w;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const size_t j = j0 + lk + q;
        const int pi = (int)(j >> jsh), pj = (int)(j & (size_t)(G.J2 - 1));
        const int r = (PATCH_ST * pi + pa) & (G.N1 - 1), c = (PATCH_ST * pj + pb) & (G.N2 - 1);
        av[q] = xs[(size_t)r * G.N2 + c];
      }
    }
  };
  const size_t jbeg = (size_t)ks * chunk, jend = jbeg + chunk;
  const int li = lane & 15, lq = lane >> 4;
  float av[8], bv[8];
  load(jbeg, av, bv);
  for (size_t j0 = jbeg; j0 < jend; j0 += PDL_KSTEP) {
    __syncthreads();   // the previous stage has been consumed
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      As[lr][lk + q] = (double)av[q];
      Bs[lr][lk + q] = (double)bv[q];
    }
    __syncthreads();
    if (j0 + PDL_KSTEP < jend) load(j0 + PDL_KSTEP, av, bv);
#pragma unroll
    for (int kk = 0; kk < PDL_KSTEP / 4; ++kk) {
      const int k = 4 * kk + lq;
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[32 * wr + 16 * t + li][k];
        b[t] = Bs[32 * wc + 16 * t + li][k];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      double* out = part + ((size_t)ks * rows + 64 * rb + 32 * wr + 16 * t + lq) * NA + 64 * cb +
                    32 * wc + 16 * u + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(size_t)(4 * r) * NA] = acc[t][u][r];
    }
}

// Sum of the KS slices in a fixed order (FP64). Rows r < n: B = X Z^T +
// sigma (G - E) (n x A, row-major); rows n + i: C = Z Z^T + sigma I into cm
// (leading dimension 256; the blocks on and below the diagonal only).
__global__ void k_pdl_reduce64(const double* __restrict__ part, const float* __restrict__ g,
                               const float* __restrict__ e, double* __restrict__ bm,
                               double* __restrict__ cm, int nv, int NA, int KS, double sigma) {
  const int rows = nv + NA;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)rows * NA) return;
  const int r = (int)(idx / NA), c = (int)(idx % NA);
  if (r >= nv && (c >> 6) > ((r - nv) >> 6)) return;
  double s = 0.0;
  for (int k = 0; k < KS; ++k) s += part[(size_t)k * rows * NA + idx];
  if (r < nv) {
    bm[idx] = s + sigma * ((double)g[idx] - (double)e[idx]);
  } else {
    const int i = r - nv;
    cm[(size_t)i * PDL_MAXM + c] = s + (i == c ? sigma : 0.0);
  }
}

// Cholesky factor L (M = L L^T) of the SPD matrix M of order m <= 256 whose
// lower triangle is a[i * lda + k] (i >= k). Output lt[k * 256 + i] = L[i][k]
// for i >= k (row k of lt is column k of L); orders above m are padded with
// the identity. One work-group of 640 threads: each of its 10 waves holds one
// 64 x 64 block on or below the diagonal of the padded matrix, each lane an
// 8 x 8 tile (lane / 8, lane % 8) of it, in registers. Gaussian elimination
// on the symmetric matrix (P[i][k] -= P[i][j] P[k][j] / P[j][j] for
// i, k > j), two columns per step: the owners publish them in LDS with their
// eliminated entries set to zero, and the pivots apart, so that every tile
// applies the same unmasked rank-2 update; the buffers alternate between
// steps, so one barrier per two columns suffices. At the end
// L[i][k] = P[i][k] / sqrt(P[k][k]).
// The block of wave w is chosen so that, with waves placed on the four SIMDs
// round-robin, the blocks still active at step j (those with block column
// >= j / 64) spread evenly: 3, 2, 1 and 1 per SIMD for the four column
// blocks.
constexpr int PDL_CHOL_THREADS = 640;

__global__ void __launch_bounds__(PDL_CHOL_THREADS)
k_pdl_chol(const float* __restrict__ a, int lda, int m, float* __restrict__ lt) {
  __shared__ __align__(16) float colb[2][2][PDL_MAXM];
  __shared__ float pivb[2][2];
  __shared__ float piv[PDL_MAXM];
  constexpr int kBi[10] = {3, 2, 3, 3, 1, 2, 2, 3, 0, 1};
  constexpr int kBk[10] = {3, 2, 2, 1, 1, 1, 0, 0, 0, 0};
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bi = kBi[w], bk = kBk[w];
  const int ti = 8 * bi + (lane >> 3), tk = 8 * bk + (lane & 7);
  float P[8][8];
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = 8 * ti + r, k = 8 * tk + c;
      float v = i == k ? 1.f : 0.f;
      if (i < m && k < m) v = i >= k ? a[(size_t)i * lda + k] : a[(size_t)k * lda + i];
      P[r][c] = v;
    }
  // Columns j and j + 1 per barrier (a rank-2 update; both lie in one tile
  // column). The owners publish both raw columns, entries i <= j (column j)
  // and i <= j + 1 (column j + 1) set to zero, and both diagonal entries;
  // every thread then forms column j + 1 after column j's elimination for
  // its own rows and columns, b = c1 - c0 c0[j + 1] / p0 (zero for
  // i <= j + 1), p1 = P[j+1][j+1] - c0[j+1]^2 / p0, and applies
  // P -= c0 c0^T / p0 + b b^T / p1. Orders above m are the identity.
  for (int j = 0; j < m; j += 2) {
    const int par = (j >> 1) & 1;
    float* cb0 = colb[par][0];
    float* cb1 = colb[par][1];
    if (tk == (j >> 3)) {
#pragma unroll
      for (int c = 0; c < 8; c += 2)
        if (c == (j & 7)) {
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int i = 8 * ti + r;
            cb0[i] = i > j ? P[r][c] : 0.f;
            cb1[i] = i > j + 1 ? P[r][c + 1] : 0.f;
            if (i == j) pivb[par][0] = P[r][c];
            if (i == j + 1) pivb[par][1] = P[r][c + 1];
          }
        }
    }
    __syncthreads();
    if (8 * ti + 7 > j && 8 * tk + 7 > j) {
      const float p0 = pivb[par][0], q = cb0[j + 1];
      const float inv0 = 1.f / p0, qi = q * inv0;
      const float inv1 = 1.f / (pivb[par][1] - q * qi);
      const float4* c0q = reinterpret_cast<const float4*>(cb0);
      const float4* c1q = reinterpret_cast<const float4*>(cb1);
      float ar[8], br[8], ac[8], bc[8];
      {
        const float4 x0 = c0q[2 * ti], x1 = c0q[2 * ti + 1];
        const float4 y0 = c1q[2 * ti], y1 = c1q[2 * ti + 1];
        const float xa[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        const float ya[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          ar[r] = xa[r];
          br[r] = 8 * ti + r > j + 1 ? fmaf(-xa[r], qi, ya[r]) : 0.f;
        }
      }
      {
        const float4 x0 = c0q[2 * tk], x1 = c0q[2 * tk + 1];
        const float4 y0 = c1q[2 * tk], y1 = c1q[2 * tk + 1];
        const float xa[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        const float ya[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          ac[c] = xa[c] * inv0;
          bc[c] = 8 * tk + c > j + 1 ? fmaf(-xa[c], qi, ya[c]) * inv1 : 0.f;
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) P[r][c] = fmaf(-br[r], bc[c], fmaf(-ar[r], ac[c], P[r][c]));
    }
  }
  if (ti == tk) {
#pragma unroll
    for (int r = 0; r < 8; ++r) piv[8 * ti + r] = sqrtf(P[r][r]);
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int k = 8 * tk + c;
    const float s = 1.f / piv[k];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int i = 8 * ti + r;
      if (i >= k) lt[(size_t)k * PDL_MAXM + i] = P[r][c] * s;
    }
  }
}

// Cholesky factor (FP64) of the SPD matrix M of order m <= 256, m % 16 == 0,
// lower triangle in a[i * lda + k] (i >= k), blocked right-looking in one
// work-group of 256 threads; a is overwritten (it holds the trailing matrix
// between panels). Output lt[k * 256 + i] = L[i][k] and lt2[i * 256 + k] =
// L[i][k] for i >= k. For every panel of 16 columns starting at b0:
//   factor: wave 0 alone, the panel (rows b0 .. m - 1) in registers, lane l
//     holding rows b0 + l + 64 s (s < 4), all 16 columns; the pivot and the
//     column entries of the diagonal block (rows < 16 live in slot 0 of
//     lanes 0 .. 15) are broadcast with readlane, so the 16 steps need no
//     barrier;
//   trailing update: a[i][k] -= sum_c L[i][c] L[k][c] over the panel's
//     columns for b0 + 16 <= k <= i < m, by all four waves in 8 x 8 tiles
//     per thread, the panel read from LDS (column-major).
// Two barriers per panel.
constexpr int PDL_CHOL64_NB = 16;

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__global__ void __launch_bounds__(256)
k_pdl_chol64(double* __restrict__ a, int lda, int m, double* __restrict__ lt,
             double* __restrict__ lt2) {
  constexpr int NB = PDL_CHOL64_NB;
  constexpr int LDP = PDL_MAXM + 8;
  __shared__ __align__(16) double pnT[NB][LDP];   // factored panel, pnT[c][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b0 = 0; b0 < m; b0 += NB) {
    const int nr = m - b0;
    if (wave == 0) {
      // whole rows of 16 entries (two-double vector loads, no per-entry
      // branch); entries above the diagonal and rows beyond nr read as zero
      double v[4][NB];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = lane + 64 * s;
        const double2* src =
            reinterpret_cast<const double2*>(a + (size_t)(b0 + (row < nr ? row : 0)) * lda + b0);
#pragma unroll
        for (int c = 0; c < NB; c += 2) {
          const double2 w = src[c / 2];
          v[s][c] = (row < nr && c <= row) ? w.x : 0.0;
          v[s][c + 1] = (row < nr && c + 1 <= row) ? w.y : 0.0;
        }
      }
      // Rows at or beyond nr hold zeros and stay zero. The updates also run
      // over the diagonal block's upper triangle (row < k), whose entries
      // are never read again (a step reads column j only below the pivot)
      // and are not written out: no per-entry masks in the inner loop.
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double d = sqrt(readlane_f64(v[0][j], j)), inv = 1.0 / d;
        double lj[4];
        lj[0] = lane > j ? v[0][j] * inv : (lane == j ? d : 0.0);
#pragma unroll
        for (int s = 1; s < 4; ++s) lj[s] = v[s][j] * inv;
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s][j] = lj[s];
#pragma unroll
        for (int k = j + 1; k < NB; ++k) {
          const double lkj = readlane_f64(lj[0], k);
#pragma unroll
          for (int s = 0; s < 4; ++s) v[s][k] -= lj[s] * lkj;
        }
      }
      // the panel with zeros above the diagonal: to LDS for the update, to
      // lt by columns and lt2 by rows (the zeros land in entries the solves
      // never read)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = lane + 64 * s;
        if (row < nr) {
          double2* dst2 = reinterpret_cast<double2*>(lt2 + (size_t)(b0 + row) * PDL_MAXM + b0);
#pragma unroll
          for (int c = 0; c < NB; c += 2) {
            const double x0 = c <= row ? v[s][c] : 0.0, x1 = c + 1 <= row ? v[s][c + 1] : 0.0;
            pnT[c][row] = x0;
            pnT[c + 1][row] = x1;
            lt[(size_t)(b0 + c) * PDL_MAXM + b0 + row] = x0;
            lt[(size_t)(b0 + c + 1) * PDL_MAXM + b0 + row] = x1;
            dst2[c / 2] = double2{x0, x1};
          }
        }
      }
    }
    // the update reads the panel from LDS only: an LDS-scoped barrier (the
    // stores of lt and lt2 need not have completed)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    // trailing update of rows and columns b0 + NB .. m - 1 (8 x 8 tiles on
    // and below the diagonal, tile (ti, tk), tk <= ti, numbered row by row)
    const int nt = (nr - NB) / 8;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = tid; t < ntiles; t += 256) {
      int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (ti * (ti + 1) / 2 > t) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      const int tk = t - ti * (ti + 1) / 2;
      const int r0 = NB + 8 * ti, c0 = NB + 8 * tk;   // panel-relative rows
      // the tile of the trailing matrix, loaded before the products (its
      // latency overlaps them); acc starts from it
      double acc[8][8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const double2* src =
            reinterpret_cast<const double2*>(a + (size_t)(b0 + r0 + r) * lda + b0 + c0);
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
          const double2 w = src[c / 2];
          acc[r][c] = w.x;
          acc[r][c + 1] = w.y;
        }
      }
#pragma unroll 2
      for (int q = 0; q < NB; ++q) {
        double x[8], y[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          x[r] = pnT[q][r0 + r];
          y[r] = pnT[q][c0 + r];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int c = 0; c < 8; ++c) acc[r][c] -= x[r] * y[c];
      }
      // whole tile rows back (entries above the diagonal of a diagonal tile
      // are never read again)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        double2* dst = reinterpret_cast<double2*>(a + (size_t)(b0 + r0 + r) * lda + b0 + c0);
#pragma unroll
        for (int c = 0; c < 8; c += 2) dst[c / 2] = double2{acc[r][c], acc[r][c + 1]};
      }
    }
    __syncthreads();   // the next panel reads the updated trailing matrix
  }
}

// LDS floats of k_pdl_trsolve for order m: packed columns of L and 1 / L[k][k]
__host__ __device__ constexpr int pdl_trsolve_lds_floats(int m) { return m * (m + 1) / 2 + m; }

// Rows of X = B M^-1 with M = L L^T (lt from k_pdl_chol, order m): for every
// row b of B, x solves M x^T = b^T (M symmetric): L y = b^T (forward), then
// L^T x = y (backward), both column by column. One row per wave (lane holds
// entries lane + 64 r, r < NR = ceil(m / 64)), four waves per work-group; L
// is staged in LDS as packed columns (column k at offset k m - k (k - 1) / 2,
// entries k..m-1). In each sweep the division by L[k][k] of the entry that
// step k finishes is applied to the broadcast value only, and to the entries
// themselves once at the end (an entry is not read again after its step).
// The solve is bound by instruction issue (one dependent chain per wave):
// the next step's LDS operands are loaded before the current step's
// arithmetic. B entry (row, col) is b[row * bsr + col * bsc]; X is written
// row-major (q x m) to xo (FP32) and/or xbf (BF16) when those are not null.
template <int NR>
__global__ void __launch_bounds__(256)
k_pdl_trsolve(const float* __restrict__ lt, int m, const float* __restrict__ b, int bsr, int bsc,
              int q, float* __restrict__ xo, uint16_t* __restrict__ xbf) {
  extern __shared__ float Lp[];
  float* rd = Lp + m * (m + 1) / 2;
  const int mm = m * m;
  for (int base = 0; base < mm; base += 256 * 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * 256 + threadIdx.x;
      const int k = idx / m, i = idx - k * m;
      v[u] = (idx < mm && i >= k) ? lt[(size_t)k * PDL_MAXM + i] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * 256 + threadIdx.x;
      const int k = idx / m, i = idx - k * m;
      if (idx < mm && i >= k) Lp[k * m - k * (k - 1) / 2 + (i - k)] = v[u];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += 256) rd[k] = 1.f / Lp[k * m - k * (k - 1) / 2];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= q) return;
  float y[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int c = lane + 64 * r;
    y[r] = c < m ? b[(size_t)row * bsr + (size_t)c * bsc] : 0.f;
  }
  // entry k lives in slot k / 64 of lane k % 64: the sweeps run over the
  // 64-entry blocks with the slot a compile-time index (a runtime slot index
  // would put y in scratch memory)
  auto scale = [&]() {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      if (i < m) y[r] *= rd[i];
    }
  };
  // forward: L y = b; column k of L at col(k)[i], i >= k (zero for i <= k)
  auto colv = [&](int k, float (&v)[NR], float& rk) {
    const float* col = Lp + k * m - k * (k - 1) / 2 - k;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      v[r] = (i > k && i < m) ? col[i] : 0.f;
    }
    rk = rd[k];
  };
  float cv[NR], rk;
  colv(0, cv, rk);
#pragma unroll
  for (int rb = 0; rb < NR; ++rb) {
    const int kend = m < 64 * (rb + 1) ? m : 64 * (rb + 1);
    for (int k = 64 * rb; k < kend; ++k) {
      float nv[NR], nr = 0.f;
      if (k + 1 < m) colv(k + 1, nv, nr);
      const float yk =
          __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y[rb]), k & 63)) * rk;
#pragma unroll
      for (int r = 0; r < NR; ++r) y[r] = fmaf(-cv[r], yk, y[r]);
#pragma unroll
      for (int r = 0; r < NR; ++r) cv[r] = nv[r];
      rk = nr;
    }
  }
  scale();
  // backward: L^T x = y; row k of L (entries i < k) at Lp[i m - i (i - 1) / 2 + k - i]
  auto rowv = [&](int k, float (&v)[NR], float& rkk) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      v[r] = i < k ? Lp[i * m - i * (i - 1) / 2 + (k - i)] : 0.f;
    }
    rkk = rd[k];
  };
  rowv(m - 1, cv, rk);
#pragma unroll
  for (int rb = NR - 1; rb >= 0; --rb) {
    const int kbeg = m - 1 < 64 * rb + 63 ? m - 1 : 64 * rb + 63;
    for (int k = kbeg; k >= 64 * rb; --k) {
      float nv[NR], nr = 0.f;
      if (k > 0) rowv(k - 1, nv, nr);
      const float xk =
          __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y[rb]), k & 63)) * rk;
#pragma unroll
      for (int r = 0; r < NR; ++r) y[r] = fmaf(-cv[r], xk, y[r]);
#pragma unroll
      for (int r = 0; r < NR; ++r) cv[r] = nv[r];
      rk = nr;
    }
  }
  scale();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int c = lane + 64 * r;
    if (c < m) {
      if (xo) xo[(size_t)row * m + c] = y[r];
      if (xbf) xbf[(size_t)row * m + c] = f2bf(y[r]);
    }
  }
}

// Rows of X = B M^-1 with M = L L^T in FP64 (order m, a multiple of 64, at
// most 256): lt holds L by columns (lt[k * 256 + i] = L[i][k]), lt2 by rows
// (lt2[i * 256 + k] = L[i][k]), both from k_pdl_chol<double>. For every row
// b of B (n x m, row-major), L y = b^T (forward, column by column), then
// L^T x = y (backward, row by row of L). One row per wave, entry c in slot
// c / 64 of lane c % 64; the column (row) of L that step k needs is read
// from global memory, PF steps ahead of its use, through a ring of
// registers, and y_k is broadcast from its lane by two readlanes.
template <int NR>
__global__ void __launch_bounds__(256)
k_pdl_trsolve64(const double* __restrict__ lt, const double* __restrict__ lt2, int m,
                const double* __restrict__ b, int q, double* __restrict__ xo) {
  constexpr int PF = 8;
  __shared__ double rd[PDL_MAXM];
  for (int k = threadIdx.x; k < m; k += 256) rd[k] = 1.0 / lt[(size_t)k * PDL_MAXM + k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= q) return;
  double y[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int c = lane + 64 * r;
    y[r] = c < m ? b[(size_t)row * m + c] : 0.0;
  }
  auto bcast = [&](double v, int l) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
  };
  // forward: y_i -= L[i][k] y_k / L[k][k] for i > k, then y_k /= L[k][k]
  // (the division of the finished entry is applied to the broadcast value
  // only, and to the entries once at the end)
  double ring[PF][NR];
  auto colv = [&](int k, double (&v)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      v[r] = (k < m && i > k && i < m) ? lt[(size_t)k * PDL_MAXM + i] : 0.0;
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) colv(u, ring[u]);
#pragma unroll
  for (int rb = 0; rb < NR; ++rb) {
#pragma unroll 1
    for (int k0 = 64 * rb; k0 < 64 * rb + 64 && k0 < m; k0 += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int k = k0 + u;
        const double yk = bcast(y[rb], k & 63) * rd[k];
#pragma unroll
        for (int r = 0; r < NR; ++r) y[r] -= ring[u][r] * yk;
        colv(k + PF, ring[u]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = lane + 64 * r;
    if (i < m) y[r] *= rd[i];
  }
  // backward: x_i -= L[k][i] x_k / L[k][k] for i < k, k from m - 1 down
  auto rowv = [&](int k, double (&v)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = lane + 64 * r;
      v[r] = (k >= 0 && i < k) ? lt2[(size_t)k * PDL_MAXM + i] : 0.0;
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) rowv(m - 1 - u, ring[u]);
#pragma unroll
  for (int rb = NR - 1; rb >= 0; --rb) {
    if (64 * rb >= m) continue;
#pragma unroll 1
    for (int k0 = 64 * rb + 63; k0 >= 64 * rb; k0 -= PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int k = k0 - u;
        const double xk = bcast(y[rb], k & 63) * rd[k];
#pragma unroll
        for (int r = 0; r < NR; ++r) y[r] -= ring[u][r] * xk;
        rowv(k - PF, ring[u]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int c = lane + 64 * r;
    if (c < m) xo[(size_t)row * m + c] = y[r] * rd[c];
  }
}

// G = (D + E) / ||D + E||_F, E <- E + D - G from the FP64 D, G and E stored
// in FP32 and G in BF16 (count = n A entries, one work-group of 1024
// threads; the squared norm is summed in FP64 in a fixed order). res (optional, a check of the dictionary penalty):
// res[0] = ||D - G||^2, res[1] = ||G - G_prev||^2 in FP64.
__global__ void __launch_bounds__(1024)
k_pdl_project(const double* __restrict__ d, float* __restrict__ g, float* __restrict__ e,
              uint16_t* __restrict__ gbf, int count, double* __restrict__ res) {
  __shared__ double red[16], red2[2][16];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    const double w = (double)d[i] + (double)e[i];
    s += w * w;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) tot += red[k];
  const double inv = 1.0 / sqrt(tot);
  double rd = 0.0, sd = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    const double dv = (double)d[i], ev = (double)e[i];
    const double gd = (dv + ev) * inv;
    const float gv = (float)gd;
    if (res) {
      const double a = gd - dv, b = gd - (double)g[i];
      rd += a * a;
      sd += b * b;
    }
    g[i] = gv;
    e[i] = (float)(ev + dv - gd);
    gbf[i] = f2bf(gv);
  }
  if (res) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      rd += __shfl_down(rd, off, 64);
      sd += __shfl_down(sd, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red2[0][threadIdx.x >> 6] = rd;
      red2[1][threadIdx.x >> 6] = sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        a += red2[0][k];
        b += red2[1][k];
      }
      res[0] = a;
      res[1] = b;
    }
  }
}

// E <- c E (count entries): a change sigma -> sigma' of the dictionary
// penalty rescales the scaled dual by c = sigma / sigma'.
__global__ void k_pdl_scale(float* __restrict__ e, int count, float c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) e[i] *= c;
}

// cm[i * 256 + k] = rho [i == k] + sum_a G[i][a] G[k][a] for i >= k
// (G: n x A row-major); 16 x 16 output tiles, grid (n / 16, n / 16).
__global__ void __launch_bounds__(256)
k_pdl_gram(const float* __restrict__ g, int NA, float rho, float* __restrict__ cm) {
  __shared__ float Ga[16][17], Gb[16][17];
  const int bi = blockIdx.y, bk = blockIdx.x;
  if (bk > bi) return;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc = 0.f;
  for (int a0 = 0; a0 < NA; a0 += 16) {
    Ga[ty][tx] = g[(size_t)(16 * bi + ty) * NA + a0 + tx];
    Gb[ty][tx] = g[(size_t)(16 * bk + ty) * NA + a0 + tx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc = fmaf(Ga[ty][q], Gb[tx][q], acc);
    __syncthreads();
  }
  const int i = 16 * bi + ty, k = 16 * bk + tx;
  if (i >= k) cm[(size_t)i * PDL_MAXM + k] = acc + (i == k ? rho : 0.f);
}

// Start of a solve: G = D0, E = 0 (count entries).
__global__ void k_pdl_start(const float* __restrict__ d0, float* __restrict__ g,
                            float* __restrict__ e, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    g[i] = d0[i];
    e[i] = 0.f;
  }
}

}  // namespace cip
