// Patch-dictionary synthesis prior (Eq. patch_based), sparse-code update of
// Algorithm 2 on MFMA (gfx950 v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Geometry: Q x Q x S patches (Q = 8) spanning all planes, extracted
// circularly at stride st = 4 (P^T P = 4 I). Patch vector element
// s*64 + a*8 + b of patch (pi, pj) is x[s][4 pi + a][4 pj + b]; the patch
// index is j = pi * J2 + pj with J1 = N1 / 4, J2 = N2 / 4. A work-group owns a
// tile of 64 patches, TPR x TPC (TPC = min(64, J2)).
//
// Per tile, with the ADMM state v = z + u_prev (t = soft(v), u = clip(v),
// w = t - u = 2 soft(v) - v, all as in the analysis passes):
//   GEMM1  e  = P_j x - D w            (n x 64,  K = A)
//   GEMM2  z  = w + M1 e,  M1 = D^T (rho I + D D^T)^-1   (A x 64, K = n)
//          v <- z + clip(v)            (soft threshold + dual, Eq. softADMM)
//   GEMM3  D z                         (n x 64,  K = A)
// z = w + M1 (P x - D w) equals Eq. solz_patch2,
// (rho I + D^T D)^-1 (D^T P x + rho w), by the push-through identity; it never
// forms the badly conditioned (rho I + D^T D)^-1 and its correction term is
// small, which suits BF16 operands. D z of the 64 patches is overlap-added
// inside the tile (fixed summation order) and written to a per-tile buffer;
// k_patch_assemble sums the (at most 4) tiles covering each pixel, giving
// P^T D~ z for the next x-update (Eq. solx_synt) without atomics.
#pragma once
#include "kernels.hpp"

namespace cip {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int PATCH_Q = 8;
constexpr int PATCH_ST = 4;
constexpr int PATCH_NP = 64;   // patches per work-group tile

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t* p) {
  uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}

struct PatchGeo {
  int N1, N2, J1, J2, TPR, TPC, ntc, RR, RC;
};

__host__ __device__ inline PatchGeo patch_geo(int N1, int N2) {
  PatchGeo g;
  g.N1 = N1;
  g.N2 = N2;
  g.J1 = N1 / PATCH_ST;
  g.J2 = N2 / PATCH_ST;
  g.TPC = g.J2 < PATCH_NP ? g.J2 : PATCH_NP;
  g.TPR = PATCH_NP / g.TPC;
  g.ntc = g.J2 / g.TPC;
  g.RR = PATCH_ST * g.TPR + (PATCH_Q - PATCH_ST);
  g.RC = PATCH_ST * g.TPC + (PATCH_Q - PATCH_ST);
  return g;
}

// LDS bytes of k_patch_z
template <int S, int NA> constexpr int patch_lds_bytes() {
  constexpr int NV = 64 * S;
  constexpr int wb = PATCH_NP * (NA + 8) * 2;
  constexpr int eb = PATCH_NP * (NV + 8) * 2;
  constexpr int dz = PATCH_NP * NV * 4;
  return wb + eb > dz ? wb + eb : dz;
}

// What k_patch_z runs: the whole update (codes, state, D z), only the codes
// and state (z also written in FP32 to zf), or only D z from the codes in zf
// (after a dictionary change).
enum { PZ_FULL = 0, PZ_CODES = 1, PZ_SYNTH = 2 };

// Sparse-code update for one tile of 64 patches per work-group (4 waves).
//   x   [S][N1][N2]  current image x^{l+1}
//   v   [NA][J]      state, updated in place (first: treated as 0)
//   tb  per-tile overlap-added D z, [tile][S][RR][RC]
//   Dg  [NV][NA] bf16, M1g [NA][NV] bf16 (row-major)
//   zf  [NA][J]      codes z in FP32 (PZ_CODES: written; PZ_SYNTH: read)
template <int S, int NA, int MODE>
__global__ void __launch_bounds__(256)
k_patch_z(const float* __restrict__ x, float* __restrict__ v, float* __restrict__ tb,
          const uint16_t* __restrict__ Dg, const uint16_t* __restrict__ M1g, PatchGeo G,
          float kappa, int first, float* __restrict__ zf) {
  constexpr int NV = 64 * S;
  constexpr int WS = NA + 8;   // LDS row stride of W / Z (bf16)
  constexpr int ES = NV + 8;   // LDS row stride of E (bf16)
  static_assert(NA % 64 == 0, "atoms must be a multiple of 64");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* WB = reinterpret_cast<uint16_t*>(smem_raw);
  uint16_t* EB = WB + PATCH_NP * WS;
  float* DZ = reinterpret_cast<float*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l32 = lane & 31, lhi = lane >> 5;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tr = tile / G.ntc, tc = tile % G.ntc;
  const size_t J = (size_t)G.J1 * G.J2;
  auto jglob = [&](int jl) -> size_t {
    return (size_t)(tr * G.TPR + jl / G.TPC) * G.J2 + tc * G.TPC + jl % G.TPC;
  };

  if constexpr (MODE == PZ_SYNTH) {
    // codes from zf, as bf16 rows WB[patch][atom]
    for (int idx = threadIdx.x; idx < NA * PATCH_NP; idx += 256) {
      const int a = idx / PATCH_NP, jl = idx % PATCH_NP;
      WB[jl * WS + a] = f2bf(zf[(size_t)a * J + jglob(jl)]);
    }
    __syncthreads();
  } else {
    // 0. w = t - u = 2 soft(v) - v, as bf16 rows WB[patch][atom]
    for (int idx = threadIdx.x; idx < NA * PATCH_NP; idx += 256) {
      const int a = idx / PATCH_NP, jl = idx % PATCH_NP;
      const float vv = first ? 0.f : v[(size_t)a * J + jglob(jl)];
      WB[jl * WS + a] = f2bf(2.f * soft_f(vv, kappa) - vv);
    }
    __syncthreads();

    // 1. GEMM1: acc = D w; epilogue e = P x - D w -> EB[patch][i]
    if (wave < NV / 64) {
      f32x16 acc[2][2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = f32x16{};
      // the patch samples of the epilogue are loaded first (latency overlaps the products)
      float xp[2][2][16];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int jl = 32 * n + l32;
          const int pr0 = (tr * G.TPR + jl / G.TPC) * PATCH_ST;
          const int pc0 = (tc * G.TPC + jl % G.TPC) * PATCH_ST;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int row = 64 * wave + 32 * m + 8 * (i / 4) + 4 * lhi + (i % 4);
            const int s = row >> 6, a = (row >> 3) & 7, b = row & 7;
            const int pr = (pr0 + a) & (G.N1 - 1), pc = (pc0 + b) & (G.N2 - 1);
            xp[m][n][i] = x[((size_t)s * G.N1 + pr) * G.N2 + pc];
          }
        }
      const uint16_t* Da = Dg + (size_t)(64 * wave + l32) * NA + 8 * lhi;
#pragma unroll 4
      for (int ks = 0; ks < NA / 16; ++ks) {
        bf16x8 a0 = ld_bf16x8(Da + 16 * ks);
        bf16x8 a1 = ld_bf16x8(Da + 32 * NA + 16 * ks);
        bf16x8 b0 = ld_bf16x8(WB + l32 * WS + 16 * ks + 8 * lhi);
        bf16x8 b1 = ld_bf16x8(WB + (32 + l32) * WS + 16 * ks + 8 * lhi);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int jl = 32 * n + l32;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int row = 64 * wave + 32 * m + 8 * (i / 4) + 4 * lhi + (i % 4);
            EB[jl * ES + row] = f2bf(xp[m][n][i] - acc[m][n][i]);
          }
        }
    }
    __syncthreads();

    // 2. GEMM2: acc = M1 e; z = w + acc; v <- z + clip(v); z -> WB (bf16)
    for (int wb = wave; wb < NA / 64; wb += 4) {
      f32x16 acc[2][2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = f32x16{};
      // the state of the epilogue is loaded first (latency overlaps the products)
      float vs[2][2][16];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const size_t jg = jglob(32 * n + l32);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int atom = 64 * wb + 32 * m + 8 * (i / 4) + 4 * lhi + (i % 4);
            vs[m][n][i] = first ? 0.f : v[(size_t)atom * J + jg];
          }
        }
      const uint16_t* Ma = M1g + (size_t)(64 * wb + l32) * NV + 8 * lhi;
#pragma unroll 4
      for (int ks = 0; ks < NV / 16; ++ks) {
        bf16x8 a0 = ld_bf16x8(Ma + 16 * ks);
        bf16x8 a1 = ld_bf16x8(Ma + 32 * NV + 16 * ks);
        bf16x8 b0 = ld_bf16x8(EB + l32 * ES + 16 * ks + 8 * lhi);
        bf16x8 b1 = ld_bf16x8(EB + (32 + l32) * ES + 16 * ks + 8 * lhi);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int jl = 32 * n + l32;
          const size_t jg = jglob(jl);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int atom = 64 * wb + 32 * m + 8 * (i / 4) + 4 * lhi + (i % 4);
            const float vv = vs[m][n][i];
            const float z = (2.f * soft_f(vv, kappa) - vv) + acc[m][n][i];
            v[(size_t)atom * J + jg] = z + clip_f(vv, kappa);
            WB[jl * WS + atom] = f2bf(z);
            if constexpr (MODE == PZ_CODES) zf[(size_t)atom * J + jg] = z;
          }
        }
    }
    if constexpr (MODE == PZ_CODES) return;
    __syncthreads();
  }

  // 3. GEMM3: D z, then overlap-add inside the tile
  f32x16 acc3[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc3[m][n] = f32x16{};
  if (wave < NV / 64) {
    const uint16_t* Da = Dg + (size_t)(64 * wave + l32) * NA + 8 * lhi;
#pragma unroll 4
    for (int ks = 0; ks < NA / 16; ++ks) {
      bf16x8 a0 = ld_bf16x8(Da + 16 * ks);
      bf16x8 a1 = ld_bf16x8(Da + 32 * NA + 16 * ks);
      bf16x8 b0 = ld_bf16x8(WB + l32 * WS + 16 * ks + 8 * lhi);
      bf16x8 b1 = ld_bf16x8(WB + (32 + l32) * WS + 16 * ks + 8 * lhi);
      acc3[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc3[0][0], 0, 0, 0);
      acc3[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc3[0][1], 0, 0, 0);
      acc3[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc3[1][0], 0, 0, 0);
      acc3[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc3[1][1], 0, 0, 0);
    }
  }
  __syncthreads();   // WB / EB are reused as DZ below
  if (wave < NV / 64) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int jl = 32 * n + l32;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = 64 * wave + 32 * m + 8 * (i / 4) + 4 * lhi + (i % 4);
          DZ[jl * NV + row] = acc3[m][n][i];
        }
      }
  }
  __syncthreads();
  // tile region S x RR x RC: every pixel sums its (<= 4) patches in a fixed order
  const int RA = G.RR * G.RC;
  float* out = tb + (size_t)tile * S * RA;
  for (int idx = threadIdx.x; idx < S * RA; idx += 256) {
    const int s = idx / RA, rem = idx % RA, rr = rem / G.RC, cc = rem % G.RC;
    float sum = 0.f;
#pragma unroll
    for (int da = 1; da >= 0; --da) {
      const int ar = rr / PATCH_ST - da;
      if (ar < 0 || ar >= G.TPR) continue;
      const int a = rr - PATCH_ST * ar;
      if (a >= PATCH_Q) continue;
#pragma unroll
      for (int db = 1; db >= 0; --db) {
        const int ac = cc / PATCH_ST - db;
        if (ac < 0 || ac >= G.TPC) continue;
        const int b = cc - PATCH_ST * ac;
        if (b >= PATCH_Q) continue;
        sum += DZ[(ar * G.TPC + ac) * NV + s * 64 + a * 8 + b];
      }
    }
    out[idx] = sum;
  }
}

// r = P^T D~ z: every pixel sums the tiles whose regions cover it (its own
// tile and, within Q - st pixels of a tile edge, the previous tile along that
// axis, circularly), in a fixed order.
// Thread (C, R, s) of a 3D grid (no index division).
__global__ void k_patch_assemble(const float* __restrict__ tb, float* __restrict__ r, int S,
                                 PatchGeo G) {
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= G.N2) return;
  const int R = blockIdx.y, s = blockIdx.z;
  const size_t idx = ((size_t)s * G.N1 + R) * G.N2 + C;
  const int TH = PATCH_ST * G.TPR, TW = PATCH_ST * G.TPC;
  const int ntr = G.J1 / G.TPR;
  const int RA = G.RR * G.RC;
  const int tr0 = R / TH, lr0 = R - tr0 * TH;
  const int tc0 = C / TW, lc0 = C - tc0 * TW;
  float sum = 0.f;
#pragma unroll
  for (int dr = 0; dr < 2; ++dr) {
    if (dr == 1 && lr0 >= PATCH_Q - PATCH_ST) break;
    const int tr = dr ? (tr0 + ntr - 1) % ntr : tr0;
    const int lr = dr ? lr0 + TH : lr0;
#pragma unroll
    for (int dc = 0; dc < 2; ++dc) {
      if (dc == 1 && lc0 >= PATCH_Q - PATCH_ST) break;
      const int tc = dc ? (tc0 + G.ntc - 1) % G.ntc : tc0;
      const int lc = dc ? lc0 + TW : lc0;
      const size_t t = (size_t)tr * G.ntc + tc;
      sum += tb[(t * S + s) * RA + lr * G.RC + lc];
    }
  }
  r[idx] = sum;
}

}  // namespace cip
