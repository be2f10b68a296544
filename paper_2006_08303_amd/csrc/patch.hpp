// Patch-dictionary synthesis prior (Eq. patch_based), sparse-code update of
// Algorithm 2 on MFMA (gfx950 v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Geometry: Q x Q x S patches (Q = 8) spanning all planes, extracted
// circularly at stride st = 4 (P^T P = 4 I). Patch vector element
// s*64 + a*8 + b of patch (pi, pj) is x[s][4 pi + a][4 pj + b]; the patch
// index is j = pi * J2 + pj with J1 = N1 / 4, J2 = N2 / 4. A work-group owns a
// tile of 64 patches, TPR x TPC (TPC = min(64, J2)); with this ordering the
// tile's patches are the 64 consecutive indices 64 tile .. 64 tile + 63.
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
// small, which suits BF16 operands. Each GEMM's rows are split evenly over
// the 4 waves (16-row MFMA blocks), every wave covering all 64 patches. D z of
// the 64 patches is overlap-added inside the tile (fixed summation order)
// and written to a per-tile buffer; k_patch_assemble sums the (at most 4)
// tiles covering each pixel, giving P^T D~ z for the next x-update
// (Eq. solx_synt) without atomics.
//
// The state v is stored patch-major, [J][A] (the A codes of a patch are
// contiguous), so a tile's state is one contiguous block and every thread
// moves four codes of one patch at a time.
#pragma once
#include "kernels.hpp"

namespace cip {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

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
  int ltpc;   // log2(TPC)
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
  g.ltpc = 0;
  while ((1 << g.ltpc) < g.TPC) ++g.ltpc;
  return g;
}

// LDS of k_patch_z: one region holding in turn WB [64][NA + 8] bf16 (w),
// EB [64][NV + 8] bf16 (e) and WB again (z), the B operands of the three
// products (rows 16-byte aligned, the pad spreads consecutive patches over
// the banks), and finally DZ [64][NV + 4] float (D z of every patch). At
// S = 3, A = 256 that is 50 KB, three work-groups per CU.
template <int S, int NA> constexpr int patch_lds_bytes() {
  constexpr int NV = 64 * S;
  constexpr int wb = PATCH_NP * (NA + 8) * 2;
  constexpr int eb = PATCH_NP * (NV + 8) * 2;
  constexpr int dz = PATCH_NP * (NV + 4) * 4;
  constexpr int m = wb > eb ? wb : eb;
  return m > dz ? m : dz;
}

// What k_patch_z runs: the whole update (codes, state, D z), only the codes
// and state (z also written in FP32 to zf), or only D z from the codes in zf
// (after a dictionary change).
enum { PZ_FULL = 0, PZ_CODES = 1, PZ_SYNTH = 2 };

__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
  const bf16x4 h = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};   // round to nearest even
  return __builtin_bit_cast(uint2, h);
}

// One product C (RB blocks of 16 rows of A, all 64 patches) += A B over K:
// A rows from global memory (bf16, row stride K; the dictionary tables stay
// in L2), B from LDS (patch rows of stride BS, K contiguous). Lane l holds A
// row (l % 16) and B column (l % 16) at k = 8 (l / 16) .. + 7 of every
// 32-wide k step; C block (rb, cb) holds rows 4 (l / 16) + i (i < 4) of
// column l % 16. The A operands are loaded PF k steps ahead (a ring of
// PF + 1 register sets) so that the L2 latency overlaps the products.
template <int RB, int K, int BS>
__device__ __forceinline__ void patch_mfma(f32x4 (&acc)[RB][4], const uint16_t* __restrict__ A,
                                           const uint16_t* B, int c16, int q4) {
  constexpr int KS = K / 32;
  constexpr int PF = KS < 2 ? KS : 2;
  const uint16_t* Ar = A + (size_t)c16 * K + 8 * q4;
  const uint16_t* Br = B + c16 * BS + 8 * q4;
  bf16x8 a[PF + 1][RB];
#pragma unroll
  for (int p = 0; p < PF; ++p)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[p][rb] = ld_bf16x8(Ar + (size_t)rb * 16 * K + 32 * p);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    if (ks + PF < KS) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        a[(ks + PF) % (PF + 1)][rb] = ld_bf16x8(Ar + (size_t)rb * 16 * K + 32 * (ks + PF));
    }
    bf16x8 b[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) b[cb] = ld_bf16x8(Br + cb * 16 * BS + 32 * ks);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[rb][cb] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks % (PF + 1)][rb], b[cb], acc[rb][cb], 0, 0, 0);
  }
}

// Sparse-code update for one tile of 64 patches per work-group (4 waves).
//   x   [S][N1][N2]  current image x^{l+1}
//   v   [J][NA]      state, updated in place (first: treated as 0)
//   tb  per-tile overlap-added D z, [tile][S][RR][RC]
//   Dg  [NV][NA] bf16, M1g [NA][NV] bf16 (row-major)
//   zf  [NA][J]      codes z in FP32 (PZ_CODES: written; PZ_SYNTH: read)
//   rs  when not null (adaptive penalty, Section IV-C): every wave writes
//       rs[2 (4 tile + wave)] = sum (z - t)^2 and rs[... + 1] =
//       sum (t - t_prev)^2 over its codes, t = soft(v_new), t_prev = soft(v)
template <int S, int NA, int MODE>
__global__ void __launch_bounds__(256, 2)
k_patch_z(const float* __restrict__ x, float* __restrict__ v, float* __restrict__ tb,
          const uint16_t* __restrict__ Dg, const uint16_t* __restrict__ M1g, PatchGeo G,
          float kappa, int first, float* __restrict__ zf, float* __restrict__ rs) {
  constexpr int NV = 64 * S;
  constexpr int WS = NA + 8;   // LDS row stride of W / Z (bf16)
  constexpr int ES = NV + 8;   // LDS row stride of E (bf16)
  constexpr int DS = NV + 4;   // LDS row stride of DZ (float)
  constexpr int RB1 = NV / 64;   // 16-row blocks per wave of the n x 64 products
  constexpr int RB2 = NA / 64;   // 16-row blocks per wave of the A x 64 product
  static_assert(NA % 64 == 0, "atoms must be a multiple of 64");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint16_t* WB = reinterpret_cast<uint16_t*>(smem_raw);
  uint16_t* EB = WB;   // e replaces w once every wave has finished GEMM1
  float* DZ = reinterpret_cast<float*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, q4 = lane >> 4;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tr = tile / G.ntc, tc = tile - tr * G.ntc;
  const size_t J = (size_t)G.J1 * G.J2;
  const size_t j0 = (size_t)tile * PATCH_NP;   // first patch of the tile
  float* vt = v + j0 * NA;                     // the tile's state block [64][NA]

  if constexpr (MODE == PZ_SYNTH) {
    // codes from zf, as bf16 rows WB[patch][atom] (lanes over patches: the
    // zf reads are contiguous)
    constexpr int NIT = PATCH_NP * NA / 4 / 256;
    float zl[NIT][4];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = threadIdx.x + 256 * k;
      const int jl = it & (PATCH_NP - 1), a = 4 * (it >> 6);
      const float* zp = zf + (size_t)a * J + j0 + jl;
      zl[k][0] = zp[0];
      zl[k][1] = zp[J];
      zl[k][2] = zp[2 * J];
      zl[k][3] = zp[3 * J];
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = threadIdx.x + 256 * k;
      const int jl = it & (PATCH_NP - 1), a = 4 * (it >> 6);
      *reinterpret_cast<uint2*>(WB + jl * WS + a) =
          pack_bf16x4(zl[k][0], zl[k][1], zl[k][2], zl[k][3]);
    }
    __syncthreads();
  } else {
    // 0. w = t - u = 2 soft(v) - v, as bf16 rows WB[patch][atom]; every
    // thread's state loads are issued before the first conversion
    constexpr int NIT = PATCH_NP * NA / 4 / 256;
    float4 vl[NIT];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = threadIdx.x + 256 * k;
      const int jl = it / (NA / 4), a = 4 * (it % (NA / 4));
      vl[k] = first ? float4{0.f, 0.f, 0.f, 0.f}
                    : *reinterpret_cast<const float4*>(vt + jl * NA + a);
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int it = threadIdx.x + 256 * k;
      const int jl = it / (NA / 4), a = 4 * (it % (NA / 4));
      const float4 vv = vl[k];
      *reinterpret_cast<uint2*>(WB + jl * WS + a) =
          pack_bf16x4(2.f * soft_f(vv.x, kappa) - vv.x, 2.f * soft_f(vv.y, kappa) - vv.y,
                      2.f * soft_f(vv.z, kappa) - vv.z, 2.f * soft_f(vv.w, kappa) - vv.w);
    }
    // the patch samples of the epilogue, issued before the products: rows
    // r0 .. r0 + 3 of a block are pixels (s, a, b0 .. b0 + 3) of one patch row,
    // four consecutive floats of x (b0 is 0 or 4, columns stay 16-byte aligned)
    float4 xp[RB1][4];
#pragma unroll
    for (int rb = 0; rb < RB1; ++rb) {
      const int r0 = 16 * (RB1 * wave + rb) + 4 * q4;
      const int s = r0 >> 6, a = (r0 >> 3) & 7, b0 = r0 & 7;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int jl = 16 * cb + c16;
        const int pr = (PATCH_ST * (tr * G.TPR + (jl >> G.ltpc)) + a) & (G.N1 - 1);
        const int pc = (PATCH_ST * (tc * G.TPC + (jl & (G.TPC - 1))) + b0) & (G.N2 - 1);
        xp[rb][cb] = *reinterpret_cast<const float4*>(x + ((size_t)s * G.N1 + pr) * G.N2 + pc);
      }
    }
    __syncthreads();

    // 1. GEMM1: acc = D w; epilogue e = P x - D w -> EB[patch][row]
    {
      f32x4 acc[RB1][4];
#pragma unroll
      for (int rb = 0; rb < RB1; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f32x4{};
      patch_mfma<RB1, NA, WS>(acc, Dg + (size_t)16 * RB1 * wave * NA, WB, c16, q4);
      __syncthreads();   // every wave has read w: e overwrites it
#pragma unroll
      for (int rb = 0; rb < RB1; ++rb) {
        const int r0 = 16 * (RB1 * wave + rb) + 4 * q4;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int jl = 16 * cb + c16;
          const float4 p = xp[rb][cb];
          const f32x4 d = acc[rb][cb];
          *reinterpret_cast<uint2*>(EB + jl * ES + r0) =
              pack_bf16x4(p.x - d[0], p.y - d[1], p.z - d[2], p.w - d[3]);
        }
      }
    }
    __syncthreads();

    // 2. GEMM2: acc = M1 e; z = w + acc; v <- z + clip(v); z -> WB (bf16)
    {
      // the state of the epilogue, issued before the products
      float4 vs[RB2][4];
#pragma unroll
      for (int rb = 0; rb < RB2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int a0 = 16 * (RB2 * wave + rb) + 4 * q4, jl = 16 * cb + c16;
          vs[rb][cb] = first ? float4{0.f, 0.f, 0.f, 0.f}
                             : *reinterpret_cast<const float4*>(vt + jl * NA + a0);
        }
      f32x4 acc[RB2][4];
#pragma unroll
      for (int rb = 0; rb < RB2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f32x4{};
      patch_mfma<RB2, NV, ES>(acc, M1g + (size_t)16 * RB2 * wave * NV, EB, c16, q4);
      __syncthreads();   // every wave has read e: z overwrites it
      float r2 = 0.f, s2 = 0.f;   // residual sums of the adaptive penalty
#pragma unroll
      for (int rb = 0; rb < RB2; ++rb) {
        const int a0 = 16 * (RB2 * wave + rb) + 4 * q4;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int jl = 16 * cb + c16;
          const float4 vv = vs[rb][cb];
          const f32x4 m = acc[rb][cb];
          float4 z, vn;
          z.x = (2.f * soft_f(vv.x, kappa) - vv.x) + m[0];
          z.y = (2.f * soft_f(vv.y, kappa) - vv.y) + m[1];
          z.z = (2.f * soft_f(vv.z, kappa) - vv.z) + m[2];
          z.w = (2.f * soft_f(vv.w, kappa) - vv.w) + m[3];
          vn.x = z.x + clip_f(vv.x, kappa);
          vn.y = z.y + clip_f(vv.y, kappa);
          vn.z = z.z + clip_f(vv.z, kappa);
          vn.w = z.w + clip_f(vv.w, kappa);
          *reinterpret_cast<float4*>(vt + jl * NA + a0) = vn;
          *reinterpret_cast<uint2*>(WB + jl * WS + a0) = pack_bf16x4(z.x, z.y, z.z, z.w);
          if (rs) {
            const float zz[4] = {z.x, z.y, z.z, z.w}, nn[4] = {vn.x, vn.y, vn.z, vn.w},
                        oo[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float tn = soft_f(nn[i], kappa), tp = soft_f(oo[i], kappa);
              r2 += (zz[i] - tn) * (zz[i] - tn);
              s2 += (tn - tp) * (tn - tp);
            }
          }
          if constexpr (MODE == PZ_CODES) {
            float* zp = zf + (size_t)a0 * J + j0 + jl;
            zp[0] = z.x;
            zp[J] = z.y;
            zp[2 * J] = z.z;
            zp[3 * J] = z.w;
          }
        }
      }
      if (rs) {   // wave sums in a fixed order, one pair per wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          r2 += __shfl_xor(r2, off, 64);
          s2 += __shfl_xor(s2, off, 64);
        }
        if (lane == 0) {
          rs[2 * (4 * tile + wave)] = r2;
          rs[2 * (4 * tile + wave) + 1] = s2;
        }
      }
    }
    if constexpr (MODE == PZ_CODES) return;
    __syncthreads();
  }

  // 3. GEMM3: D z, then overlap-add inside the tile
  {
    f32x4 acc[RB1][4];
#pragma unroll
    for (int rb = 0; rb < RB1; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f32x4{};
    patch_mfma<RB1, NA, WS>(acc, Dg + (size_t)16 * RB1 * wave * NA, WB, c16, q4);
    __syncthreads();   // WB / EB are reused as DZ below
#pragma unroll
    for (int rb = 0; rb < RB1; ++rb) {
      const int r0 = 16 * (RB1 * wave + rb) + 4 * q4;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int jl = 16 * cb + c16;
        const f32x4 d = acc[rb][cb];
        *reinterpret_cast<float4*>(DZ + jl * DS + r0) = float4{d[0], d[1], d[2], d[3]};
      }
    }
  }
  __syncthreads();
  // tile region S x RR x RC: every pixel sums its (<= 4) patches in a fixed
  // order (patch row rr / 4 - 1 before rr / 4, patch column cc / 4 - 1
  // before cc / 4). One region row per wave at a time (the patch rows are
  // then wave-uniform); each lane forms four consecutive pixels 4 c4 ..
  // 4 c4 + 3, which share their patches: columns 4..7 of patch c4 - 1 and
  // 0..3 of patch c4, one float4 each.
  const int RR = G.RR, RC = G.RC;
  float* out = tb + (size_t)tile * S * RR * RC;
  for (int row = wave; row < S * RR; row += 4) {
    const int s = row / RR, rr = row - s * RR;
    for (int c4 = lane; c4 < RC / 4; c4 += 64) {
      float4 sum = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int da = 1; da >= 0; --da) {
        const int ar = (rr >> 2) - da;
        const int a = rr - PATCH_ST * ar;
        if (ar < 0 || ar >= G.TPR || a >= PATCH_Q) continue;
#pragma unroll
        for (int db = 1; db >= 0; --db) {
          const int ac = c4 - db;
          if (ac < 0 || ac >= G.TPC) continue;
          const float4 q = *reinterpret_cast<const float4*>(
              DZ + (ar * G.TPC + ac) * DS + s * 64 + a * 8 + 4 * db);
          sum.x += q.x;
          sum.y += q.y;
          sum.z += q.z;
          sum.w += q.w;
        }
      }
      *reinterpret_cast<float4*>(out + row * RC + 4 * c4) = sum;
    }
  }
}

// r = P^T D~ z: every pixel sums the tiles whose regions cover it (its own
// tile and, within Q - st pixels of a tile edge, the previous tile along that
// axis, circularly), in a fixed order. Thread (C4, R, s) of a 3D grid handles
// the four columns 4 C4 .. 4 C4 + 3, which always have the same covering
// tiles (tile widths and region strides are multiples of 4), as float4.
__global__ void k_patch_assemble(const float* __restrict__ tb, float* __restrict__ r, int S,
                                 PatchGeo G) {
  const int C4 = blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * C4 >= G.N2) return;
  const int C = 4 * C4, R = blockIdx.y, s = blockIdx.z;
  const size_t idx = ((size_t)s * G.N1 + R) * G.N2 + C;
  const int TH = PATCH_ST * G.TPR, TW = PATCH_ST * G.TPC;
  const int ntr = G.J1 / G.TPR;
  const int RA = G.RR * G.RC;
  const int tr0 = R / TH, lr0 = R - tr0 * TH;
  const int tc0 = C / TW, lc0 = C - tc0 * TW;
  // the four candidate tiles are loaded unconditionally (a tile that does
  // not cover the pixel is read at its own row / column 0 and weighted 0),
  // so that the loads are in flight together; the sum keeps its order
  float4 q[2][2];
  float wq[2][2];
#pragma unroll
  for (int dr = 0; dr < 2; ++dr) {
    const bool rin = dr == 0 || lr0 < PATCH_Q - PATCH_ST;
    const int tr = dr ? (tr0 + ntr - 1) % ntr : tr0;
    const int lr = dr ? (rin ? lr0 + TH : 0) : lr0;
#pragma unroll
    for (int dc = 0; dc < 2; ++dc) {
      const bool cin = dc == 0 || lc0 < PATCH_Q - PATCH_ST;
      const int tc = dc ? (tc0 + G.ntc - 1) % G.ntc : tc0;
      const int lc = dc ? (cin ? lc0 + TW : 0) : lc0;
      const size_t t = (size_t)tr * G.ntc + tc;
      q[dr][dc] = *reinterpret_cast<const float4*>(tb + (t * S + s) * RA + lr * G.RC + lc);
      wq[dr][dc] = rin && cin ? 1.f : 0.f;
    }
  }
  float4 sum = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int dr = 0; dr < 2; ++dr)
#pragma unroll
    for (int dc = 0; dc < 2; ++dc) {
      if (wq[dr][dc] == 0.f) continue;
      sum.x += q[dr][dc].x;
      sum.y += q[dr][dc].y;
      sum.z += q[dr][dc].z;
      sum.w += q[dr][dc].w;
    }
  *reinterpret_cast<float4*>(r + idx) = sum;
}

}  // namespace cip
