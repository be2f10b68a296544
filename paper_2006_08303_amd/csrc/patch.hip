// Launchers of the patch-dictionary kernels (separate translation unit).
#include "launch.hpp"
#include "patch.hpp"
#include "patch_dl.hpp"
#include "patch_launch.hpp"
#include "sizes.hpp"

namespace cip {

bool patch_supported(int S, int NA) {
  return S >= 1 && S <= 4 && (NA == 64 || NA == 128 || NA == 256);
}

size_t patch_z_residual_floats(int N1, int N2) {
  const PatchGeo G = patch_geo(N1, N2);
  return (size_t)(G.J1 / G.TPR) * G.ntc * 4 * 2;
}

hipError_t patch_z_launch(int S, int NA, const float* x, float* v, float* tb, const uint16_t* D,
                          const uint16_t* M1, int N1, int N2, float kappa, int first,
                          hipStream_t st, int mode, float* zf, float* rs) {
  const PatchGeo G = patch_geo(N1, N2);
  const int tiles = (G.J1 / G.TPR) * G.ntc;
  static_assert(PZ_MODE_FULL == PZ_FULL && PZ_MODE_CODES == PZ_CODES && PZ_MODE_SYNTH == PZ_SYNTH,
                "launcher and kernel modes agree");
  if (mode != PZ_FULL && !zf) return hipErrorInvalidValue;
#define CIP_PATCH_MODE(SS, AA, MM)                                                            \
  launch(k_patch_z<SS, AA, MM>, tiles, 256, (size_t)patch_lds_bytes<SS, AA>(), st, x, v, tb, D, \
         M1, G, kappa, first, zf, rs)
#define CIP_PATCH_CASE(SS, AA)                                                  \
  if (S == SS && NA == AA)                                                      \
    return mode == PZ_FULL    ? CIP_PATCH_MODE(SS, AA, PZ_FULL)                 \
           : mode == PZ_CODES ? CIP_PATCH_MODE(SS, AA, PZ_CODES)                \
                              : CIP_PATCH_MODE(SS, AA, PZ_SYNTH);
  CIP_PATCH_CASE(1, 64) CIP_PATCH_CASE(1, 128) CIP_PATCH_CASE(1, 256)
  CIP_PATCH_CASE(2, 64) CIP_PATCH_CASE(2, 128) CIP_PATCH_CASE(2, 256)
  CIP_PATCH_CASE(3, 64) CIP_PATCH_CASE(3, 128) CIP_PATCH_CASE(3, 256)
  CIP_PATCH_CASE(4, 64) CIP_PATCH_CASE(4, 128) CIP_PATCH_CASE(4, 256)
#undef CIP_PATCH_CASE
#undef CIP_PATCH_MODE
  return hipErrorInvalidValue;
}

hipError_t patch_assemble_launch(int S, const float* tb, float* r, int N1, int N2, hipStream_t st) {
  const PatchGeo G = patch_geo(N1, N2);
  hipLaunchKernelGGL(k_patch_assemble, dim3((N2 / 4 + 63) / 64, N1, S), dim3(64), 0, st, tb, r, S,
                     G);
  return hipGetLastError();
}

size_t patch_tile_buffer_floats(int S, int N1, int N2) {
  const PatchGeo G = patch_geo(N1, N2);
  return (size_t)(G.J1 / G.TPR) * G.ntc * S * G.RR * G.RC;
}

int patch_dict_splits(int N1, int N2) {
  const size_t J = (size_t)(N1 / PATCH_ST) * (N2 / PATCH_ST);
  const size_t ks = J / PDL_KSTEP;
  return (int)(ks < 64 ? ks : 64);
}

hipError_t patch_dict_start(const float* d0, const PatchDictBufs& b, int nv, int NA,
                            hipStream_t st) {
  const int count = nv * NA;
  return launch(k_pdl_start, (count + 255) / 256, 256, 0, st, d0, b.g, b.e, count);
}

// Rows of B M^-1 (k_pdl_trsolve, one row per wave) for order m <= 256.
// The LDS limit of the four instances is raised once per process (not on
// every launch, so that solves captured into a graph issue kernels only).
static hipError_t trsolve_lds_limit() {
  static hipError_t status = [] {
    const int lds = pdl_trsolve_lds_floats(PDL_MAXM) * 4;
    const void* k[4] = {reinterpret_cast<const void*>(k_pdl_trsolve<1>),
                        reinterpret_cast<const void*>(k_pdl_trsolve<2>),
                        reinterpret_cast<const void*>(k_pdl_trsolve<3>),
                        reinterpret_cast<const void*>(k_pdl_trsolve<4>)};
    for (const void* f : k) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }();
  return status;
}

static hipError_t trsolve(const float* lt, int m, const float* b, int bsr, int bsc, int q, float* xo,
                          uint16_t* xbf, hipStream_t st) {
  hipError_t e = trsolve_lds_limit();
  if (e != hipSuccess) return e;
  const dim3 grid((q + 3) / 4), block(256);
  const size_t lds = (size_t)pdl_trsolve_lds_floats(m) * 4;
  switch ((m + 63) / 64) {
    case 1: hipLaunchKernelGGL(k_pdl_trsolve<1>, grid, block, lds, st, lt, m, b, bsr, bsc, q, xo, xbf); break;
    case 2: hipLaunchKernelGGL(k_pdl_trsolve<2>, grid, block, lds, st, lt, m, b, bsr, bsc, q, xo, xbf); break;
    case 3: hipLaunchKernelGGL(k_pdl_trsolve<3>, grid, block, lds, st, lt, m, b, bsr, bsc, q, xo, xbf); break;
    case 4: hipLaunchKernelGGL(k_pdl_trsolve<4>, grid, block, lds, st, lt, m, b, bsr, bsc, q, xo, xbf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One step of the dictionary ADMM and the new code tables (see patch_dl.hpp).
hipError_t patch_dict_m1(const PatchDictBufs& b, int S, int NA, float rho, hipStream_t st) {
  const int nv = 64 * S;
  hipError_t e;
  hipLaunchKernelGGL(k_pdl_gram, dim3(nv / 16, nv / 16), dim3(256), 0, st, (const float*)b.g, NA,
                     rho, b.cm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch(k_pdl_chol, 1, PDL_CHOL_THREADS, 0, st, (const float*)b.cm, PDL_MAXM, nv,
                  b.lt)) != hipSuccess)
    return e;
  return trsolve(b.lt, nv, b.g, 1, NA, NA, nullptr, b.m1bf, st);
}

hipError_t patch_dict_scale_dual(const PatchDictBufs& b, int count, float c, hipStream_t st) {
  return launch(k_pdl_scale, (count + 255) / 256, 256, 0, st, b.e, count, c);
}

hipError_t patch_dict_step(const float* x, const PatchDictBufs& b, int S, int NA, int N1, int N2,
                           double sigma, float rho, hipStream_t st, double* res) {
  const PatchGeo G = patch_geo(N1, N2);
  const int nv = 64 * S, rows = nv + NA;
  const int KS = patch_dict_splits(N1, N2);
  const int chunk = (int)(((size_t)G.J1 * G.J2) / KS);
  if (nv > PDL_MAXM || NA > PDL_MAXM || NA % 64 || chunk % PDL_KSTEP) return hipErrorInvalidValue;
  hipError_t e;
  // X Z^T and Z Z^T in FP64
  hipLaunchKernelGGL(k_pdl_gemm64, dim3(rows / 64, NA / 64, KS), dim3(256), 0, st, x, b.zf,
                     b.part, G, S, NA, chunk);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t nr = (size_t)rows * NA;
  if ((e = launch(k_pdl_reduce64, (int)((nr + 255) / 256), 256, 0, st, (const double*)b.part,
                  (const float*)b.g, (const float*)b.e, b.bm, b.cm64, nv, NA, KS, sigma)) !=
      hipSuccess)
    return e;
  // D = B (Z Z^T + sigma I)^-1 in FP64
  double* lt2 = b.lt64 + (size_t)PDL_MAXM * PDL_MAXM;
  if ((e = launch(k_pdl_chol64, 1, 256, 0, st, b.cm64, PDL_MAXM, NA, b.lt64, lt2)) != hipSuccess)
    return e;
  const dim3 tg((nv + 3) / 4), tb(256);
  switch (NA / 64) {
    case 1: hipLaunchKernelGGL(k_pdl_trsolve64<1>, tg, tb, 0, st, b.lt64, lt2, NA, b.bm, nv, b.d); break;
    case 2: hipLaunchKernelGGL(k_pdl_trsolve64<2>, tg, tb, 0, st, b.lt64, lt2, NA, b.bm, nv, b.d); break;
    case 3: hipLaunchKernelGGL(k_pdl_trsolve64<3>, tg, tb, 0, st, b.lt64, lt2, NA, b.bm, nv, b.d); break;
    case 4: hipLaunchKernelGGL(k_pdl_trsolve64<4>, tg, tb, 0, st, b.lt64, lt2, NA, b.bm, nv, b.d); break;
    default: return hipErrorInvalidValue;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // G, E and the BF16 dictionary
  if ((e = launch(k_pdl_project, 1, 1024, 0, st, (const double*)b.d, b.g, b.e, b.dbf, nv * NA,
                  res)) != hipSuccess)
    return e;
  // M1 = G^T (rho I + G G^T)^-1 in BF16
  return patch_dict_m1(b, S, NA, rho, st);
}

bool patch_grid_ok(int N1, int N2) {
  if (N1 % PATCH_ST || N2 % PATCH_ST) return false;
  const PatchGeo G = patch_geo(N1, N2);
  return G.J2 % G.TPC == 0 && G.J1 % G.TPR == 0 && G.TPR * G.TPC == PATCH_NP;
}

}  // namespace cip
