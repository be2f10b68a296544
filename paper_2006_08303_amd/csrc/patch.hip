// Launchers of the patch-dictionary kernels (separate translation unit).
#include "launch.hpp"
#include "patch.hpp"
#include "patch_launch.hpp"

namespace cip {

bool patch_supported(int S, int NA) {
  return S >= 1 && S <= 4 && (NA == 64 || NA == 128 || NA == 256);
}

hipError_t patch_z_launch(int S, int NA, const float* x, float* v, float* tb, const uint16_t* D,
                          const uint16_t* M1, int N1, int N2, float kappa, int first,
                          hipStream_t st) {
  const PatchGeo G = patch_geo(N1, N2);
  const int tiles = (G.J1 / G.TPR) * G.ntc;
#define CIP_PATCH_CASE(SS, AA)                                                           \
  if (S == SS && NA == AA)                                                               \
    return launch(k_patch_z<SS, AA>, tiles, 256, (size_t)patch_lds_bytes<SS, AA>(), st, x, v, \
                  tb, D, M1, G, kappa, first);
  CIP_PATCH_CASE(1, 64) CIP_PATCH_CASE(1, 128) CIP_PATCH_CASE(1, 256)
  CIP_PATCH_CASE(2, 64) CIP_PATCH_CASE(2, 128) CIP_PATCH_CASE(2, 256)
  CIP_PATCH_CASE(3, 64) CIP_PATCH_CASE(3, 128) CIP_PATCH_CASE(3, 256)
  CIP_PATCH_CASE(4, 64) CIP_PATCH_CASE(4, 128) CIP_PATCH_CASE(4, 256)
#undef CIP_PATCH_CASE
  return hipErrorInvalidValue;
}

hipError_t patch_assemble_launch(int S, const float* tb, float* r, int N1, int N2, hipStream_t st) {
  const PatchGeo G = patch_geo(N1, N2);
  const size_t n = (size_t)S * N1 * N2;
  return launch(k_patch_assemble, (int)((n + 255) / 256), 256, 0, st, tb, r, S, G);
}

size_t patch_tile_buffer_floats(int S, int N1, int N2) {
  const PatchGeo G = patch_geo(N1, N2);
  return (size_t)(G.J1 / G.TPR) * G.ntc * S * G.RR * G.RC;
}

bool patch_grid_ok(int N1, int N2) {
  if (N1 % PATCH_ST || N2 % PATCH_ST) return false;
  const PatchGeo G = patch_geo(N1, N2);
  return G.J2 % G.TPC == 0 && G.J1 % G.TPR == 0 && G.TPR * G.TPC == PATCH_NP;
}

}  // namespace cip
