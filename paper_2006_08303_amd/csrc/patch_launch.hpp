// Host-side entry points of the patch-dictionary kernels (patch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cip {

bool patch_supported(int S, int NA);
bool patch_grid_ok(int N1, int N2);
size_t patch_tile_buffer_floats(int S, int N1, int N2);
// mode: full update, codes and state only (z to zf in FP32), or D z only
// from the codes in zf
enum { PZ_MODE_FULL = 0, PZ_MODE_CODES = 1, PZ_MODE_SYNTH = 2 };
// rs: when not null, residual partial sums of the adaptive penalty (two floats
// per wave: patch_z_residual_floats of them).
hipError_t patch_z_launch(int S, int NA, const float* x, float* v, float* tb, const uint16_t* D,
                          const uint16_t* M1, int N1, int N2, float kappa, int first,
                          hipStream_t st, int mode = 0, float* zf = nullptr, float* rs = nullptr);
size_t patch_z_residual_floats(int N1, int N2);

// Device buffers of the online patch-dictionary update (patch_dl.hpp):
//   zf [A][J] codes, part [KS][n + A][A] split products, bm / d [n][A]
//   right-hand side and D, cm / lt [256][256] system and its factor,
//   g / e [n][A] dictionary and dual, dbf [n][A] / m1bf [A][n] BF16 tables.
// Device buffers of the online patch-dictionary update: the FP32 codes zf
// [A][J]; the FP64 D-step's product slices, right-hand side, matrix, factor
// (by columns, then by rows) and D; the FP32 matrix and factor of M1; G, E
// (FP32) and the BF16 tables of G and M1.
struct PatchDictBufs {
  float* zf;
  double *part, *bm, *cm64, *lt64, *d;
  float *cm, *lt, *g, *e;
  uint16_t *dbf, *m1bf;
};
int patch_dict_splits(int N1, int N2);
hipError_t patch_dict_start(const float* d0, const PatchDictBufs& b, int nv, int NA,
                            hipStream_t st);
// one D, G, E step and M1 of the new G; res (optional, device): ||D - G||^2,
// ||G - G_prev||^2 in FP64
hipError_t patch_dict_step(const float* x, const PatchDictBufs& b, int S, int NA, int N1, int N2,
                           double sigma, float rho, hipStream_t st, double* res = nullptr);
// M1 = G^T (rho I + G G^T)^-1 (BF16) of the current G
hipError_t patch_dict_m1(const PatchDictBufs& b, int S, int NA, float rho, hipStream_t st);
// E <- c E (count = n A entries)
hipError_t patch_dict_scale_dual(const PatchDictBufs& b, int count, float c, hipStream_t st);
hipError_t patch_assemble_launch(int S, const float* tb, float* r, int N1, int N2, hipStream_t st);

}  // namespace cip
