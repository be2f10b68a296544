// Host-side entry points of the patch-dictionary kernels (patch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cip {

bool patch_supported(int S, int NA);
bool patch_grid_ok(int N1, int N2);
size_t patch_tile_buffer_floats(int S, int N1, int N2);
hipError_t patch_z_launch(int S, int NA, const float* x, float* v, float* tb, const uint16_t* D,
                          const uint16_t* M1, int N1, int N2, float kappa, int first,
                          hipStream_t st);
hipError_t patch_assemble_launch(int S, const float* tb, float* r, int N1, int N2, hipStream_t st);

}  // namespace cip
