// Kernel launch helper shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

namespace cip {

// Launch `kern` with `lds` bytes of dynamic LDS (raising the per-kernel LDS
// limit when above 64 KiB) and return the launch status.
template <typename KernelT, typename... Args>
hipError_t launch(KernelT kern, int grid, int block, size_t lds, hipStream_t st, Args... args) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, args...);
  return hipGetLastError();
}

}  // namespace cip
