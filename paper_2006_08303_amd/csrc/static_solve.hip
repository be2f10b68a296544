// One-shot reconstruction that allocates no device memory: the plan's
// workspace (tables and solve state) lives in a library-owned static device
// buffer instead of caller-provided memory, for callers that cannot call
// hipMalloc. The work itself is cip_plan_create + cip_solve: the same kernels
// on the same data, so results equal those of a plan built on caller memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cip.h"
#include "errors.hpp"

using namespace cip;

namespace {

constexpr size_t kScratchBytes = size_t(CIP_STATIC_WORKSPACE_BYTES);
constexpr int kMaxDevices = 64;

// The buffer. In host code this name is only a stand-in for the device
// object: every host use goes through the per-device address returned by
// hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;                       // one call at a time per process
void* g_scratch[kMaxDevices] = {};     // device address of `scratch`, per device

}  // namespace

extern "C" int cip_solve_static(int K, int S, int N1, int N2, const float* d_psf,
                                const cip_prior_desc* prior, double rho, double lambda,
                                const float* d_y, int iters, float* d_x, void* stream) {
  if (!d_psf || !prior || !d_y || !d_x) return fail(CIP_EINVAL, "NULL argument");
  if (iters < 1) return fail(CIP_EINVAL, "iters must be >= 1");
  size_t need = 0;
  int rc = cip_plan_workspace_bytes(K, S, N1, N2, prior, &need);
  if (rc) return rc;
  if (need > kScratchBytes)
    return fail(CIP_ENOSPC, "cip_solve_static: this problem needs " + std::to_string(need) +
                                " bytes of workspace; the static buffer holds " +
                                std::to_string(kScratchBytes));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(CIP_EHIP, "cip_solve_static: no usable current device");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CIP_EHIP, std::string("hipGetSymbolAddress of the static workspace: ") +
                                hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  cip_plan_t plan = nullptr;
  rc = cip_plan_create(K, S, N1, N2, d_psf, prior, rho, lambda, g_scratch[dev], kScratchBytes,
                       stream, &plan);
  if (rc) return rc;
  rc = cip_solve(plan, d_y, iters, d_x, stream);
  // the next call overwrites the buffer: finish this one before returning
  hipError_t e = hipStreamSynchronize(st);
  cip_plan_destroy(plan);
  if (rc) return rc;
  if (e != hipSuccess)
    return fail(CIP_EHIP, std::string("cip_solve_static: ") + hipGetErrorString(e));
  return CIP_OK;
}
