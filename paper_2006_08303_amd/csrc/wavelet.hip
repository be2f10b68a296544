// Launchers of the wavelet (x) DCT prior's kernels (separate translation unit).
#include "launch.hpp"
#include "wavelet.hpp"
#include "wavelet_launch.hpp"

namespace cip {

namespace {
int blocks(size_t n) { return (int)((n + 255) / 256); }

// work-groups of a level with T x T coefficient tiles per band
dim3 tile_grid(int R, int C, int planes, int T) {
  return dim3((C / 2 + T - 1) / T, (R / 2 + T - 1) / T, planes);
}

// 32 x 32 tiles (less halo per coefficient) when they still give two
// work-groups per compute unit, else 16 x 16
bool big_tiles(int R, int C, int planes) {
  const dim3 g = tile_grid(R, C, planes, 32);
  return (size_t)g.x * g.y * g.z >= 512;
}
}  // namespace

// Staging areas of the low-low bands: the top-left and bottom-right
// quadrants of tmp (every level after the first fits in a quadrant).
hipError_t wavelet_forward(const float* x, float* coef, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st) {
  float* area[2] = {tmp, tmp + (size_t)(N1 / 2) * N2 + N2 / 2};
  const float* src = x;
  for (int l = 0; l < levels; ++l) {
    const int R = N1 >> l, C = N2 >> l;
    float* ll = l == levels - 1 ? coef : area[l & 1];
    if (big_tiles(R, C, planes))
      hipLaunchKernelGGL(k_dwt2<32>, tile_grid(R, C, planes, 32), dim3(256), 0, st, src, ll, coef,
                         N1, N2, R, C);
    else
      hipLaunchKernelGGL(k_dwt2<16>, tile_grid(R, C, planes, 16), dim3(256), 0, st, src, ll, coef,
                         N1, N2, R, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    src = ll;
  }
  return hipSuccess;
}

hipError_t wavelet_inverse(float* coef, float* x, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st) {
  float* area[2] = {tmp, tmp + (size_t)(N1 / 2) * N2 + N2 / 2};
  const float* ll = coef;
  for (int l = levels - 1; l >= 0; --l) {
    const int R = N1 >> l, C = N2 >> l;
    float* dst = l == 0 ? x : area[l & 1];
    if (big_tiles(R, C, planes))
      hipLaunchKernelGGL(k_idwt2<32>, tile_grid(R, C, planes, 32), dim3(256), 0, st, ll,
                         (const float*)coef, dst, N1, N2, R, C);
    else
      hipLaunchKernelGGL(k_idwt2<16>, tile_grid(R, C, planes, 16), dim3(256), 0, st, ll,
                         (const float*)coef, dst, N1, N2, R, C);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ll = dst;
  }
  return hipSuccess;
}

hipError_t wavelet_state(float* coef, float* v, const float* cs, int S, int N1, int N2,
                         float kappa, int first, hipStream_t st, float* rs) {
  const size_t plane = (size_t)N1 * N2;
  switch (S) {
#define CIP_WS(SS)                                                                            \
  case SS:                                                                                    \
    return launch(k_wdct_state<SS>, blocks(plane), 256, 0, st, coef, v, cs, plane, kappa, first, \
                  rs);
    CIP_WS(1) CIP_WS(2) CIP_WS(3) CIP_WS(4) CIP_WS(5) CIP_WS(6) CIP_WS(7) CIP_WS(8)
#undef CIP_WS
  }
  return hipErrorInvalidValue;
}

int wavelet_state_groups(int N1, int N2) { return blocks((size_t)N1 * N2); }

hipError_t wavelet_emit(float* coef, float* v, const float* cs, int S, int N1, int N2,
                        float kappa, float sc, hipStream_t st) {
  const size_t plane = (size_t)N1 * N2;
  switch (S) {
#define CIP_WE(SS)                                                                             \
  case SS:                                                                                     \
    return launch(k_wdct_emit<SS>, blocks(plane), 256, 0, st, coef, v, cs, plane, kappa, sc);
    CIP_WE(1) CIP_WE(2) CIP_WE(3) CIP_WE(4) CIP_WE(5) CIP_WE(6) CIP_WE(7) CIP_WE(8)
#undef CIP_WE
  }
  return hipErrorInvalidValue;
}

}  // namespace cip
