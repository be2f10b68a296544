// Launchers of the wavelet (x) DCT prior's kernels (separate translation unit).
#include "launch.hpp"
#include "wavelet.hpp"
#include "wavelet_launch.hpp"

namespace cip {

namespace {
int blocks(size_t n) { return (int)((n + 255) / 256); }
}  // namespace

hipError_t wavelet_forward(const float* x, float* coef, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st) {
  int R = N1, C = N2;
  hipError_t e;
  for (int l = 0; l < levels; ++l) {
    const float* src = l == 0 ? x : coef;
    if ((e = launch(k_dwt_rows, blocks((size_t)planes * R * (C / 2)), 256, 0, st, src, tmp, planes,
                    N1, N2, R, C)) != hipSuccess)
      return e;
    if ((e = launch(k_dwt_cols, blocks((size_t)planes * (R / 2) * C), 256, 0, st,
                    (const float*)tmp, coef, planes, N1, N2, R, C)) != hipSuccess)
      return e;
    R /= 2;
    C /= 2;
  }
  return hipSuccess;
}

hipError_t wavelet_inverse(float* coef, float* x, float* tmp, int planes, int N1, int N2,
                           int levels, hipStream_t st) {
  hipError_t e;
  for (int l = levels - 1; l >= 0; --l) {
    const int R = N1 >> l, C = N2 >> l;
    float* dst = l == 0 ? x : coef;
    if ((e = launch(k_idwt_cols, blocks((size_t)planes * (R / 2) * C), 256, 0, st,
                    (const float*)coef, tmp, planes, N1, N2, R, C)) != hipSuccess)
      return e;
    if ((e = launch(k_idwt_rows, blocks((size_t)planes * R * (C / 2)), 256, 0, st,
                    (const float*)tmp, dst, planes, N1, N2, R, C)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

hipError_t wavelet_state(float* coef, float* v, const float* cs, int S, int N1, int N2,
                         float kappa, int first, hipStream_t st) {
  const size_t plane = (size_t)N1 * N2;
  switch (S) {
#define CIP_WS(SS) \
  case SS: return launch(k_wdct_state<SS>, blocks(plane), 256, 0, st, coef, v, cs, plane, kappa, first);
    CIP_WS(1) CIP_WS(2) CIP_WS(3) CIP_WS(4) CIP_WS(5) CIP_WS(6) CIP_WS(7) CIP_WS(8)
#undef CIP_WS
  }
  return hipErrorInvalidValue;
}

}  // namespace cip
