// Launchers of the ADMM column pass, one per column length N1; each is
// compiled in its own translation unit (col_pass.hip with CIP_COL_N = N1).
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "sizes.hpp"

namespace cip {

#define CIP_DECLARE_COL(NN)                                                                  \
  hipError_t admm_col_launch_##NN(int S, bool dct, const cx<float>* Gin, cx<float>* Yout,      \
                                  int H2, const float* Adiag, const cx<float>* Aoff,           \
                                  const cx<float>* xh0, const cx<float>* tw,                   \
                                  const cx<float>* ew, const float* band, int zero_in,         \
                                  int dct_out, hipStream_t st);
CIP_FOR_EACH_SIZE(CIP_DECLARE_COL)
#undef CIP_DECLARE_COL

}  // namespace cip
