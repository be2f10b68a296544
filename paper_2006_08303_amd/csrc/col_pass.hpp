// Launchers of the ADMM column pass, one per column length N1; each is
// compiled in its own translation unit (col_pass.hip with CIP_COL_N = N1).
#pragma once
#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace cip {

#define CIP_DECLARE_COL(NN)                                                                  \
  hipError_t admm_col_launch_##NN(int S, bool dct, const cx<float>* Gin, cx<float>* Yout,      \
                                  int H2, const float* Adiag, const cx<float>* Aoff,           \
                                  const cx<float>* xh0, const cx<float>* tw,                   \
                                  const cx<float>* ew, int zero_in, int dct_out, hipStream_t st);
CIP_DECLARE_COL(16)
CIP_DECLARE_COL(32)
CIP_DECLARE_COL(64)
CIP_DECLARE_COL(128)
CIP_DECLARE_COL(256)
CIP_DECLARE_COL(512)
CIP_DECLARE_COL(1024)
CIP_DECLARE_COL(2048)
#undef CIP_DECLARE_COL

}  // namespace cip
