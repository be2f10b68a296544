// ADMM column pass launcher for one column length, CIP_COL_N (set by the
// build; one translation unit per length keeps compilation parallel).
#include "col_pass.hpp"
#include "kernels.hpp"
#include "launch.hpp"

#ifndef CIP_COL_N
#error "CIP_COL_N must be defined"
#endif

#define CIP_CAT2(a, b) a##b
#define CIP_CAT(a, b) CIP_CAT2(a, b)

namespace cip {

template <int NN, bool DCT>
static hipError_t col_n(int S, const cx<float>* Gin, cx<float>* Yout, int H2, const float* Adiag,
                        const cx<float>* Aoff, const cx<float>* xh0, const cx<float>* tw,
                        const cx<float>* ew, const float* band, int zero_in, int dct_out,
                        hipStream_t st) {
  const int T = NN / ppt_col<NN>();
  auto run = [&](auto kern, size_t lds_floats) {
    // H2 - 1 work-groups: columns 0 and N2/2 share one (pair mode)
    return launch(kern, H2 - 1, S * T, lds_floats * 4, st, Gin, Yout, H2, Adiag, Aoff, xh0, tw,
                  ew, band, zero_in, dct_out);
  };
  switch (S) {
    case 1: return run(k_admm_col<NN, DCT, 1>, col_lds_floats<NN, DCT, 1>());
    case 2: return run(k_admm_col<NN, DCT, 2>, col_lds_floats<NN, DCT, 2>());
    case 3: return run(k_admm_col<NN, DCT, 3>, col_lds_floats<NN, DCT, 3>());
    case 4: return run(k_admm_col<NN, DCT, 4>, col_lds_floats<NN, DCT, 4>());
    case 5: return run(k_admm_col<NN, DCT, 5>, col_lds_floats<NN, DCT, 5>());
    case 6: return run(k_admm_col<NN, DCT, 6>, col_lds_floats<NN, DCT, 6>());
    case 7: return run(k_admm_col<NN, DCT, 7>, col_lds_floats<NN, DCT, 7>());
    case 8: return run(k_admm_col<NN, DCT, 8>, col_lds_floats<NN, DCT, 8>());
  }
  return hipErrorInvalidValue;
}

hipError_t CIP_CAT(admm_col_launch_, CIP_COL_N)(int S, bool dct, const cx<float>* Gin,
                                                 cx<float>* Yout, int H2, const float* Adiag,
                                                 const cx<float>* Aoff, const cx<float>* xh0,
                                                 const cx<float>* tw, const cx<float>* ew,
                                                 const float* band, int zero_in, int dct_out,
                                                 hipStream_t st) {
  return dct ? col_n<CIP_COL_N, true>(S, Gin, Yout, H2, Adiag, Aoff, xh0, tw, ew, band, zero_in,
                                      dct_out, st)
             : col_n<CIP_COL_N, false>(S, Gin, Yout, H2, Adiag, Aoff, xh0, tw, ew, nullptr, zero_in,
                                       dct_out, st);
}

}  // namespace cip
