// Launchers of the convolutional-dictionary kernels (separate translation unit).
#include "conv.hpp"
#include "conv_launch.hpp"
#include "launch.hpp"
#include "sizes.hpp"

namespace cip {

hipError_t conv_place_filter(const float* filt, double* dst, int L, int N1, int N2, hipStream_t st) {
  const size_t n = (size_t)N1 * N2;
  return launch(k_place_filter, (int)((n + 255) / 256), 256, 0, st, filt, dst, L, N1, N2);
}

hipError_t conv_tables(const cx<double>* th64, cx<float>* th32, float* gam, float* eta, int M,
                       size_t F, double rho, double mu, int N1, int N2, hipStream_t st) {
  return launch(k_conv_tables, (int)((F + 255) / 256), 256, 0, st, th64, th32, gam, eta, M, F, rho,
                mu, N1, N2);
}

hipError_t conv_col_fft(int dir, const cx<float>* in, cx<float>* out, int P, int N1, int H2,
                        const cx<float>* tw, hipStream_t st) {
  CIP_DISPATCH_N(N1, {
    const int T = NN / ppt_col<NN>();
    const size_t lds = (size_t)(NN + CONV_PC * padded_len(NN)) * 8;
    const int grid = H2 * ((P + CONV_PC - 1) / CONV_PC);
    if (dir > 0) return launch(k_col_fft_batch<NN, 1>, grid, CONV_PC * T, lds, st, in, out, P, H2, tw);
    return launch(k_col_fft_batch<NN, -1>, grid, CONV_PC * T, lds, st, in, out, P, H2, tw);
  });
  return hipSuccess;
}

hipError_t conv_freq(cx<float>* gv, cx<float>* dhat, cx<float>* xhat, const cx<float>* xh0,
                     const float* Adiag, const cx<float>* Aoff, const cx<float>* th,
                     const float* gam, const float* eta, int M, int S, size_t F, int first,
                     int zero_g, int do_z, hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_CF(SS)                                                                              \
  case SS:                                                                                      \
    return launch(k_conv_freq<SS>, grid, 128, 0, st, gv, dhat, xhat, xh0, Adiag, Aoff, th, gam, \
                  eta, M, F, first, zero_g, do_z);
  switch (S) {
    CIP_CF(1)
    CIP_CF(2)
    CIP_CF(3)
    CIP_CF(4)
    CIP_CF(5)
    CIP_CF(6)
    CIP_CF(7)
    CIP_CF(8)
  }
#undef CIP_CF
  return hipErrorInvalidValue;
}

hipError_t conv_tables3(const cx<double>* th64, cx<float>* th32, float* gam, int M, int S,
                        size_t F, double rho, hipStream_t st) {
  return launch(k_conv_tables3, (int)((F + 255) / 256), 256, 0, st, th64, th32, gam, M, S, F, rho);
}

hipError_t conv_freq3(cx<float>* gv, cx<float>* dhat, cx<float>* xhat, const cx<float>* xh0,
                      const float* Adiag, const cx<float>* Aoff, const cx<float>* th,
                      const float* gam, const cx<float>* bw, int M, int S, size_t F, int first,
                      int zero_g, int do_z, hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_CF3(SS)                                                                            \
  case SS:                                                                                     \
    return launch(k_conv_freq3<SS>, grid, 128, 0, st, gv, dhat, xhat, xh0, Adiag, Aoff, th, gam, \
                  bw, M, F, first, zero_g, do_z);
  switch (S) {
    CIP_CF3(1)
    CIP_CF3(2)
    CIP_CF3(3)
    CIP_CF3(4)
    CIP_CF3(5)
    CIP_CF3(6)
    CIP_CF3(7)
    CIP_CF3(8)
  }
#undef CIP_CF3
  return hipErrorInvalidValue;
}

#define CIP_S_SWITCH(CASE) \
  switch (S) {             \
    CASE(1)                \
    CASE(2)                \
    CASE(3)                \
    CASE(4)                \
    CASE(5)                \
    CASE(6)                \
    CASE(7)                \
    CASE(8)                \
  }

hipError_t cdl_dfreq(const cx<float>* xhat, const cx<float>* zh, const cx<float>* gehat,
                     const cx<float>* ehat, cx<float>* dsp, const cx<float>* bw, int M, int S,
                     size_t F, float sigma, hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_DF(SS)                                                                           \
  case SS:                                                                                   \
    return launch(k_cdl_dfreq<SS>, grid, 128, 0, st, xhat, zh, gehat, ehat, dsp, bw, M, F, \
                  sigma);
  CIP_S_SWITCH(CIP_DF)
#undef CIP_DF
  return hipErrorInvalidValue;
}

hipError_t cdl_dfreq2(const cx<float>* xhat, const cx<float>* zh, const cx<float>* gehat,
                      const cx<float>* ehat, cx<float>* dsp, int M, int S, size_t F, float sigma,
                      hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_DF2(SS)                                                                             \
  case SS:                                                                                      \
    return launch(k_cdl_dfreq2<SS>, grid, 128, 0, st, xhat, zh, gehat, ehat, dsp, M, F, sigma);
  CIP_S_SWITCH(CIP_DF2)
#undef CIP_DF2
  return hipErrorInvalidValue;
}

hipError_t conv_tables2f(const cx<float>* th, float* gam, float* eta, int M, size_t F, double rho,
                         double mu, int N1, int N2, hipStream_t st) {
  return launch(k_conv_tables2f, (int)((F + 255) / 256), 256, 0, st, th, gam, eta, M, F, rho, mu,
                N1, N2);
}

hipError_t conv_dhat2(const cx<float>* zh, const cx<float>* th, cx<float>* dhat, int M, int S,
                      size_t F, hipStream_t st) {
  return launch(k_conv_dhat2, (int)((F + 255) / 256), 256, 0, st, zh, th, dhat, M, S, F);
}

hipError_t cdl_project(const float* dpl, const float* e, float* gtap, int M, int S, int N1, int N2,
                       int L, hipStream_t st) {
  return launch(k_cdl_project, M, 256, 0, st, dpl, e, gtap, S, N1, N2, L);
}

hipError_t cdl_fdual_res(cx<float>* e, cx<float>* ge, const cx<float>* sd, cx<float>* gs,
                         size_t n, size_t F, int N1, int N2, const float* gtap,
                         const float* gprev, size_t ntaps, float* part, hipStream_t st) {
  return launch(k_cdl_fdual_res, CDL_RES_GROUPS, 256, 0, st, e, ge, sd, gs, n, F, N1, N2, gtap,
                gprev, ntaps, part);
}

hipError_t cdl_rescale_dual(cx<float>* e, cx<float>* ge, const cx<float>* gs, size_t n, float c,
                            hipStream_t st) {
  return launch(k_cdl_rescale_dual, (int)((n + 255) / 256), 256, 0, st, e, ge, gs, n, c);
}

hipError_t cdl_fdual(cx<float>* e, cx<float>* ge, const cx<float>* sd, cx<float>* gs, size_t n,
                     hipStream_t st) {
  return launch(k_cdl_fdual, (int)((n + 255) / 256), 256, 0, st, e, ge, sd, gs, n);
}

hipError_t cdl_fzero(cx<float>* e, size_t n, hipStream_t st) {
  return launch(k_cdl_fzero, (int)((n + 255) / 256), 256, 0, st, e, n);
}

hipError_t cdl_place(const float* gtap, float* out, int M, int S, int N1, int N2, int L,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_cdl_place, dim3((N2 + 255) / 256, N1, M * S), dim3(256), 0, st, gtap, out,
                     N1, N2, L);
  return hipGetLastError();
}

hipError_t conv_tables3f(const cx<float>* th2, cx<float>* th32, float* gam, const cx<float>* bw,
                         int M, int S, size_t F, float rho, hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_TF(SS)                                                                    \
  case SS:                                                                            \
    return launch(k_conv_tables3f<SS>, grid, 128, 0, st, th2, th32, gam, bw, M, F, rho);
  CIP_S_SWITCH(CIP_TF)
#undef CIP_TF
  return hipErrorInvalidValue;
}

hipError_t conv_dhat3(const cx<float>* zh, const cx<float>* th, cx<float>* dhat,
                      const cx<float>* bw, int M, int S, size_t F, hipStream_t st) {
  const int grid = (int)((F + 127) / 128);
#define CIP_DH(SS)                                                                   \
  case SS:                                                                           \
    return launch(k_conv_dhat3<SS>, grid, 128, 0, st, zh, th, dhat, bw, M, F);
  CIP_S_SWITCH(CIP_DH)
#undef CIP_DH
  return hipErrorInvalidValue;
}

#undef CIP_S_SWITCH

hipError_t conv_row(const cx<float>* Vin, cx<float>* Gout, float* V, int P, int N1, int N2,
                    const cx<float>* tw, float kappa, float zscale, int first, hipStream_t st,
                    float* rs) {
  CIP_DISPATCH_N(N2, {
    const int T = NN / ppt_row<NN>();
    const size_t lds = (size_t)(2 * NN + row_work_floats<NN, float>(PAIRS, true)) * 4;
    return launch(k_conv_row<NN>, P * (N1 / RT), PAIRS * T, lds, st, Vin, Gout, V, N1, tw, kappa,
                  zscale, first, rs);
  });
  return hipSuccess;
}

size_t conv_row_residual_floats(int P, int N1, int N2) {
  const int nt = PAIRS * (N2 / ppt_row_n(N2));   // threads of a k_conv_row group
  const size_t waves = nt < 64 ? 1 : (size_t)(nt / 64);
  return 2 * waves * (size_t)P * (N1 / RT);
}

hipError_t conv_reemit(float* V, float* W, size_t n, float kappa, float kappa_new, float sc,
                       hipStream_t st) {
  return launch(k_conv_reemit, 2048, 256, 0, st, V, W, n, kappa, kappa_new, sc);
}

}  // namespace cip
