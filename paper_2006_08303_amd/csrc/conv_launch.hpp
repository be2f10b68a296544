// Host-side entry points of the convolutional-dictionary kernels (conv.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "fft.hpp"

namespace cip {

hipError_t conv_place_filter(const float* filt, double* dst, int L, int N1, int N2, hipStream_t st);
hipError_t conv_tables(const cx<double>* th64, cx<float>* th32, float* gam, float* eta, int M,
                       size_t F, double rho, double mu, int N1, int N2, hipStream_t st);
hipError_t conv_col_fft(int dir, const cx<float>* in, cx<float>* out, int P, int N1, int H2,
                        const cx<float>* tw, hipStream_t st);
hipError_t conv_freq(cx<float>* gv, cx<float>* dhat, cx<float>* xhat, const cx<float>* xh0,
                     const float* Adiag, const cx<float>* Aoff, const cx<float>* th,
                     const float* gam, const float* eta, int M, int S, size_t F, int first,
                     int zero_g, int do_z, hipStream_t st);
hipError_t conv_tables3(const cx<double>* th64, cx<float>* th32, float* gam, int M, int S,
                        size_t F, double rho, hipStream_t st);
hipError_t conv_freq3(cx<float>* gv, cx<float>* dhat, cx<float>* xhat, const cx<float>* xh0,
                      const float* Adiag, const cx<float>* Aoff, const cx<float>* th,
                      const float* gam, const cx<float>* bw, int M, int S, size_t F, int first,
                      int zero_g, int do_z, hipStream_t st);
// 3D dictionary update (see conv.hpp)
// d-updates (3D and 2D forms); dsp receives d^ + e^
hipError_t cdl_dfreq(const cx<float>* xhat, const cx<float>* zh, const cx<float>* gehat,
                     const cx<float>* ehat, cx<float>* dsp, const cx<float>* bw, int M, int S,
                     size_t F, float sigma, hipStream_t st);
hipError_t cdl_dfreq2(const cx<float>* xhat, const cx<float>* zh, const cx<float>* gehat,
                      const cx<float>* ehat, cx<float>* dsp, int M, int S, size_t F, float sigma,
                      hipStream_t st);
hipError_t conv_tables2f(const cx<float>* th, float* gam, float* eta, int M, size_t F, double rho,
                         double mu, int N1, int N2, hipStream_t st);
hipError_t conv_dhat2(const cx<float>* zh, const cx<float>* th, cx<float>* dhat, int M, int S,
                      size_t F, hipStream_t st);
hipError_t cdl_project(const float* dpl, const float* e, float* gtap, int M, int S, int N1, int N2,
                       int L, hipStream_t st);
// frequency-domain dual (see conv.hpp): from s = d^ + e^ and g^,
// e^ += d^ - g^ (= s - g^), ge = g^ - e^, gs = g^
hipError_t cdl_fdual(cx<float>* e, cx<float>* ge, const cx<float>* sd, cx<float>* gs, size_t n,
                     hipStream_t st);
// the same at a check of sigma: partial sums of |d^ - g^|^2 (half-spectrum
// weights) and of |gtap - gprev|^2, one pair per work-group (CDL_RES_GROUPS)
constexpr int CDL_RES_GROUPS = 1024;
hipError_t cdl_fdual_res(cx<float>* e, cx<float>* ge, const cx<float>* sd, cx<float>* gs,
                         size_t n, size_t F, int N1, int N2, const float* gtap,
                         const float* gprev, size_t ntaps, float* part, hipStream_t st);
// sigma -> sigma': e^ <- c e^, ge = gs - e^ (c = sigma / sigma')
hipError_t cdl_rescale_dual(cx<float>* e, cx<float>* ge, const cx<float>* gs, size_t n, float c,
                            hipStream_t st);
hipError_t cdl_fzero(cx<float>* e, size_t n, hipStream_t st);
hipError_t cdl_place(const float* gtap, float* out, int M, int S, int N1, int N2, int L,
                     hipStream_t st);
hipError_t conv_tables3f(const cx<float>* th2, cx<float>* th32, float* gam, const cx<float>* bw,
                         int M, int S, size_t F, float rho, hipStream_t st);
hipError_t conv_dhat3(const cx<float>* zh, const cx<float>* th, cx<float>* dhat,
                      const cx<float>* bw, int M, int S, size_t F, hipStream_t st);
// rs: optional residual sums of the split z = t (k_conv_row), sized by
// conv_row_residual_floats
hipError_t conv_row(const cx<float>* Vin, cx<float>* Gout, float* V, int P, int N1, int N2,
                    const cx<float>* tw, float kappa, float zscale, int first, hipStream_t st,
                    float* rs = nullptr);
size_t conv_row_residual_floats(int P, int N1, int N2);
// state V re-expressed for a new penalty, W = t - u' (k_conv_reemit)
hipError_t conv_reemit(float* V, float* W, size_t n, float kappa, float kappa_new, float sc,
                       hipStream_t st);

}  // namespace cip
