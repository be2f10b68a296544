// Host side of the C ABI declared in include/cip.h: plan creation (tables,
// FP64 kernel spectra, FP64 Gram pseudo-inverses), forward / adjoint
// operators and the ADMM solve loop of Algorithm 1 (Dogan & Oktem,
// Section IV-A), each step launched as a hand-written HIP kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cip.h"
#include "gram.hpp"
#include "kernels.hpp"

using namespace cip;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CIP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace carve-up. Every field is a byte offset into the caller's buffer.
struct Layout {
  size_t twN1f, twN2f, twN1d, twN2d;  // FFT twiddles
  size_t fw1, iv1, ia1, fw2, iv2, ia2;  // DCT tables (N1 and N2)
  size_t lam32, Adiag, Aoff, Mm, xh0;   // per-frequency tables
  size_t bufA, bufB;                    // RT staging (max(K,S) planes)
  size_t state;                         // ADMM state
  size_t lam64, rt64, pl64;             // plan-time FP64 scratch
  size_t total;
};

int state_floats_per_voxel(int kind) {
  switch (kind) {
    case CIP_PRIOR_DCT2D: return 1;
    case CIP_PRIOR_TV2D: return 4;   // 2 components, double-buffered
    case CIP_PRIOR_TV3D: return 6;   // 3 components, double-buffered
    default: return -1;
  }
}

Layout make_layout(int K, int S, int N1, int N2, int kind) {
  Layout L{};
  const size_t H2 = N2 / 2 + 1, F = (size_t)N1 * H2, P = (size_t)(K > S ? K : S);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align256(bytes);
    return r;
  };
  L.twN1f = take(N1 * 8);
  L.twN2f = take(N2 * 8);
  L.twN1d = take(N1 * 16);
  L.twN2d = take(N2 * 16);
  L.fw1 = take(N1 * 8);
  L.iv1 = take(N1 * 8);
  L.ia1 = take(N1 * 4);
  L.fw2 = take(N2 * 8);
  L.iv2 = take(N2 * 8);
  L.ia2 = take(N2 * 4);
  L.lam32 = take((size_t)K * S * F * 8);
  L.Adiag = take((size_t)S * F * 4);
  L.Aoff = take((size_t)(S * (S - 1) / 2) * F * 8 + 8);
  L.Mm = take((size_t)S * K * F * 8);
  L.xh0 = take((size_t)S * F * 8);
  L.bufA = take(P * F * 8);
  L.bufB = take(P * F * 8);
  L.state = take((size_t)state_floats_per_voxel(kind) * S * N1 * N2 * 4);
  L.lam64 = take((size_t)K * S * F * 16);
  L.rt64 = take(F * 16);
  L.pl64 = take((size_t)N1 * N2 * 8);
  L.total = o;
  return L;
}

int validate(int K, int S, int N1, int N2, const cip_prior_desc* prior) {
  if (!prior) return fail(CIP_EINVAL, "prior descriptor is NULL");
  if (K < 1 || K > 8 || S < 1 || S > 8) return fail(CIP_EINVAL, "K and S must be in [1, 8]");
  if (!is_pow2(N1) || !is_pow2(N2) || N1 < 16 || N2 < 16 || N1 > 2048 || N2 > 2048)
    return fail(CIP_EUNSUPPORTED, "N1 and N2 must be powers of two in [16, 2048]");
  if (state_floats_per_voxel(prior->kind) < 0)
    return fail(CIP_EUNSUPPORTED, "unsupported prior kind");
  if (prior->kind != CIP_PRIOR_DCT2D)
    return fail(CIP_EUNSUPPORTED, "this build serves the DCT2D prior only");
  if (!(prior->beta > 0.0)) return fail(CIP_EINVAL, "beta must be > 0");
  return CIP_OK;
}

}  // namespace

struct cip_plan_s {
  int K, S, N1, N2, H2, kind;
  double beta, rho, lambda;
  unsigned char* ws;
  Layout L;
  bool solved_once;
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

// ---------------------------------------------------------------- launch helpers
namespace {

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

constexpr int ppt_rt(int N) { return N >= 16 ? 16 : N; }

#define DISPATCH_N(N, CALL)                                   \
  switch (N) {                                                \
    case 16: { constexpr int NN = 16; CALL; } break;          \
    case 32: { constexpr int NN = 32; CALL; } break;          \
    case 64: { constexpr int NN = 64; CALL; } break;          \
    case 128: { constexpr int NN = 128; CALL; } break;        \
    case 256: { constexpr int NN = 256; CALL; } break;        \
    case 512: { constexpr int NN = 512; CALL; } break;        \
    case 1024: { constexpr int NN = 1024; CALL; } break;      \
    case 2048: { constexpr int NN = 2048; CALL; } break;      \
    default: return hipErrorInvalidValue;                     \
  }

template <typename Re>
hipError_t row_r2c(const Re* in, cx<Re>* out, int P, int N1, int N2, const cx<Re>* tw, hipStream_t st) {
  constexpr bool staged = sizeof(Re) == 4;
  DISPATCH_N(N2, {
    const int T = NN / ppt_rt(NN);
    const int ng = staged ? PAIRS : 1;
    size_t fft_l = (size_t)ng * 2 * padded_len(NN) * sizeof(Re);
    size_t stg_l = staged ? (size_t)(NN / 2 + 1) * RT * 2 * sizeof(Re) : 0;
    size_t lds = fft_l > stg_l ? fft_l : stg_l;
    int grid = staged ? P * (N1 / RT) : P * (N1 / 2);
    return launch(k_row_r2c<NN, Re, staged>, grid, ng * T, lds, st, in, out, N1, tw);
  });
  return hipSuccess;
}

hipError_t row_c2r(const cx<float>* in, float* out, int P, int N1, int N2, float scale,
                   const cx<float>* tw, hipStream_t st) {
  DISPATCH_N(N2, {
    const int T = NN / ppt_rt(NN);
    size_t fft_l = (size_t)PAIRS * 2 * padded_len(NN) * 4;
    size_t stg_l = (size_t)(NN / 2 + 1) * RT * 2 * 4;
    size_t lds = fft_l > stg_l ? fft_l : stg_l;
    return launch(k_row_c2r<NN>, P * (N1 / RT), PAIRS * T, lds, st, in, out, N1, scale, tw);
  });
  return hipSuccess;
}

template <typename Re, int OP>
hipError_t col_op(const cx<Re>* in, void* out, int Pin, int Pout, int N1, int H2,
                  const cx<Re>* tw, const cx<Re>* mat, int spec_plane, hipStream_t st) {
  const int PM = Pin > Pout ? Pin : Pout;
  DISPATCH_N(N1, {
    const int T = NN / ppt_rt(NN);
    size_t lds = (size_t)PM * 2 * padded_len(NN) * sizeof(Re);
    return launch(k_col_op<NN, Re, OP>, H2, PM * T, lds, st, in, out, Pin, Pout, H2, tw, mat,
                  spec_plane);
  });
  return hipSuccess;
}

hipError_t admm_row_dct(cip_plan_t p, int mode, hipStream_t st, float* xout) {
  const Layout& L = p->L;
  float kappa = (float)(p->lambda / p->rho);
  DISPATCH_N(p->N2, {
    const int T = NN / ppt_rt(NN);
    size_t fft_l = (size_t)PAIRS * 2 * padded_len(NN) * 4;
    size_t stg_l = (size_t)(NN / 2 + 1) * RT * 2 * 4;
    size_t lds = fft_l > stg_l ? fft_l : stg_l;
    return launch(k_admm_row_dct<NN>, p->S * (p->N1 / RT), PAIRS * T, lds, st,
                  p->at<const cx<float>>(L.bufB), p->at<cx<float>>(L.bufA), p->at<float>(L.state),
                  p->N1, p->at<const cx<float>>(L.twN2f), p->at<const cx<float>>(L.fw2),
                  p->at<const cx<float>>(L.iv2), p->at<const float>(L.ia2), kappa, mode, xout);
  });
  return hipSuccess;
}

hipError_t admm_col(cip_plan_t p, int zero_in, int dct_out, hipStream_t st) {
  const Layout& L = p->L;
  const bool dct = p->kind == CIP_PRIOR_DCT2D;
  DISPATCH_N(p->N1, {
    const int T = NN / ppt_rt(NN);
    size_t lds = (size_t)p->S * 2 * padded_len(NN) * 4;
    auto args = [&](auto kern) {
      return launch(kern, p->H2, p->S * T, lds, st, p->at<const cx<float>>(L.bufA),
                    p->at<cx<float>>(L.bufB), p->S, p->H2, p->at<const float>(L.Adiag),
                    p->at<const cx<float>>(L.Aoff), p->at<const cx<float>>(L.xh0),
                    p->at<const cx<float>>(L.twN1f), p->at<const cx<float>>(L.fw1),
                    p->at<const cx<float>>(L.iv1), p->at<const float>(L.ia1), zero_in, dct_out);
    };
    return dct ? args(k_admm_col<NN, true>) : args(k_admm_col<NN, false>);
  });
  return hipSuccess;
}

hipError_t gram(cip_plan_t p, hipStream_t st) {
  GramArgs a;
  a.K = p->K;
  a.N1 = p->N1;
  a.N2 = p->N2;
  a.H2 = p->H2;
  a.beta = p->beta;
  a.scale = 1.0 / ((double)p->N1 * (double)p->N2);
  a.rcond = 1e-12;
  a.wgt = p->rho;
  a.coefA = p->rho;
  a.tv_symbol = (p->kind == CIP_PRIOR_TV2D || p->kind == CIP_PRIOR_TV3D) ? 1 : 0;
  a.band_lap = p->kind == CIP_PRIOR_TV3D ? 1 : 0;
  const Layout& L = p->L;
  const size_t F = (size_t)p->N1 * p->H2;
  const int block = 128;
  const int grid = (int)((F + block - 1) / block);
  auto run = [&](auto kern) {
    return launch(kern, grid, block, 0, st, p->at<const cx<double>>(L.lam64), a,
                  p->at<float>(L.Adiag), p->at<cx<float>>(L.Aoff), p->at<cx<float>>(L.Mm),
                  p->at<cx<float>>(L.lam32));
  };
  switch (p->S) {
    case 1: return run(k_gram<1>);
    case 2: return run(k_gram<2>);
    case 3: return run(k_gram<3>);
    case 4: return run(k_gram<4>);
    case 5: return run(k_gram<5>);
    case 6: return run(k_gram<6>);
    case 7: return run(k_gram<7>);
    case 8: return run(k_gram<8>);
  }
  return hipErrorInvalidValue;
}

void twiddles(int N, std::vector<cx<float>>& f, std::vector<cx<double>>& d) {
  f.resize(N);
  d.resize(N);
  for (int m = 0; m < N; ++m) {
    double a = 2.0 * M_PI * (double)m / (double)N;
    d[m] = cx<double>{std::cos(a), -std::sin(a)};
    f[m] = cx<float>{(float)d[m].x, (float)d[m].y};
  }
}

void dct_tables(int N, std::vector<cx<float>>& fw, std::vector<cx<float>>& iv, std::vector<float>& ia) {
  fw.resize(N);
  iv.resize(N);
  ia.resize(N);
  for (int k = 0; k < N; ++k) {
    double al = k == 0 ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
    double a = M_PI * (double)k / (2.0 * N);
    fw[k] = cx<float>{(float)(al * std::cos(a)), (float)(-al * std::sin(a))};
    iv[k] = cx<float>{(float)(std::cos(a) / N), (float)(std::sin(a) / N)};
    ia[k] = (float)(1.0 / al);
  }
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* cip_last_error(void) { return g_last_error.c_str(); }

int cip_plan_workspace_bytes(int K, int S, int N1, int N2, const cip_prior_desc* prior,
                             size_t* bytes) {
  int rc = validate(K, S, N1, N2, prior);
  if (rc) return rc;
  if (!bytes) return fail(CIP_EINVAL, "bytes is NULL");
  *bytes = make_layout(K, S, N1, N2, prior->kind).total;
  return CIP_OK;
}

int cip_plan_create(int K, int S, int N1, int N2, const float* d_psf, const cip_prior_desc* prior,
                    double rho, double lambda, void* d_workspace, size_t ws_bytes, void* stream,
                    cip_plan_t* out) {
  int rc = validate(K, S, N1, N2, prior);
  if (rc) return rc;
  if (!d_psf || !d_workspace || !out) return fail(CIP_EINVAL, "NULL pointer argument");
  if (!(rho > 0.0) || !(lambda >= 0.0)) return fail(CIP_EINVAL, "need rho > 0 and lambda >= 0");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(CIP_EINVAL, "workspace must be 256-byte aligned");
  Layout L = make_layout(K, S, N1, N2, prior->kind);
  if (ws_bytes < L.total) return fail(CIP_ENOSPC, "workspace too small");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  cip_plan_s* p = new cip_plan_s();
  p->K = K;
  p->S = S;
  p->N1 = N1;
  p->N2 = N2;
  p->H2 = N2 / 2 + 1;
  p->kind = prior->kind;
  p->beta = prior->beta;
  p->rho = rho;
  p->lambda = lambda;
  p->ws = reinterpret_cast<unsigned char*>(d_workspace);
  p->L = L;
  p->solved_once = false;

  auto cleanup_fail = [&](int code, const std::string& m) {
    delete p;
    return fail(code, m);
  };
#define PLAN_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return cleanup_fail(CIP_EHIP, std::string(#expr) + ": " + \
                                              hipGetErrorString(e_));               \
  } while (0)

  std::vector<cx<float>> t1f, t2f, fw, iv;
  std::vector<cx<double>> t1d, t2d;
  std::vector<float> ia;
  twiddles(N1, t1f, t1d);
  twiddles(N2, t2f, t2d);
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN1f), t1f.data(), N1 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN2f), t2f.data(), N2 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN1d), t1d.data(), N1 * 16, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN2d), t2d.data(), N2 * 16, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipStreamSynchronize(st));
  dct_tables(N1, fw, iv, ia);
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.fw1), fw.data(), N1 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.iv1), iv.data(), N1 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.ia1), ia.data(), N1 * 4, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipStreamSynchronize(st));
  dct_tables(N2, fw, iv, ia);
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.fw2), fw.data(), N2 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.iv2), iv.data(), N2 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.ia2), ia.data(), N2 * 4, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipStreamSynchronize(st));

  // FP64 spectra of the K*S kernels: each float plane is promoted exactly to
  // double, then transformed along rows and columns in FP64.
  {
    const size_t plane = (size_t)N1 * N2;
    double* d_pl = p->at<double>(L.pl64);
    for (int ks = 0; ks < K * S; ++ks) {
      PLAN_HIP(launch(k_promote, (int)((plane + 255) / 256), 256, 0, st,
                      d_psf + (size_t)ks * plane, d_pl, plane));
      PLAN_HIP(row_r2c<double>(d_pl, p->at<cx<double>>(L.rt64), 1, N1, N2,
                               p->at<const cx<double>>(L.twN2d), st));
      PLAN_HIP((col_op<double, OP_SPEC>(p->at<const cx<double>>(L.rt64), p->at<void>(L.lam64), 1, 1,
                                        N1, p->H2, p->at<const cx<double>>(L.twN1d), nullptr, ks,
                                        st)));
    }
  }
  PLAN_HIP(gram(p, st));
  PLAN_HIP(hipStreamSynchronize(st));
  *out = p;
  return CIP_OK;
#undef PLAN_HIP
}

int cip_forward(cip_plan_t p, const float* d_x, float* d_y, void* stream) {
  if (!p || !d_x || !d_y) return fail(CIP_EINVAL, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Layout& L = p->L;
  float sc = (float)(1.0 / ((double)p->N1 * p->N2));
  HIP_TRY(row_r2c<float>(d_x, p->at<cx<float>>(L.bufA), p->S, p->N1, p->N2,
                         p->at<const cx<float>>(L.twN2f), st));
  HIP_TRY((col_op<float, OP_FWD>(p->at<const cx<float>>(L.bufA), p->at<void>(L.bufB), p->S, p->K,
                                 p->N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                 p->at<const cx<float>>(L.lam32), 0, st)));
  HIP_TRY(row_c2r(p->at<const cx<float>>(L.bufB), d_y, p->K, p->N1, p->N2, sc,
                  p->at<const cx<float>>(L.twN2f), st));
  return CIP_OK;
}

int cip_adjoint(cip_plan_t p, const float* d_y, float* d_x, void* stream) {
  if (!p || !d_x || !d_y) return fail(CIP_EINVAL, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Layout& L = p->L;
  float sc = (float)(1.0 / ((double)p->N1 * p->N2));
  HIP_TRY(row_r2c<float>(d_y, p->at<cx<float>>(L.bufA), p->K, p->N1, p->N2,
                         p->at<const cx<float>>(L.twN2f), st));
  HIP_TRY((col_op<float, OP_ADJ>(p->at<const cx<float>>(L.bufA), p->at<void>(L.bufB), p->K, p->S,
                                 p->N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                 p->at<const cx<float>>(L.lam32), 0, st)));
  HIP_TRY(row_c2r(p->at<const cx<float>>(L.bufB), d_x, p->S, p->N1, p->N2, sc,
                  p->at<const cx<float>>(L.twN2f), st));
  return CIP_OK;
}

int cip_solve(cip_plan_t p, const float* d_y, int iters, float* d_x, void* stream) {
  if (!p || !d_y || !d_x) return fail(CIP_EINVAL, "NULL argument");
  if (iters < 1) return fail(CIP_EINVAL, "iters must be >= 1");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Layout& L = p->L;
  // Alg. 1 step 2 (per solve): x_hat0 = Psi^+ beta Lambda^H F y / (N1 N2)
  HIP_TRY(row_r2c<float>(d_y, p->at<cx<float>>(L.bufA), p->K, p->N1, p->N2,
                         p->at<const cx<float>>(L.twN2f), st));
  HIP_TRY((col_op<float, OP_XHAT0>(p->at<const cx<float>>(L.bufA), p->at<void>(L.xh0), p->K, p->S,
                                   p->N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                   p->at<const cx<float>>(L.Mm), 0, st)));
  // iteration 1 (t = u = 0): column pass only
  HIP_TRY(admm_col(p, 1, iters > 1 ? 1 : 0, st));
  for (int l = 1; l < iters; ++l) {
    HIP_TRY(admm_row_dct(p, l == 1 ? ROW_FIRST : ROW_FULL, st, nullptr));
    HIP_TRY(admm_col(p, 0, l < iters - 1 ? 1 : 0, st));
  }
  HIP_TRY(admm_row_dct(p, ROW_FINAL, st, d_x));
  p->solved_once = true;
  return CIP_OK;
}

int cip_plan_destroy(cip_plan_t p) {
  delete p;
  return CIP_OK;
}

int cip_time_kernel(cip_plan_t p, int which, int reps, void* stream, double* avg_us) {
  if (!p || !avg_us || reps < 1) return fail(CIP_EINVAL, "bad argument");
  if (!p->solved_once) return fail(CIP_EINVAL, "run cip_solve on this plan first");
  if (which < 0 || which > 1) return fail(CIP_EINVAL, "which must be 0 or 1");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) {
    if (which == 0) HIP_TRY(admm_row_dct(p, ROW_FULL, st, nullptr));
    else HIP_TRY(admm_col(p, 0, 1, st));
  }
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_us = 1000.0 * ms / reps;
  return CIP_OK;
}

}  // extern "C"
