// Host side of the C ABI declared in include/cip.h: plan creation (tables,
// FP64 kernel spectra, FP64 Gram pseudo-inverses), forward / adjoint
// operators and the ADMM solve loop of Algorithm 1 (Dogan & Oktem,
// Section IV-A), each step launched as a hand-written HIP kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cip.h"
#include "gram.hpp"
#include "col_pass.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "norms.hpp"
#include "itv.hpp"
#include "patch_launch.hpp"
#include "wavelet_launch.hpp"
#include "conv_launch.hpp"
#include "errors.hpp"
#include "sizes.hpp"

using namespace cip;

namespace cip {
// Exact float -> double promotion of one plane (plan time).
__global__ void k_promote(const float* __restrict__ src, double* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}
}  // namespace cip

namespace {


#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(CIP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace carve-up. A plan's memory has two regions: the tables (twiddles,
// spectra, per-frequency inverses, dictionaries; read-only once the plan is
// built) followed by the solve state (x_hat0, staging, ADMM state; written by
// every solve). The FP64 scratch used while the plan is built aliases the
// state region, which is dead until the first solve. Every field is a byte
// offset into its region; offsets into the state region carry STATE_BIT.
// Plans attached to a built plan (cip_plan_attach) share its tables and have
// a state region of their own.
constexpr size_t STATE_BIT = size_t(1) << 62;
constexpr int XCHANGE_GROUPS = 256;   // work-groups of k_xchange

struct Layout {
  size_t twN1f, twN2f, twN1d, twN2d;  // FFT twiddles
  size_t twN2f8;                        // row twiddles, 8 points per thread (tuning variant)
  size_t ew1, ew2;                      // DCT tables exp(-i pi k / 2N) (N1 and N2)
  size_t lam32, Adiag, Aoff, Mm, xh0;   // per-frequency tables (x_hat0 per solve)
  size_t band;                          // DCT3D: band DCT-II matrix [S][S]
  size_t bufA, bufB;                    // RT staging (max(K,S) planes)
  size_t state;                         // ADMM state
  size_t lam64, rt64, pl64;             // plan-time FP64 scratch (lam64 resident if adaptive)
  size_t xbuf, sums;                    // adaptive solves: iterates, norm partial sums
  size_t dbf, m1bf, vpatch, tbuf, rimg;  // patch prior: D, M1 (bf16), codes, tiles, P^T D z
  size_t dbf0, m1bf0, pd0, pzf, ppart, pbm, pd, pcm, plt, pg, pe;  // patch dictionary learning
  size_t pcm64, plt64;                  // FP64 matrix and factor of the D-step
  size_t th32, gam, eta, gv, dhat, xhat, rtc, vconv, th64;  // conv prior
  size_t bw;                                                 // 3D conv: band DFT matrix
  size_t wband, wcoef, wtmp;            // wavelet (x) DCT: band DCT, coefficients, staging
  size_t filt0, gtap, gehat, dsp, ecdl, dpl;                 // 3D dictionary update
  size_t gprev;                         // conv learning with adaptive penalties: G_prev taps
  size_t tprev;                         // isotropic TV with adaptive penalties: t of the last store
  size_t tables;                        // bytes of the table region
  size_t state_bytes;                   // bytes of the state region
  size_t total;                         // tables + state_bytes
};

int state_floats_per_voxel(int kind) {
  switch (kind) {
    case CIP_PRIOR_DCT2D: return 1;
    case CIP_PRIOR_DCT3D: return 1;
    case CIP_PRIOR_ITV2D: return 6;  // u, dual p (2 components, double-buffered), f
    case CIP_PRIOR_ITV3D: return 8;  // u, dual p (3 components, double-buffered), f
    case CIP_PRIOR_TV2D: return 4;   // 2 components, double-buffered
    case CIP_PRIOR_TV3D: return 7;   // 3 components, double-buffered; x
    case CIP_PRIOR_PATCH: return 0;  // codes live in their own region
    case CIP_PRIOR_CONV2D: return 0;
    case CIP_PRIOR_CONV3D: return 0;
    case CIP_PRIOR_WDCT3D: return 1;  // v = T x + u
    default: return -1;
  }
}

Layout make_layout(int K, int S, int N1, int N2, const cip_prior_desc* prior) {
  Layout L{};
  const int kind = prior->kind;
  const size_t H2 = N2 / 2 + 1, F = (size_t)N1 * H2, P = (size_t)(K > S ? K : S);
  size_t ot = 0, os = 0, oc = 0;
  auto tab = [&](size_t bytes) {
    size_t r = ot;
    ot += align256(bytes);
    return r;
  };
  auto sta = [&](size_t bytes) {
    size_t r = os;
    os += align256(bytes);
    return r | STATE_BIT;
  };
  auto scr = [&](size_t bytes) {   // plan-time scratch, aliases the state region
    size_t r = oc;
    oc += align256(bytes);
    return r | STATE_BIT;
  };
  L.twN1f = tab(N1 * 8);
  L.twN2f = tab(N2 * 8);
  L.twN2f8 = is_pow2(N2) ? tab(N2 * 8) : 0;   // row twiddles for 8 points per thread
  L.twN1d = tab(N1 * 16);
  L.twN2d = tab(N2 * 16);
  L.ew1 = tab(N1 * 8);
  L.ew2 = tab(N2 * 8);
  L.lam32 = tab((size_t)K * S * F * 8);
  L.Adiag = tab((size_t)S * F * 4);
  L.Aoff = tab((size_t)(S * (S - 1) / 2) * F * 8 + 8);
  L.Mm = tab((size_t)S * K * F * 8);
  L.band = kind == CIP_PRIOR_DCT3D ? tab((size_t)S * S * 4) : 0;   // band DCT matrix C_S
  L.xh0 = sta((size_t)S * F * 8);
  L.bufA = sta(P * F * 8);
  L.bufB = sta(P * F * 8);
  L.state = sta((size_t)state_floats_per_voxel(kind) * S * N1 * N2 * 4);
  const bool adaptive = (prior->flags & CIP_PLAN_ADAPTIVE) != 0;
  const bool synthesis = kind == CIP_PRIOR_PATCH || kind == CIP_PRIOR_CONV2D ||
                         kind == CIP_PRIOR_CONV3D;
  // the FP64 spectra stay resident when the penalty may change during a solve
  // (analysis priors: Psi depends on rho; the synthesis x-update does not)
  L.lam64 = adaptive && !synthesis ? tab((size_t)K * S * F * 16) : scr((size_t)K * S * F * 16);
  if (adaptive) {
    L.xbuf = sta((size_t)2 * S * N1 * N2 * 4);      // x^(l-1), x^l of the checks
    size_t nsum = (size_t)S * (N1 / 8) * 4;         // norm-pass partial sums
    if (kind == CIP_PRIOR_PATCH) {
      const size_t ps = patch_z_residual_floats(N1, N2) + 2 * XCHANGE_GROUPS + 4;
      if (ps > nsum) nsum = ps;
    }
    if (kind == CIP_PRIOR_CONV2D || kind == CIP_PRIOR_CONV3D) {
      // row-pass residuals, k_xchange sums, two FP64 totals, the dictionary
      // residuals and their two FP64 totals
      const size_t cs = conv_row_residual_floats(prior->n_filters * S, N1, N2) +
                        2 * XCHANGE_GROUPS + 4 + 2 * CDL_RES_GROUPS + 4;
      if (cs > nsum) nsum = cs;
    }
    if (kind == CIP_PRIOR_WDCT3D) {
      // state-pass residuals, k_xchange sums, two FP64 totals
      const size_t ws = 2 * (size_t)wavelet_state_groups(N1, N2) + 2 * XCHANGE_GROUPS + 4;
      if (ws > nsum) nsum = ws;
    }
    L.sums = sta(nsum * 4);
  }
  if (adaptive && (kind == CIP_PRIOR_ITV2D || kind == CIP_PRIOR_ITV3D))
    L.tprev = sta((size_t)S * N1 * N2 * 4);
  L.rt64 = scr(F * 16);
  L.pl64 = scr((size_t)N1 * N2 * 8);
  if (kind == CIP_PRIOR_WDCT3D) {
    L.wband = tab((size_t)S * S * 4);
    L.wcoef = sta((size_t)S * N1 * N2 * 4);
    L.wtmp = sta((size_t)S * N1 * N2 * 4);
    L.rimg = sta((size_t)S * N1 * N2 * 4);
  }
  if (kind == CIP_PRIOR_PATCH) {
    const size_t nv = (size_t)64 * S, na = (size_t)prior->n_atoms;
    const size_t J = (size_t)(N1 / 4) * (N2 / 4);
    // a learned dictionary changes D and M1 during a solve: they then belong
    // to the solve state, and the plan keeps the tables of its initial one
    const bool learn = (prior->flags & CIP_PLAN_DICT_UPDATE) != 0;
    L.dbf = learn ? sta(nv * na * 2) : tab(nv * na * 2);
    L.m1bf = learn ? sta(na * nv * 2) : tab(na * nv * 2);
    if (learn) {
      const size_t KS = (size_t)patch_dict_splits(N1, N2);
      L.dbf0 = tab(nv * na * 2);
      L.m1bf0 = tab(na * nv * 2);
      L.pd0 = tab(nv * na * 4);
      L.pzf = sta(na * J * 4);
      L.ppart = sta(KS * (nv + na) * na * 8);
      L.pbm = sta(nv * na * 8);
      L.pd = sta(nv * na * 8);
      L.pcm = sta((size_t)256 * 256 * 4);
      L.plt = sta((size_t)256 * 256 * 4);
      L.pcm64 = sta((size_t)256 * 256 * 8);
      L.plt64 = sta((size_t)2 * 256 * 256 * 8);
      L.pg = sta(nv * na * 4);
      L.pe = sta(nv * na * 4);
    }
    L.vpatch = sta(na * J * 4);
    L.tbuf = sta(patch_tile_buffer_floats(S, N1, N2) * 4);
    L.rimg = sta((size_t)S * N1 * N2 * 4);
  }
  if (kind == CIP_PRIOR_CONV2D || kind == CIP_PRIOR_CONV3D) {
    const size_t M = (size_t)prior->n_filters;
    const size_t B = kind == CIP_PRIOR_CONV3D ? (size_t)S : 1;   // band frequencies
    // a learned dictionary changes the filter tables during a solve: they
    // then belong to the solve state
    const bool learn = (prior->flags & CIP_PLAN_DICT_UPDATE) != 0;
    L.th32 = learn ? sta(M * B * F * 8) : tab(M * B * F * 8);
    L.gam = learn ? sta(B * F * 4) : tab(B * F * 4);
    if (learn) {
      // filter planes: M S (3D) or M (2D, common filters)
      const size_t P = M * B;
      const size_t taps = P * (size_t)prior->filt_l * prior->filt_l;
      L.filt0 = tab(taps * 4);
      L.gtap = sta(taps * 4);
      L.gehat = sta(P * F * 8);
      L.dsp = sta(P * F * 8);
      L.ecdl = sta(P * F * 8);   // the dual as plane spectra
      L.dpl = sta(P * (size_t)N1 * N2 * 4);
      if (adaptive) L.gprev = sta(taps * 4);
    }
    L.eta = learn ? sta(F * 4) : tab(F * 4);
    L.bw = kind == CIP_PRIOR_CONV3D ? tab((size_t)S * S * 8) : 0;
    L.gv = sta(M * S * F * 8);
    L.dhat = sta((size_t)S * F * 8);
    L.xhat = sta((size_t)S * F * 8);
    L.rtc = sta(M * S * F * 8);
    L.vconv = sta(M * S * (size_t)N1 * N2 * 4);
    // the FP64 filter spectra stay resident when the penalty may change
    // during a solve (the z-update tables are rebuilt from them)
    L.th64 = adaptive && !learn ? tab(M * B * F * 16) : scr(M * B * F * 16);
  }
  L.tables = ot;
  L.state_bytes = os > oc ? os : oc;
  L.total = L.tables + L.state_bytes;
  return L;
}

int validate(int K, int S, int N1, int N2, const cip_prior_desc* prior) {
  if (!prior) return fail(CIP_EINVAL, "prior descriptor is NULL");
  if (K < 1 || K > 8 || S < 1 || S > 8) return fail(CIP_EINVAL, "K and S must be in [1, 8]");
  if (!size_supported(N1) || !size_supported(N2))
    return fail(CIP_EUNSUPPORTED,
                "N1 and N2 must be powers of two in [16, 2048] or one of 384, 768, 1536");
  if (state_floats_per_voxel(prior->kind) < 0)
    return fail(CIP_EUNSUPPORTED, "unsupported prior kind");
  if (!(prior->beta > 0.0)) return fail(CIP_EINVAL, "beta must be > 0");
  if ((prior->kind == CIP_PRIOR_ITV2D || prior->kind == CIP_PRIOR_ITV3D) &&
      (prior->tv_inner < 0 || prior->tv_inner > 10000))
    return fail(CIP_EINVAL, "tv_inner must be in [0, 10000]");
  if (prior->kind == CIP_PRIOR_WDCT3D) {
    const int lv = prior->wt_levels > 0 ? prior->wt_levels : 3;
    if (prior->wt_levels < 0 || lv > 10) return fail(CIP_EINVAL, "wt_levels must be in [0, 10]");
    if (N1 % (1 << lv) || N2 % (1 << lv))
      return fail(CIP_EUNSUPPORTED, "wavelet prior: N1 and N2 must be multiples of 2^wt_levels");
  }
  if (prior->kind == CIP_PRIOR_PATCH) {
    if (!is_pow2(N1) || !is_pow2(N2))
      return fail(CIP_EUNSUPPORTED, "patch prior: power-of-two grids only");
    if (prior->patch_q != 8 || prior->patch_stride != 4)
      return fail(CIP_EUNSUPPORTED, "patch prior: only 8 x 8 x S patches at stride 4");
    if (!patch_supported(S, prior->n_atoms))
      return fail(CIP_EUNSUPPORTED, "patch prior: needs S <= 4 and 64, 128 or 256 atoms");
    if (!patch_grid_ok(N1, N2)) return fail(CIP_EUNSUPPORTED, "patch prior: grid too small");
    if (prior->patch_t != 0 && prior->patch_t != S)
      return fail(CIP_EUNSUPPORTED, "patch prior: patches must span every plane (patch_t 0 or S)");
  }
  if (prior->kind == CIP_PRIOR_CONV2D) {
    if (prior->per_band == 1)
      return fail(CIP_EUNSUPPORTED, "conv prior: only a common filter set for every plane");
    if (prior->per_band != 0) return fail(CIP_EINVAL, "per_band must be 0 or 1");
  }
  if (prior->kind == CIP_PRIOR_CONV2D || prior->kind == CIP_PRIOR_CONV3D) {
    if (prior->n_filters < 1 || prior->n_filters > 32)
      return fail(CIP_EUNSUPPORTED, "conv prior: 1 to 32 filters");
    if (prior->filt_l < 1 || prior->filt_l > N1 || prior->filt_l > N2)
      return fail(CIP_EINVAL, "conv prior: filter size must be in [1, min(N1, N2)]");
    if (!(prior->mu >= 0.0)) return fail(CIP_EINVAL, "conv prior: mu must be >= 0");
    if (prior->kind == CIP_PRIOR_CONV3D && prior->mu != 0.0)
      return fail(CIP_EUNSUPPORTED, "3D conv prior: no gradient term (mu must be 0)");
  }
  if (prior->flags & CIP_PLAN_DICT_UPDATE) {
    if (prior->kind != CIP_PRIOR_CONV3D && prior->kind != CIP_PRIOR_CONV2D &&
        prior->kind != CIP_PRIOR_PATCH)
      return fail(CIP_EUNSUPPORTED, "dictionary learning: patch and convolutional priors only");
    if (!(prior->sigma >= 0.0)) return fail(CIP_EINVAL, "sigma must be >= 0");
  }
  return CIP_OK;
}

}  // namespace

struct cip_plan_s {
  int K, S, N1, N2, H2, kind, n_atoms, n_filters;
  double beta, rho, lambda;
  unsigned char* ws;    // table region
  unsigned char* sws;   // state region
  Layout L;
  bool solved_once;
  bool attached;        // shares another plan's tables
  bool adaptive;        // FP64 spectra resident: the penalty may change in a solve
  bool learn;           // the dictionary is learned during every solve
  double sigma;         // penalty of the dictionary ADMM
  double mu;            // conv prior: gradient (Tikhonov) weight
  int filt_l;           // conv priors: filter side L
  int row_np;           // row pairs per work-group of the DCT row pass (2 or 4)
  int row_ppt;          // points per thread of the analysis row passes (default or 8)
  int tv_inner;         // isotropic TV: Chambolle iterations per ADMM iteration
  int wt_levels;        // wavelet (x) DCT: levels of the 2D wavelet transform
  std::vector<float> dict_host;   // patch prior with CIP_PLAN_ADAPTIVE: D, to rebuild M1
  // analysis priors: the iteration loop of a solve (iterations 2 .. iters)
  // captured into a hipGraph once the plan has been solved twice in a row
  // with the same iteration count; rebuilt when that count or the row-pass
  // shape changes
  hipGraph_t loop_graph = nullptr;
  hipGraphExec_t loop_exec = nullptr;
  int loop_iters = 0;   // iteration count the graph was captured for (0: none)
  int last_iters = 0;   // iteration count of the previous solve
  void drop_loop_graph() {
    if (loop_exec) (void)hipGraphExecDestroy(loop_exec);
    if (loop_graph) (void)hipGraphDestroy(loop_graph);
    loop_exec = nullptr;
    loop_graph = nullptr;
    loop_iters = 0;
  }
  ~cip_plan_s() { drop_loop_graph(); }
  template <typename T> T* at(size_t off) const {
    return reinterpret_cast<T*>((off & STATE_BIT) ? sws + (off & ~STATE_BIT) : ws + off);
  }
};

bool is_dct(const cip_plan_s* p) {
  return p->kind == CIP_PRIOR_DCT2D || p->kind == CIP_PRIOR_DCT3D;
}

bool is_itv(const cip_plan_s* p) {
  return p->kind == CIP_PRIOR_ITV2D || p->kind == CIP_PRIOR_ITV3D;
}

// ---------------------------------------------------------------- launch helpers
namespace {



#define DISPATCH_N CIP_DISPATCH_N

template <typename Re>
hipError_t row_r2c(const Re* in, cx<Re>* out, int P, int N1, int N2, const cx<Re>* tw, hipStream_t st) {
  constexpr bool staged = sizeof(Re) == 4;
  DISPATCH_N(N2, {
    const int T = NN / ppt_row<NN>();
    const int ng = staged ? PAIRS : 1;
    size_t lds = (size_t)(2 * NN + row_work_floats<NN, Re>(ng, staged)) * sizeof(Re);
    int grid = staged ? P * (N1 / RT) : P * (N1 / 2);
    return launch(k_row_r2c<NN, Re, staged>, grid, ng * T, lds, st, in, out, N1, tw);
  });
  return hipSuccess;
}

hipError_t row_c2r(const cx<float>* in, float* out, int P, int N1, int N2, float scale,
                   const cx<float>* tw, hipStream_t st) {
  DISPATCH_N(N2, {
    const int T = NN / ppt_row<NN>();
    size_t lds = (size_t)(2 * NN + row_work_floats<NN, float>(PAIRS, true)) * 4;
    return launch(k_row_c2r<NN>, P * (N1 / RT), PAIRS * T, lds, st, in, out, N1, scale, tw);
  });
  return hipSuccess;
}

template <typename Re, int OP>
hipError_t col_op(const cx<Re>* in, void* out, int Pin, int Pout, int N1, int H2,
                  const cx<Re>* tw, const cx<Re>* mat, int spec_plane, hipStream_t st) {
  const int PM = Pin > Pout ? Pin : Pout;
  DISPATCH_N(N1, {
    const int T = NN / ppt_col<NN>();
    size_t lds = (size_t)(2 * NN + PM * 2 * padded_len(NN)) * sizeof(Re);
    return launch(k_col_op<NN, Re, OP>, H2, PM * T, lds, st, in, out, Pin, Pout, H2, tw, mat,
                  spec_plane);
  });
  return hipSuccess;
}

// rho: penalty of the current iteration (the plan's unless the adaptive solve
// changed it); sc = rho / rho_next when the penalty changes after this pass
// (the state is then re-expressed for rho_next), else 1.
hipError_t admm_row_dct(cip_plan_t p, int mode, hipStream_t st, float* xout, double rho = 0.0,
                        float sc = 1.f) {
  const Layout& L = p->L;
  float kappa = (float)(p->lambda / (rho > 0.0 ? rho : p->rho));
  auto run = [&](auto kern, int NN, int np, int ppt, size_t work_floats) {
    return launch(kern, p->S * (p->N1 / RT) * (PAIRS / np), np * (NN / ppt),
                  (size_t)(4 * NN + work_floats) * 4, st, p->at<const cx<float>>(L.bufB),
                  p->at<cx<float>>(L.bufA), p->at<float>(L.state), p->N1,
                  p->at<const cx<float>>(ppt == ppt_row_n(NN) ? L.twN2f : L.twN2f8),
                  p->at<const cx<float>>(L.ew2), kappa, mode, xout, sc);
  };
  DISPATCH_N(p->N2, {
    constexpr int PD = ppt_row<NN>();
    constexpr int P8 = ((NN & (NN - 1)) == 0 && NN >= 16) ? 8 : PD;
    const bool alt = p->row_ppt == 8 && P8 != PD;   // tuning variant
    if (alt && p->row_np == 2)
      return run(k_admm_row_dct<NN, 2, P8>, NN, 2, P8, row_work_floats<NN, float>(2, true));
    if (alt) return run(k_admm_row_dct<NN, 4, P8>, NN, 4, P8, row_work_floats<NN, float>(4, true));
    if (p->row_np == 2)
      return run(k_admm_row_dct<NN, 2, PD>, NN, 2, PD, row_work_floats<NN, float>(2, true));
    return run(k_admm_row_dct<NN, 4, PD>, NN, 4, PD, row_work_floats<NN, float>(4, true));
  });
  return hipSuccess;
}

// Row pass of the TV priors; pass number l >= 1 of the solve (state buffers
// alternate so that halo rows of the previous state stay readable).
// x_ready (TV3D): the x buffer already holds x of the current spectra (the
// norm pass of this iteration wrote it).
hipError_t admm_row_tv(cip_plan_t p, int l, hipStream_t st, double rho = 0.0, float sc = 1.f,
                       bool x_ready = false) {
  const Layout& L = p->L;
  float kappa = (float)(p->lambda / (rho > 0.0 ? rho : p->rho));
  const bool band = p->kind == CIP_PRIOR_TV3D;
  const size_t buf = (size_t)(band ? 3 : 2) * p->S * p->N1 * p->N2;
  const float* vin = p->at<float>(L.state) + (size_t)((l + 1) & 1) * buf;
  float* vout = p->at<float>(L.state) + (size_t)(l & 1) * buf;
  auto run = [&](auto kern, int threads, size_t work_floats, bool use8, int parts = 1) {
    return launch(kern, p->S * (p->N1 / RT) * parts, threads,
                  (size_t)(2 * p->N2 + work_floats) * 4, st,
                  p->at<const cx<float>>(L.bufB), p->at<cx<float>>(L.bufA), vin, vout, p->S,
                  p->N1, p->at<const cx<float>>(use8 ? L.twN2f8 : L.twN2f), kappa,
                  l == 1 ? 1 : 0, sc);
  };
  // TV3D: x of every plane in image space once (after both state buffers),
  // then the row pass reads the neighbouring planes' rows from it
  float* xim = p->at<float>(L.state) + 2 * buf;
  auto run3 = [&](auto kern, int threads, size_t work_floats, bool use8, int parts = 1) {
    if (!x_ready) {
      hipError_t e = row_c2r(p->at<const cx<float>>(L.bufB), xim, p->S, p->N1, p->N2, 1.0f,
                             p->at<const cx<float>>(L.twN2f), st);
      if (e != hipSuccess) return e;
    }
    return launch(kern, p->S * (p->N1 / RT) * parts, threads,
                  (size_t)(2 * p->N2 + work_floats) * 4, st, (const float*)xim,
                  p->at<cx<float>>(L.bufA), vin, vout, p->S, p->N1,
                  p->at<const cx<float>>(use8 ? L.twN2f8 : L.twN2f), kappa, l == 1 ? 1 : 0, sc);
  };
  DISPATCH_N(p->N2, {
    constexpr int PD = ppt_row<NN>();
    // 8 points per thread only where the work-group stays within 1024 threads
    constexpr int P8 = ((NN & (NN - 1)) == 0 && NN >= 16 && NN <= 1024) ? 8 : PD;
    const bool use8 = p->row_ppt == 8 && P8 != PD;   // tuning variant
    const int threads = (PAIRS + 1) * (NN / (use8 ? P8 : PD));
    if (p->row_np == 2) {   // half tiles: 2 own row pairs per work-group
      const int th2 = 3 * (NN / (use8 ? P8 : PD));
      if (band)
        return use8 ? run3(k_admm_row_tv3<NN, P8, 2>, th2, tv_work_floats<NN, 2>(), true, RT / 4)
                    : run3(k_admm_row_tv3<NN, PD, 2>, th2, tv_work_floats<NN, 2>(), false, RT / 4);
      return use8 ? run(k_admm_row_tv<NN, P8, 2>, th2, tv_work_floats<NN, 2>(), true, RT / 4)
                  : run(k_admm_row_tv<NN, PD, 2>, th2, tv_work_floats<NN, 2>(), false, RT / 4);
    }
    if (band)
      return use8 ? run3(k_admm_row_tv3<NN, P8>, threads, tv_work_floats<NN>(), true)
                  : run3(k_admm_row_tv3<NN, PD>, threads, tv_work_floats<NN>(), false);
    return use8 ? run(k_admm_row_tv<NN, P8>, threads, tv_work_floats<NN>(), true)
                : run(k_admm_row_tv<NN, PD>, threads, tv_work_floats<NN>(), false);
  });
  return hipSuccess;
}

// Isotropic TV t-update and dual update of pass l (see itv.hpp). The dual
// alternates between buffers A and B over the Chambolle launches; pass l
// starts from the buffer where pass l - 1 left it (A for l = 1, zeroed by the
// prep kernel).
// Chambolle iterations per launch (= tile halo). Measured at 1024^2 x 3 with
// 20 iterations (per-plane TV): 4 -> 204 us, 5 -> 189 us, 8 -> 204 us,
// 10 -> 207 us per ADMM row pass; the results are bitwise the same for every
// halo.
constexpr int ITV_KB = 5;

// Band-coupled Chambolle launch: the tile side is 32 where all S planes of a
// 42 x 42 region fit in 64 KiB of LDS (S <= 3) and the grid allows it, else 16.
constexpr int ITV3_NT = 512;
template <int S_>
hipError_t itv3_launch(bool t32, int grid32, int grid16, hipStream_t st, const float* f,
                       float* const* in, float* const* out, int N1, int N2, int m, float inv_mu) {
  if constexpr (S_ <= 3) {
    if (t32)
      return launch(k_itv3_chambolle<S_, 32, ITV_KB, ITV3_NT>, grid32, ITV3_NT, 0, st, f, in[0],
                    in[1], in[2], out[0], out[1], out[2], N1, N2, m, inv_mu, 1.f / 12.f);
  }
  return launch(k_itv3_chambolle<S_, 16, ITV_KB, ITV3_NT>, grid16, ITV3_NT, 0, st, f, in[0],
                in[1], in[2], out[0], out[1], out[2], N1, N2, m, inv_mu, 1.f / 12.f);
}

// Dual buffers of the isotropic TV state: pd[b][c] is component c of buffer b
// (component 2 only when coupled along the bands).
struct ItvState {
  float* u;
  float* pd[2][3];
  float* f;
  int nl;   // Chambolle launches per ADMM iteration
};

ItvState itv_state(cip_plan_t p) {
  const size_t n = (size_t)p->S * p->N1 * p->N2;
  const bool band = p->kind == CIP_PRIOR_ITV3D;
  const int nc = band ? 3 : 2;
  ItvState s;
  s.u = p->at<float>(p->L.state);
  float* u = s.u;
  s.pd[0][0] = u + n;
  s.pd[0][1] = u + 2 * n;
  s.pd[0][2] = band ? u + 3 * n : nullptr;
  s.pd[1][0] = u + (1 + nc) * n;
  s.pd[1][1] = u + (2 + nc) * n;
  s.pd[1][2] = band ? u + 6 * n : nullptr;
  s.f = u + (1 + 2 * nc) * n;
  s.nl = (p->tv_inner + ITV_KB - 1) / ITV_KB;
  return s;
}

// Closing row pass of iteration l: t = f - mu div p, u = c (f - t), spectrum
// of t - u to bufA. Pass l leaves the dual in buffer (l nl) mod 2.
hipError_t itv_finish(cip_plan_t p, int l, float mu, float c, hipStream_t st) {
  const ItvState sv = itv_state(p);
  const int fin = (int)(((long long)l * sv.nl) & 1);
  const int grid = p->S * (p->N1 / RT);
  const bool band = p->kind == CIP_PRIOR_ITV3D;
  DISPATCH_N(p->N2, {
    const int T = NN / ppt_row<NN>();
    size_t lds = (size_t)(2 * NN + row_work_floats<NN, float>(PAIRS, true)) * 4;
    return band ? launch(k_itv_finish<NN, true>, grid, PAIRS * T, lds, st, sv.f, sv.pd[fin][0],
                         sv.pd[fin][1], sv.pd[fin][2], p->S, sv.u, p->at<cx<float>>(p->L.bufA),
                         p->N1, p->at<const cx<float>>(p->L.twN2f), mu, c)
                : launch(k_itv_finish<NN, false>, grid, PAIRS * T, lds, st, sv.f, sv.pd[fin][0],
                         sv.pd[fin][1], sv.pd[fin][2], p->S, sv.u, p->at<cx<float>>(p->L.bufA),
                         p->N1, p->at<const cx<float>>(p->L.twN2f), mu, c);
  });
  return hipSuccess;
}

// xo: when given, x^l is also written there (adaptive checks).
hipError_t itv_row(cip_plan_t p, int l, hipStream_t st, double rho, float* xo = nullptr) {
  const Layout& L = p->L;
  const float mu = (float)(p->lambda / (rho > 0.0 ? rho : p->rho));
  const bool band = p->kind == CIP_PRIOR_ITV3D;
  const ItvState sv = itv_state(p);
  const int nl = sv.nl;
  const int start = (int)(((long long)(l - 1) * nl) & 1);
  const int grid = p->S * (p->N1 / RT);
  hipError_t e = hipSuccess;
  DISPATCH_N(p->N2, {
    const int T = NN / ppt_row<NN>();
    size_t lds = (size_t)(2 * NN + row_work_floats<NN, float>(PAIRS, true)) * 4;
    e = launch(k_itv_prep<NN>, grid, PAIRS * T, lds, st, p->at<const cx<float>>(L.bufB), sv.u,
               sv.f, sv.pd[start][0], sv.pd[start][1], sv.pd[start][2], xo, p->N1,
               p->at<const cx<float>>(L.twN2f), l == 1 ? 1 : 0);
  });
  if (e != hipSuccess) return e;
  const bool t32 = p->N1 % 32 == 0 && p->N2 % 32 == 0;
  const int ts = t32 ? 32 : 16;
  const int cgrid = p->S * (p->N1 / ts) * (p->N2 / ts);
  const int g32 = t32 ? (p->N1 / 32) * (p->N2 / 32) : 0, g16 = (p->N1 / 16) * (p->N2 / 16);
  for (int j = 0; j < nl; ++j) {
    const int in = (start + j) & 1, out = in ^ 1;
    const int m = std::min(ITV_KB, p->tv_inner - j * ITV_KB);
    float* const* pin = sv.pd[in];
    float* const* pout = sv.pd[out];
    if (band) {
      switch (p->S) {
#define ITV3_CASE(SS)                                                                       \
  case SS:                                                                                  \
    e = itv3_launch<SS>(t32, g32, g16, st, sv.f, pin, pout, p->N1, p->N2, m, 1.f / mu);     \
    break;
        ITV3_CASE(1) ITV3_CASE(2) ITV3_CASE(3) ITV3_CASE(4)
        ITV3_CASE(5) ITV3_CASE(6) ITV3_CASE(7) ITV3_CASE(8)
#undef ITV3_CASE
        default: return hipErrorInvalidValue;
      }
    } else {
      e = t32 ? launch(k_itv_chambolle<32, ITV_KB>, cgrid, 256, 0, st, sv.f, pin[0], pin[1],
                       pout[0], pout[1], p->N1, p->N2, m, 1.f / mu, 0.125f)
              : launch(k_itv_chambolle<16, ITV_KB>, cgrid, 256, 0, st, sv.f, pin[0], pin[1],
                       pout[0], pout[1], p->N1, p->N2, m, 1.f / mu, 0.125f);
    }
    if (e != hipSuccess) return e;
  }
  return itv_finish(p, l, mu, 1.f, st);
}

hipError_t admm_row(cip_plan_t p, int l, hipStream_t st, double rho = 0.0, float sc = 1.f,
                     bool x_ready = false) {
  if (is_itv(p)) return itv_row(p, l, st, rho);
  if (is_dct(p))
    return admm_row_dct(p, l == 1 ? ROW_FIRST : ROW_FULL, st, nullptr, rho, sc);
  return admm_row_tv(p, l, st, rho, sc, x_ready);
}

// Norm pass of a checked iteration l (see norms.hpp): partial sums to
// L.sums, one float4 per work-group; returns the number of work-groups.
hipError_t norm_pass(cip_plan_t p, int l, double rho, float* xcur, const float* xprev,
                     hipStream_t st, int* groups) {
  const Layout& L = p->L;
  const float kappa = (float)(p->lambda / rho);
  const int first = l == 1 ? 1 : 0;
  const int grid = p->S * (p->N1 / RT);
  *groups = grid;
  if (is_dct(p)) {
    DISPATCH_N(p->N2, {
      const int T = NN / ppt_row<NN>();
      size_t lds = (size_t)(4 * NN + row_work_floats<NN, float>(PAIRS, true)) * 4;
      return launch(k_norm_dct<NN>, grid, PAIRS * T, lds, st, p->at<const cx<float>>(L.bufB),
                    p->at<const float>(L.state), p->N1, p->at<const cx<float>>(L.twN2f),
                    p->at<const cx<float>>(L.ew2), kappa, first, xcur, xprev,
                    p->at<float>(L.sums));
    });
    return hipSuccess;
  }
  const bool band = p->kind == CIP_PRIOR_TV3D;
  const size_t buf = (size_t)(band ? 3 : 2) * p->S * p->N1 * p->N2;
  const float* vin = p->at<float>(L.state) + (size_t)((l + 1) & 1) * buf;
  // TV3D: x of every plane to the x buffer of the state (the row pass that
  // follows on the same spectra is told that it is there)
  float* xim = p->at<float>(L.state) + 2 * buf;
  if (band) {
    hipError_t e = row_c2r(p->at<const cx<float>>(L.bufB), xim, p->S, p->N1, p->N2, 1.0f,
                           p->at<const cx<float>>(L.twN2f), st);
    if (e != hipSuccess) return e;
  }
  DISPATCH_N(p->N2, {
    const int T = NN / ppt_row<NN>();
    size_t lds = (size_t)(2 * NN + tv_work_floats<NN>()) * 4;
    if (band)
      return launch(k_norm_tv<NN, true>, grid, (PAIRS + 1) * T, lds, st,
                    p->at<const cx<float>>(L.bufB), vin, p->S, p->N1,
                    p->at<const cx<float>>(L.twN2f), kappa, first, xcur, xprev,
                    p->at<float>(L.sums), (const float*)xim);
    return launch(k_norm_tv<NN, false>, grid, (PAIRS + 1) * T, lds, st,
                  p->at<const cx<float>>(L.bufB), vin, p->S, p->N1,
                  p->at<const cx<float>>(L.twN2f), kappa, first, xcur, xprev,
                  p->at<float>(L.sums), (const float*)nullptr);
  });
  return hipSuccess;
}

hipError_t admm_col(cip_plan_t p, int zero_in, int dct_out, hipStream_t st) {
  const Layout& L = p->L;
  const bool dct = is_dct(p);
#define CIP_COL_CASE(NN)                                                                        \
  case NN:                                                                                      \
    return admm_col_launch_##NN(p->S, dct, p->at<const cx<float>>(L.bufA),                      \
                                p->at<cx<float>>(L.bufB), p->H2, p->at<const float>(L.Adiag),    \
                                p->at<const cx<float>>(L.Aoff), p->at<const cx<float>>(L.xh0),   \
                                p->at<const cx<float>>(L.twN1f), p->at<const cx<float>>(L.ew1),  \
                                L.band ? p->at<const float>(L.band) : nullptr, zero_in,          \
                                dct_out, st);
  switch (p->N1) {
    CIP_FOR_EACH_SIZE(CIP_COL_CASE)
  }
#undef CIP_COL_CASE
  return hipErrorInvalidValue;
}

// Algorithm 2 with the patch prior. Per iteration l = 1..L:
//   x-update (Eq. solx_synt_DFT): row FFT of r = P^T D~ z^{l-1} (r = 0 for
//   l = 1), column FFT + per-frequency solve + inverse column FFT, inverse
//   row FFT -> x^l (written to d_x);
//   for l < L: sparse-code update, soft threshold, dual update and the
//   tiles' D z on MFMA (k_patch_z), then r = P^T D~ z^l (k_patch_assemble).
//   With a learned dictionary the code update writes z in FP32 and skips
//   D z; one step of the dictionary ADMM follows (D, G, E and the BF16
//   tables of G), then D z with the new G.
PatchDictBufs patch_dict_bufs(cip_plan_t p) {
  const Layout& L = p->L;
  PatchDictBufs b;
  b.zf = p->at<float>(L.pzf);
  b.part = p->at<double>(L.ppart);
  b.bm = p->at<double>(L.pbm);
  b.d = p->at<double>(L.pd);
  b.cm64 = p->at<double>(L.pcm64);
  b.lt64 = p->at<double>(L.plt64);
  b.cm = p->at<float>(L.pcm);
  b.lt = p->at<float>(L.plt);
  b.g = p->at<float>(L.pg);
  b.e = p->at<float>(L.pe);
  b.dbf = p->at<uint16_t>(L.dbf);
  b.m1bf = p->at<uint16_t>(L.m1bf);
  return b;
}

hipError_t patch_step(cip_plan_t p, const float* x, int first, hipStream_t st) {
  const Layout& L = p->L;
  const float kappa = (float)(p->lambda / p->rho);
  hipError_t e;
  if (p->learn) {
    const PatchDictBufs b = patch_dict_bufs(p);
    e = patch_z_launch(p->S, p->n_atoms, x, p->at<float>(L.vpatch), p->at<float>(L.tbuf), b.dbf,
                       b.m1bf, p->N1, p->N2, kappa, first, st, PZ_MODE_CODES, b.zf);
    if (e != hipSuccess) return e;
    e = patch_dict_step(x, b, p->S, p->n_atoms, p->N1, p->N2, p->sigma, (float)p->rho, st);
    if (e != hipSuccess) return e;
    e = patch_z_launch(p->S, p->n_atoms, x, p->at<float>(L.vpatch), p->at<float>(L.tbuf), b.dbf,
                       b.m1bf, p->N1, p->N2, kappa, first, st, PZ_MODE_SYNTH, b.zf);
  } else {
    e = patch_z_launch(p->S, p->n_atoms, x, p->at<float>(L.vpatch), p->at<float>(L.tbuf),
                       p->at<const uint16_t>(L.dbf), p->at<const uint16_t>(L.m1bf), p->N1, p->N2,
                       kappa, first, st);
  }
  if (e != hipSuccess) return e;
  return patch_assemble_launch(p->S, p->at<const float>(L.tbuf), p->at<float>(L.rimg), p->N1, p->N2,
                               st);
}

// Start of a solve with a learned dictionary: G = the plan's dictionary,
// E = 0, and its BF16 tables.
hipError_t patch_dict_begin(cip_plan_t p, hipStream_t st) {
  const Layout& L = p->L;
  const int nv = 64 * p->S, na = p->n_atoms;
  hipError_t e = hipMemcpyAsync(p->at<void>(L.dbf), p->at<const void>(L.dbf0), (size_t)nv * na * 2,
                                hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(p->at<void>(L.m1bf), p->at<const void>(L.m1bf0), (size_t)nv * na * 2,
                     hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  return patch_dict_start(p->at<const float>(L.pd0), patch_dict_bufs(p), nv, na, st);
}

hipError_t solve_patch(cip_plan_t p, int iters, float* d_x, hipStream_t st) {
  const Layout& L = p->L;
  hipError_t e;
  if (p->learn && (e = patch_dict_begin(p, st)) != hipSuccess) return e;
  for (int l = 1; l <= iters; ++l) {
    if (l > 1) {
      e = row_r2c<float>(p->at<const float>(L.rimg), p->at<cx<float>>(L.bufA), p->S, p->N1, p->N2,
                         p->at<const cx<float>>(L.twN2f), st);
      if (e != hipSuccess) return e;
    }
    if ((e = admm_col(p, l == 1 ? 1 : 0, 0, st)) != hipSuccess) return e;
    e = row_c2r(p->at<const cx<float>>(L.bufB), d_x, p->S, p->N1, p->N2, 1.0f,
                p->at<const cx<float>>(L.twN2f), st);
    if (e != hipSuccess) return e;
    if (l < iters && (e = patch_step(p, d_x, l == 1 ? 1 : 0, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Algorithm 2 with the patch prior and the penalty update and stopping rule
// of Section IV-C (Eq. paramS), the split z = t: at every `every`-th
// iteration l < max_iters, after the code, t and u updates,
//   r = ||z^l - t^l||, s = rho ||t^l - t^(l-1)|| (summed by the code update),
//   c = ||x^l - x^(l-1)|| / ||x^(l-1)|| (k_xchange; x^l is in d_x);
// stop with x^l when c < tol, else change rho by tau when one residual
// exceeds mu times the other: the state is re-expressed for the new penalty
// (u scaled by rho / rho') and M1 = D^T (rho' I + D D^T)^-1 is rebuilt: in
// FP64 on the host for a fixed dictionary (the plan's tables are back at its
// own rho on return), on the GPU from G with online dictionary learning.
// With learning and adapt_sigma the D, G, E step of a checked iteration also
// yields r_d = ||D - G|| and s_d = sigma ||G - G_prev||, and sigma changes
// by the same rule, E rescaled by sigma / sigma'.
void patch_dictionary_tables(const std::vector<float>& D, int nv, int na, double rho,
                             std::vector<uint16_t>& dbf, std::vector<uint16_t>& m1bf);

int solve_patch_adaptive(cip_plan_t p, const cip_adaptive_params* prm, float* d_x, hipStream_t st,
                         cip_solve_info& out) {
  const Layout& L = p->L;
  const int iters = prm->max_iters, every = prm->every;
  const int nv = 64 * p->S, na = p->n_atoms;
  const double rho0 = p->rho;
  double rho = rho0, sigma = p->sigma;
  const size_t nres = patch_z_residual_floats(p->N1, p->N2);
  float* rs = p->at<float>(L.sums);
  float* xs = rs + nres;
  double* dres = reinterpret_cast<double*>(xs + 2 * XCHANGE_GROUPS);
  float* xprev = p->at<float>(L.xbuf);
  const size_t nx = (size_t)p->S * p->N1 * p->N2;
  const size_t ncode = (size_t)na * (p->N1 / 4) * (p->N2 / 4);
  // code-update sums, k_xchange sums, the dictionary residuals (2 doubles)
  std::vector<float> hs(nres + 2 * XCHANGE_GROUPS + 4);
  const PatchDictBufs db = p->learn ? patch_dict_bufs(p) : PatchDictBufs{};
  auto set_m1 = [&](double r) -> int {
    if (p->learn) {
      HIP_TRY(patch_dict_m1(db, p->S, na, (float)r, st));
      return CIP_OK;
    }
    std::vector<uint16_t> dbf, m1bf;
    patch_dictionary_tables(p->dict_host, nv, na, r, dbf, m1bf);
    HIP_TRY(hipMemcpyAsync(p->at<void>(L.m1bf), m1bf.data(), m1bf.size() * 2,
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // m1bf is host memory of this scope
    return CIP_OK;
  };
  int rc = CIP_OK;
  if (p->learn) HIP_TRY(patch_dict_begin(p, st));
  for (int l = 1;; ++l) {
    // x-update (Eq. solx_synt_DFT) -> x^l in d_x
    if (l > 1)
      HIP_TRY(row_r2c<float>(p->at<const float>(L.rimg), p->at<cx<float>>(L.bufA), p->S, p->N1,
                             p->N2, p->at<const cx<float>>(L.twN2f), st));
    HIP_TRY(admm_col(p, l == 1 ? 1 : 0, 0, st));
    HIP_TRY(row_c2r(p->at<const cx<float>>(L.bufB), d_x, p->S, p->N1, p->N2, 1.0f,
                    p->at<const cx<float>>(L.twN2f), st));
    if (l == iters) {
      out.iters = l;
      break;
    }
    const bool check = l % every == 0;
    const bool store = (l + 1) % every == 0;
    const bool check_sigma = check && p->learn && prm->adapt_sigma;
    const float kappa = (float)(p->lambda / rho);
    if (p->learn) {
      // codes in FP32, one D, G, E step, then D z with the new G
      HIP_TRY(patch_z_launch(p->S, na, d_x, p->at<float>(L.vpatch), p->at<float>(L.tbuf), db.dbf,
                             db.m1bf, p->N1, p->N2, kappa, l == 1 ? 1 : 0, st, PZ_MODE_CODES,
                             db.zf, check ? rs : nullptr));
      HIP_TRY(patch_dict_step(d_x, db, p->S, na, p->N1, p->N2, sigma, (float)rho, st,
                              check_sigma ? dres : nullptr));
      HIP_TRY(patch_z_launch(p->S, na, d_x, p->at<float>(L.vpatch), p->at<float>(L.tbuf), db.dbf,
                             db.m1bf, p->N1, p->N2, kappa, l == 1 ? 1 : 0, st, PZ_MODE_SYNTH,
                             db.zf));
    } else {
      HIP_TRY(patch_z_launch(p->S, na, d_x, p->at<float>(L.vpatch), p->at<float>(L.tbuf),
                             p->at<const uint16_t>(L.dbf), p->at<const uint16_t>(L.m1bf), p->N1,
                             p->N2, kappa, l == 1 ? 1 : 0, st, PZ_MODE_FULL, nullptr,
                             check ? rs : nullptr));
    }
    HIP_TRY(patch_assemble_launch(p->S, p->at<const float>(L.tbuf), p->at<float>(L.rimg), p->N1,
                                  p->N2, st));
    if (check || store)
      HIP_TRY(launch(k_xchange, XCHANGE_GROUPS, 256, 0, st, (const float*)d_x, xprev, xs, nx,
                     check && l > 1 ? 1 : 0));
    if (!check) continue;
    HIP_TRY(hipMemcpyAsync(hs.data(), rs, hs.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double r2 = 0.0, s2 = 0.0, d2 = 0.0, p2 = 0.0, td[2];
    for (size_t i = 0; i < nres; i += 2) {
      r2 += hs[i];
      s2 += hs[i + 1];
    }
    for (int b = 0; b < XCHANGE_GROUPS; ++b) {
      d2 += hs[nres + 2 * b];
      p2 += hs[nres + 2 * b + 1];
    }
    std::memcpy(td, hs.data() + nres + 2 * XCHANGE_GROUPS, sizeof td);
    const double r = std::sqrt(r2), sres = rho * std::sqrt(s2);
    out.r_norm = r;
    out.s_norm = sres;
    if (l > 1) {
      out.rel_change = p2 > 0.0 ? std::sqrt(d2 / p2) : 0.0;
      if (out.rel_change < prm->tol) {
        out.iters = l;
        break;
      }
    }
    double next = rho;
    if (r > prm->mu * sres) next = prm->tau * rho;
    else if (sres > prm->mu * r) next = rho / prm->tau;
    if (next != rho) {
      HIP_TRY(launch(k_rescale_state, 1024, 256, 0, st, p->at<float>(L.vpatch), ncode, kappa,
                     (float)(rho / next)));
      if ((rc = set_m1(next)) != CIP_OK) break;
      rho = next;
      ++out.rho_changes;
    }
    if (check_sigma) {
      const double rd = std::sqrt(td[0]), sd = sigma * std::sqrt(td[1]);
      double ns = sigma;
      if (rd > prm->mu * sd) ns = prm->tau * sigma;
      else if (sd > prm->mu * rd) ns = sigma / prm->tau;
      if (ns != sigma) {
        HIP_TRY(patch_dict_scale_dual(db, nv * na, (float)(sigma / ns), st));
        sigma = ns;
        ++out.sigma_changes;
      }
    }
  }
  out.rho = rho;
  out.sigma = p->learn ? sigma : 0.0;
  if (rho != rho0 && !p->learn) {   // leave the plan's tables at its own penalty
    const int rc2 = set_m1(rho0);
    if (rc == CIP_OK) rc = rc2;
  }
  return rc;
}

// Algorithm 1 with the wavelet (x) DCT prior. Per iteration l = 1..L:
//   x-update (Eq. solx_Trans_DFT, T^T T = I): row FFT of r = T^T (t - u)
//   (r = 0 for l = 1), column FFT + per-frequency solve (rhs b + rho r^) +
//   inverse column FFT, inverse row FFT -> x^l (written to d_x);
//   for l < L: forward wavelet levels of x^l, band DCT, soft threshold and
//   dual update in v-form (Eqs. solt_trans, subu_trans), inverse band DCT and
//   wavelet levels of t - u -> r.
hipError_t solve_wdct(cip_plan_t p, int iters, float* d_x, hipStream_t st) {
  const Layout& L = p->L;
  const int S = p->S, N1 = p->N1, N2 = p->N2, lv = p->wt_levels;
  const float kappa = (float)(p->lambda / p->rho);
  float* coef = p->at<float>(L.wcoef);
  float* tmp = p->at<float>(L.wtmp);
  float* r = p->at<float>(L.rimg);
  hipError_t e;
  for (int l = 1; l <= iters; ++l) {
    if (l > 1 && (e = row_r2c<float>(r, p->at<cx<float>>(L.bufA), S, N1, N2,
                                     p->at<const cx<float>>(L.twN2f), st)) != hipSuccess)
      return e;
    if ((e = admm_col(p, l == 1 ? 1 : 0, 0, st)) != hipSuccess) return e;
    if ((e = row_c2r(p->at<const cx<float>>(L.bufB), d_x, S, N1, N2, 1.0f,
                     p->at<const cx<float>>(L.twN2f), st)) != hipSuccess)
      return e;
    if (l == iters) break;
    if ((e = wavelet_forward(d_x, coef, tmp, S, N1, N2, lv, st)) != hipSuccess) return e;
    if ((e = wavelet_state(coef, p->at<float>(L.state), p->at<const float>(L.wband), S, N1, N2,
                           kappa, l == 1 ? 1 : 0, st)) != hipSuccess)
      return e;
    if ((e = wavelet_inverse(coef, r, tmp, S, N1, N2, lv, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Algorithm 1 with the wavelet (x) DCT prior and the penalty rule of Eq.
// paramS: at a checked iteration l < iters the state pass sums
//   r^2 = sum (T x^l - t^l)^2 = sum (clip(v^l) - clip(v^(l-1)))^2,
//   (s / rho)^2 = sum (soft(v^l) - soft(v^(l-1)))^2
// per work-group (FP64 total on the device), k_xchange gives
// c = ||x^l - x^(l-1)|| / ||x^(l-1)|| (x^l is in d_x); stop with x^l when
// c < tol, else rho changes by tau when one residual exceeds mu times the
// other: the state is re-expressed for the new threshold and C_S^T (t - u')
// emitted for the inverse transform, Psi^+ and x_hat0 are rebuilt.
hipError_t gram(cip_plan_t p, hipStream_t st, double rho);

int solve_wdct_adaptive(cip_plan_t p, const float* d_y, const cip_adaptive_params* prm,
                        float* d_x, hipStream_t st, cip_solve_info& out) {
  const Layout& L = p->L;
  const int S = p->S, N1 = p->N1, N2 = p->N2, lv = p->wt_levels;
  const int iters = prm->max_iters, every = prm->every;
  const double rho0 = p->rho;
  double rho = rho0;
  float* coef = p->at<float>(L.wcoef);
  float* tmp = p->at<float>(L.wtmp);
  float* r = p->at<float>(L.rimg);
  float* v = p->at<float>(L.state);
  const float* cs = p->at<const float>(L.wband);
  const int groups = wavelet_state_groups(N1, N2);
  float* rs = p->at<float>(L.sums);
  float* xs = rs + 2 * (size_t)groups;
  double* tot = reinterpret_cast<double*>(xs + 2 * XCHANGE_GROUPS);
  float* xprev = p->at<float>(L.xbuf);
  const size_t nx = (size_t)S * N1 * N2;
  std::vector<float> hs(2 * XCHANGE_GROUPS + 4);
  auto xhat0 = [&]() -> hipError_t {
    // Alg. 1 step 2 with the current tables: x_hat0 = Psi^+ beta Lambda^H F y / (N1 N2)
    hipError_t e = row_r2c<float>(d_y, p->at<cx<float>>(L.bufA), p->K, N1, N2,
                                  p->at<const cx<float>>(L.twN2f), st);
    if (e != hipSuccess) return e;
    return col_op<float, OP_XHAT0>(p->at<const cx<float>>(L.bufA), p->at<void>(L.xh0), p->K, S,
                                   N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                   p->at<const cx<float>>(L.Mm), 0, st);
  };
  auto body = [&]() -> int {
    HIP_TRY(xhat0());
    for (int l = 1;; ++l) {
      if (l > 1)
        HIP_TRY(row_r2c<float>(r, p->at<cx<float>>(L.bufA), S, N1, N2,
                               p->at<const cx<float>>(L.twN2f), st));
      HIP_TRY(admm_col(p, l == 1 ? 1 : 0, 0, st));
      HIP_TRY(row_c2r(p->at<const cx<float>>(L.bufB), d_x, S, N1, N2, 1.0f,
                      p->at<const cx<float>>(L.twN2f), st));
      if (l == iters) {
        out.iters = l;
        break;
      }
      const bool check = l % every == 0;
      const bool store = (l + 1) % every == 0;
      const float kappa = (float)(p->lambda / rho);
      HIP_TRY(wavelet_forward(d_x, coef, tmp, S, N1, N2, lv, st));
      HIP_TRY(wavelet_state(coef, v, cs, S, N1, N2, kappa, l == 1 ? 1 : 0, st,
                            check ? rs : nullptr));
      if (check || store)
        HIP_TRY(launch(k_xchange, XCHANGE_GROUPS, 256, 0, st, (const float*)d_x, xprev, xs, nx,
                       check && l > 1 ? 1 : 0));
      if (check) {
        HIP_TRY(launch(k_sum_pairs, 1, 256, 0, st, (const float*)rs, (size_t)groups, tot));
        HIP_TRY(hipMemcpyAsync(hs.data(), xs, hs.size() * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double d2 = 0.0, p2 = 0.0, tt[2];
        for (int b = 0; b < XCHANGE_GROUPS; ++b) {
          d2 += hs[2 * b];
          p2 += hs[2 * b + 1];
        }
        std::memcpy(tt, hs.data() + 2 * XCHANGE_GROUPS, sizeof tt);
        const double rr = std::sqrt(tt[0]), sres = rho * std::sqrt(tt[1]);
        out.r_norm = rr;
        out.s_norm = sres;
        if (l > 1) {
          out.rel_change = p2 > 0.0 ? std::sqrt(d2 / p2) : 0.0;
          if (out.rel_change < prm->tol) {
            out.iters = l;   // x^l is in d_x
            break;
          }
        }
        double next = rho;
        if (rr > prm->mu * sres) next = prm->tau * rho;
        else if (sres > prm->mu * rr) next = rho / prm->tau;
        if (next != rho) {
          HIP_TRY(wavelet_emit(coef, v, cs, S, N1, N2, kappa, (float)(rho / next), st));
          HIP_TRY(gram(p, st, next));
          HIP_TRY(xhat0());
          rho = next;
          ++out.rho_changes;
        }
      }
      HIP_TRY(wavelet_inverse(coef, r, tmp, S, N1, N2, lv, st));
    }
    return CIP_OK;
  };
  int rc = body();
  out.rho = rho;
  if (rho != rho0) {   // leave the plan's tables at its own penalty
    hipError_t e = gram(p, st, rho0);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess && rc == CIP_OK)
      rc = fail(CIP_EHIP, std::string("restoring the tables: ") + hipGetErrorString(e));
  }
  return rc;
}

// Frequency pass of the conv prior (2D form, or the 3D form with its band
// DFTs).
hipError_t conv_freq_pass(cip_plan_t p, int first, int zero_g, int do_z, hipStream_t st) {
  const Layout& L = p->L;
  const size_t F = (size_t)p->N1 * p->H2;
  if (p->kind == CIP_PRIOR_CONV3D)
    return conv_freq3(p->at<cx<float>>(L.gv), p->at<cx<float>>(L.dhat), p->at<cx<float>>(L.xhat),
                      p->at<const cx<float>>(L.xh0), p->at<const float>(L.Adiag),
                      p->at<const cx<float>>(L.Aoff), p->at<const cx<float>>(L.th32),
                      p->at<const float>(L.gam), p->at<const cx<float>>(L.bw), p->n_filters, p->S,
                      F, first, zero_g, do_z, st);
  return conv_freq(p->at<cx<float>>(L.gv), p->at<cx<float>>(L.dhat), p->at<cx<float>>(L.xhat),
                   p->at<const cx<float>>(L.xh0), p->at<const float>(L.Adiag),
                   p->at<const cx<float>>(L.Aoff), p->at<const cx<float>>(L.th32),
                   p->at<const float>(L.gam), p->at<const float>(L.eta), p->n_filters, p->S, F,
                   first, zero_g, do_z, st);
}

// Online dictionary learning for the conv priors (see conv.hpp). Filter
// planes P = M S (3D) or M (2D, common filters); filter tables from g in
// FP32. Start of a solve: g = the plan's filters, e = 0, the spectra of
// g - e = g, and the tables from g.
hipError_t cdl_tables(cip_plan_t p, const cx<float>* gspec, double rho, hipStream_t st) {
  const Layout& L = p->L;
  const size_t F = (size_t)p->N1 * p->H2;
  if (p->kind == CIP_PRIOR_CONV3D)
    return conv_tables3f(gspec, p->at<cx<float>>(L.th32), p->at<float>(L.gam),
                         p->at<const cx<float>>(L.bw), p->n_filters, p->S, F, (float)rho, st);
  return conv_tables2f(p->at<const cx<float>>(L.th32), p->at<float>(L.gam), p->at<float>(L.eta),
                       p->n_filters, F, rho, p->mu, p->N1, p->N2, st);
}

hipError_t cdl_start(cip_plan_t p, hipStream_t st) {
  const Layout& L = p->L;
  const bool d3 = p->kind == CIP_PRIOR_CONV3D;
  const int M = p->n_filters, per = d3 ? p->S : 1, P = M * per, Lf = p->filt_l;
  const size_t F = (size_t)p->N1 * p->H2;
  hipError_t e = hipMemcpyAsync(p->at<void>(L.gtap), p->at<const void>(L.filt0),
                                (size_t)P * Lf * Lf * 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if ((e = cdl_fzero(p->at<cx<float>>(L.ecdl), (size_t)P * F, st)) != hipSuccess) return e;
  if ((e = cdl_place(p->at<const float>(L.gtap), p->at<float>(L.dpl), M, per, p->N1, p->N2, Lf,
                     st)) != hipSuccess)
    return e;
  if ((e = row_r2c<float>(p->at<const float>(L.dpl), p->at<cx<float>>(L.rtc), P, p->N1, p->N2,
                          p->at<const cx<float>>(L.twN2f), st)) != hipSuccess)
    return e;
  if ((e = conv_col_fft(1, p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.gehat), P, p->N1,
                        p->H2, p->at<const cx<float>>(L.twN1f), st)) != hipSuccess)
    return e;
  if (!d3 && (e = hipMemcpyAsync(p->at<void>(L.th32), p->at<const void>(L.gehat), (size_t)P * F * 8,
                                 hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  return cdl_tables(p, p->at<const cx<float>>(L.gehat), p->rho, st);
}

// One step of the dictionary ADMM after the code update of an outer
// iteration (gv holds the new codes' plane spectra, xhat those of x):
// d^ (3D: Sherman-Morrison per 3D frequency; 2D: Woodbury with an S x S
// Cholesky per frequency), returned as d^ + e^ (the dual is kept as plane
// spectra); d + e to space; g = projection of d + e; the spectra g^ of
// the placed g; e^ += d^ - g^ and the spectra of g - e; filter tables from
// g^; d^ = D(g) z for the next x-update. Two batched 2D FFTs of the filter
// planes per step.
// One D, G, E step with penalty sigma; the code tables for the next
// iterations from G at penalty rho. part (optional, a check of sigma): the
// partial sums of k_cdl_fdual_res, G_prev kept in L.gprev.
hipError_t cdl_step(cip_plan_t p, hipStream_t st, double sigma, double rho,
                    float* part = nullptr) {
  const Layout& L = p->L;
  const bool d3 = p->kind == CIP_PRIOR_CONV3D;
  const int M = p->n_filters, S = p->S, per = d3 ? S : 1, P = M * per, Lf = p->filt_l;
  const int N1 = p->N1, N2 = p->N2, H2 = p->H2;
  const size_t F = (size_t)N1 * H2;
  const cx<float>* bw = d3 ? p->at<const cx<float>>(L.bw) : nullptr;
  cx<float>* rtc = p->at<cx<float>>(L.rtc);
  cx<float>* dsp = p->at<cx<float>>(L.dsp);
  cx<float>* gehat = p->at<cx<float>>(L.gehat);
  cx<float>* ehat = p->at<cx<float>>(L.ecdl);
  float* dpl = p->at<float>(L.dpl);
  // dsp <- d^ + e^
  hipError_t e = d3 ? cdl_dfreq(p->at<const cx<float>>(L.xhat), p->at<const cx<float>>(L.gv),
                                gehat, ehat, dsp, bw, M, S, F, (float)sigma, st)
                    : cdl_dfreq2(p->at<const cx<float>>(L.xhat), p->at<const cx<float>>(L.gv),
                                 gehat, ehat, dsp, M, S, F, (float)sigma, st);
  if (e != hipSuccess) return e;
  const size_t ntaps = (size_t)P * Lf * Lf;
  if (part && (e = hipMemcpyAsync(p->at<void>(L.gprev), p->at<const void>(L.gtap), ntaps * 4,
                                  hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  // d + e in space
  if ((e = conv_col_fft(-1, dsp, rtc, P, N1, H2, p->at<const cx<float>>(L.twN1f), st)) != hipSuccess)
    return e;
  if ((e = row_c2r(rtc, dpl, P, N1, N2, (float)(1.0 / ((double)N1 * N2)),
                   p->at<const cx<float>>(L.twN2f), st)) != hipSuccess)
    return e;
  if ((e = cdl_project(dpl, nullptr, p->at<float>(L.gtap), M, per, N1, N2, Lf, st)) != hipSuccess)
    return e;
  // g^ of the placed taps, into gehat
  if ((e = cdl_place(p->at<const float>(L.gtap), dpl, M, per, N1, N2, Lf, st)) != hipSuccess)
    return e;
  if ((e = row_r2c<float>(dpl, rtc, P, N1, N2, p->at<const cx<float>>(L.twN2f), st)) != hipSuccess)
    return e;
  if ((e = conv_col_fft(1, rtc, gehat, P, N1, H2, p->at<const cx<float>>(L.twN1f), st)) != hipSuccess)
    return e;
  // 3D: g^ to dsp (d^ + e^ is read first), then the band DFT into the
  // tables; 2D: g^ are the tables
  cx<float>* gspec = d3 ? dsp : p->at<cx<float>>(L.th32);
  e = part ? cdl_fdual_res(ehat, gehat, dsp, gspec, (size_t)P * F, F, N1, N2,
                           p->at<const float>(L.gtap), p->at<const float>(L.gprev), ntaps, part,
                           st)
           : cdl_fdual(ehat, gehat, dsp, gspec, (size_t)P * F, st);
  if (e != hipSuccess) return e;
  if ((e = cdl_tables(p, gspec, rho, st)) != hipSuccess) return e;
  if (d3)
    return conv_dhat3(p->at<const cx<float>>(L.gv), p->at<const cx<float>>(L.th32),
                      p->at<cx<float>>(L.dhat), bw, M, S, F, st);
  return conv_dhat2(p->at<const cx<float>>(L.gv), p->at<const cx<float>>(L.th32),
                    p->at<cx<float>>(L.dhat), M, S, F, st);
}

// Algorithm 2 with the convolutional prior. Per iteration l = 1..L:
//   frequency pass: x^l = Psi^+ (b^ + d^{l-1}); for l < L also the
//   Sherman-Morrison code update v and d^l;
//   for l < L: inverse column FFT of v, row pass (inverse row FFT -> z^l,
//   state update, forward row FFT of t - u), forward column FFT -> g^.
// Finally x^L: inverse column and row FFTs of x^L.
hipError_t conv_iter(cip_plan_t p, int l, int last, hipStream_t st) {
  const Layout& L = p->L;
  const int P = p->n_filters * p->S;
  hipError_t e = conv_freq_pass(p, l == 1, l == 1, last ? 0 : 1, st);
  if (e != hipSuccess || last) return e;
  if (p->learn && (e = cdl_step(p, st, p->sigma, p->rho)) != hipSuccess) return e;
  e = conv_col_fft(-1, p->at<const cx<float>>(L.gv), p->at<cx<float>>(L.rtc), P, p->N1, p->H2,
                   p->at<const cx<float>>(L.twN1f), st);
  if (e != hipSuccess) return e;
  const float zscale = (float)(1.0 / ((double)p->N1 * p->N2));
  e = conv_row(p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.rtc), p->at<float>(L.vconv), P,
               p->N1, p->N2, p->at<const cx<float>>(L.twN2f), (float)(p->lambda / p->rho), zscale,
               l == 1, st);
  if (e != hipSuccess) return e;
  return conv_col_fft(1, p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.gv), P, p->N1, p->H2,
                      p->at<const cx<float>>(L.twN1f), st);
}

hipError_t solve_conv(cip_plan_t p, int iters, float* d_x, hipStream_t st) {
  const Layout& L = p->L;
  hipError_t e;
  if (p->learn && (e = cdl_start(p, st)) != hipSuccess) return e;
  for (int l = 1; l <= iters; ++l)
    if ((e = conv_iter(p, l, l == iters, st)) != hipSuccess) return e;
  e = conv_col_fft(-1, p->at<const cx<float>>(L.xhat), p->at<cx<float>>(L.bufB), p->S, p->N1, p->H2,
                   p->at<const cx<float>>(L.twN1f), st);
  if (e != hipSuccess) return e;
  return row_c2r(p->at<const cx<float>>(L.bufB), d_x, p->S, p->N1, p->N2,
                 (float)(1.0 / ((double)p->N1 * p->N2)), p->at<const cx<float>>(L.twN2f), st);
}

// Algorithm 2 with a convolutional dictionary and the penalty update and
// stopping rule of Section IV-C (Eq. paramS), split z = t: at every `every`-th
// iteration l < max_iters,
//   r = ||z^l - t^l||, s = rho ||t^l - t^(l-1)|| (summed by the row pass),
//   c = ||x^l - x^(l-1)|| / ||x^(l-1)|| (x^l formed in d_x, k_xchange);
// stop with x^l when c < tol, else change rho by tau when one residual
// exceeds mu times the other. Only the z-update depends on rho: on a change
// the state is re-expressed for the new penalty (u scaled by rho / rho'),
// g^ = F(t - u') is formed again, and gamma, eta (and theta) are rebuilt:
// in FP64 from the resident filter spectra for a fixed dictionary (the
// plan's tables are back at its own rho on return), in FP32 from the
// spectra of G with online dictionary learning. With learning and
// adapt_sigma the D, G, E step of a checked iteration also yields
//   r_d = ||D - G|| (Parseval over the spectra of the dual's change),
//   s_d = sigma ||G - G_prev|| (over the filter taps),
// and sigma changes by the same rule, the scaled dual E rescaled by
// sigma / sigma'.
int solve_conv_adaptive(cip_plan_t p, const cip_adaptive_params* prm, float* d_x, hipStream_t st,
                        cip_solve_info& out) {
  const Layout& L = p->L;
  const int iters = prm->max_iters, every = prm->every;
  const bool d3 = p->kind == CIP_PRIOR_CONV3D;
  const int M = p->n_filters, P = M * p->S, Pf = M * (d3 ? p->S : 1);
  const size_t F = (size_t)p->N1 * p->H2;
  const double rho0 = p->rho;
  double rho = rho0, sigma = p->sigma;
  const size_t nres = conv_row_residual_floats(P, p->N1, p->N2);
  float* rs = p->at<float>(L.sums);
  float* xs = rs + nres;
  double* tot = reinterpret_cast<double*>(xs + 2 * XCHANGE_GROUPS);
  float* dpart = xs + 2 * XCHANGE_GROUPS + 4;
  double* dtot = reinterpret_cast<double*>(dpart + 2 * CDL_RES_GROUPS);
  float* xprev = p->at<float>(L.xbuf);
  const size_t nx = (size_t)p->S * p->N1 * p->N2;
  const size_t ncode = (size_t)P * p->N1 * p->N2;
  const double nn = (double)p->N1 * p->N2;
  const float zscale = (float)(1.0 / nn);
  // xs .. dtot + 2: k_xchange sums, the totals, the dictionary partials and totals
  std::vector<float> hs(2 * XCHANGE_GROUPS + 4 + 2 * CDL_RES_GROUPS + 4);
  // the spectra of G (the tables' source with learning): the tables
  // themselves for 2D, the last D, G, E step's g^ for 3D
  cx<float>* gspec = d3 ? p->at<cx<float>>(L.dsp) : p->at<cx<float>>(L.th32);
  auto set_tables = [&](double r) -> hipError_t {
    if (p->learn) return cdl_tables(p, gspec, r, st);
    if (d3)
      return conv_tables3(p->at<const cx<double>>(L.th64), p->at<cx<float>>(L.th32),
                          p->at<float>(L.gam), M, p->S, F, r, st);
    return conv_tables(p->at<const cx<double>>(L.th64), p->at<cx<float>>(L.th32),
                       p->at<float>(L.gam), p->at<float>(L.eta), M, F, r, p->mu, p->N1, p->N2,
                       st);
  };
  auto x_out = [&]() -> hipError_t {   // x^l = F^-1 x^ -> d_x
    hipError_t e = conv_col_fft(-1, p->at<const cx<float>>(L.xhat), p->at<cx<float>>(L.bufB),
                                p->S, p->N1, p->H2, p->at<const cx<float>>(L.twN1f), st);
    if (e != hipSuccess) return e;
    return row_c2r(p->at<const cx<float>>(L.bufB), d_x, p->S, p->N1, p->N2, zscale,
                   p->at<const cx<float>>(L.twN2f), st);
  };
  int rc = CIP_OK;
  if (p->learn) HIP_TRY(cdl_start(p, st));
  for (int l = 1;; ++l) {
    const bool last = l == iters;
    HIP_TRY(conv_freq_pass(p, l == 1, l == 1, last ? 0 : 1, st));
    if (last) {
      HIP_TRY(x_out());
      out.iters = l;
      break;
    }
    const bool check = l % every == 0;
    const bool store = (l + 1) % every == 0;
    const bool check_sigma = check && p->learn && prm->adapt_sigma;
    const float kappa = (float)(p->lambda / rho);
    if (p->learn) HIP_TRY(cdl_step(p, st, sigma, rho, check_sigma ? dpart : nullptr));
    HIP_TRY(conv_col_fft(-1, p->at<const cx<float>>(L.gv), p->at<cx<float>>(L.rtc), P, p->N1,
                         p->H2, p->at<const cx<float>>(L.twN1f), st));
    HIP_TRY(conv_row(p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.rtc), p->at<float>(L.vconv),
                     P, p->N1, p->N2, p->at<const cx<float>>(L.twN2f), kappa, zscale, l == 1, st,
                     check ? rs : nullptr));
    HIP_TRY(conv_col_fft(1, p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.gv), P, p->N1,
                         p->H2, p->at<const cx<float>>(L.twN1f), st));
    if (check || store) {
      HIP_TRY(x_out());
      HIP_TRY(launch(k_xchange, XCHANGE_GROUPS, 256, 0, st, (const float*)d_x, xprev, xs, nx,
                     check && l > 1 ? 1 : 0));
    }
    if (!check) continue;
    HIP_TRY(launch(k_sum_pairs, 1, 256, 0, st, (const float*)rs, nres / 2, tot));
    if (check_sigma)
      HIP_TRY(launch(k_sum_pairs, 1, 256, 0, st, (const float*)dpart, (size_t)CDL_RES_GROUPS,
                     dtot));
    HIP_TRY(hipMemcpyAsync(hs.data(), xs, hs.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double d2 = 0.0, p2 = 0.0, tt[2], td[2];
    for (int b = 0; b < XCHANGE_GROUPS; ++b) {
      d2 += hs[2 * b];
      p2 += hs[2 * b + 1];
    }
    std::memcpy(tt, hs.data() + 2 * XCHANGE_GROUPS, sizeof tt);
    std::memcpy(td, hs.data() + 2 * XCHANGE_GROUPS + 4 + 2 * CDL_RES_GROUPS, sizeof td);
    const double r = std::sqrt(tt[0]), sres = rho * std::sqrt(tt[1]);
    out.r_norm = r;
    out.s_norm = sres;
    if (l > 1) {
      out.rel_change = p2 > 0.0 ? std::sqrt(d2 / p2) : 0.0;
      if (out.rel_change < prm->tol) {
        out.iters = l;   // x^l is in d_x
        break;
      }
    }
    double next = rho;
    if (r > prm->mu * sres) next = prm->tau * rho;
    else if (sres > prm->mu * r) next = rho / prm->tau;
    if (next != rho) {
      // V -> V', W = t - u' (in the memory of g^, which is formed again)
      float* w = p->at<float>(L.gv);
      HIP_TRY(conv_reemit(p->at<float>(L.vconv), w, ncode, kappa, (float)(p->lambda / next),
                          (float)(rho / next), st));
      HIP_TRY(row_r2c<float>(w, p->at<cx<float>>(L.rtc), P, p->N1, p->N2,
                             p->at<const cx<float>>(L.twN2f), st));
      HIP_TRY(conv_col_fft(1, p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.gv), P, p->N1,
                           p->H2, p->at<const cx<float>>(L.twN1f), st));
      HIP_TRY(set_tables(next));
      rho = next;
      ++out.rho_changes;
    }
    if (check_sigma) {
      const double rd = std::sqrt(td[0] / nn), sd = sigma * std::sqrt(td[1]);
      double ns = sigma;
      if (rd > prm->mu * sd) ns = prm->tau * sigma;
      else if (sd > prm->mu * rd) ns = sigma / prm->tau;
      if (ns != sigma) {
        HIP_TRY(cdl_rescale_dual(p->at<cx<float>>(L.ecdl), p->at<cx<float>>(L.gehat), gspec,
                                 (size_t)Pf * F, (float)(sigma / ns), st));
        sigma = ns;
        ++out.sigma_changes;
      }
    }
  }
  out.rho = rho;
  out.sigma = p->learn ? sigma : 0.0;
  if (rho != rho0 && !p->learn) {   // leave the plan's tables at its own penalty
    const hipError_t e = set_tables(rho0);
    if (e != hipSuccess && rc == CIP_OK) rc = fail(CIP_EHIP, hipGetErrorString(e));
  }
  return rc;
}

hipError_t gram(cip_plan_t p, hipStream_t st, double rho = 0.0) {
  if (rho <= 0.0) rho = p->rho;
  GramArgs a;
  a.K = p->K;
  a.N1 = p->N1;
  a.N2 = p->N2;
  a.H2 = p->H2;
  a.beta = p->beta;
  a.scale = 1.0 / ((double)p->N1 * (double)p->N2);
  a.rcond = 1e-12;
  const bool patch = p->kind == CIP_PRIOR_PATCH,
             conv = p->kind == CIP_PRIOR_CONV2D || p->kind == CIP_PRIOR_CONV3D;
  // analysis: Psi = rho tau I + beta L^H L, rhs = b + rho g;
  // patch synthesis: Psi = c_P I + beta L^H L with c_P = (Q / st)^2 = 4, rhs = b + g;
  // conv synthesis: c_P = 1, and the tables are unnormalised (the frequency
  // pass works with unnormalised spectra throughout)
  a.wgt = patch ? 4.0 : (conv ? 1.0 : rho);
  a.coefA = (patch || conv) ? 1.0 : rho;
  if (conv) a.scale = 1.0;
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

// Stage twiddle table of a length-N group FFT with PPT points per thread,
// in the order the device stages read it (see fft_shape): for every stage
// after the first, [k < Ns][r = 1 .. RS-1] -> W_{Ns RS}^{r k}, computed in
// double precision. Padded with zeros to N entries.
// Stage-ordered twiddle table of fft_group (same radix sequence as
// fft_shape: PPT first, then greedy divisors of PPT).
void stage_twiddles(int N, int PPT, std::vector<cx<double>>& d) {
  d.assign(N, cx<double>{0.0, 0.0});
  int off = 0, ns = PPT, rem = N / PPT;
  while (rem > 1) {
    const int rs = next_radix(rem, PPT);
    for (int k = 0; k < ns; ++k)
      for (int r = 1; r < rs; ++r) {
        double a = 2.0 * M_PI * (double)r * (double)k / ((double)ns * rs);
        d[off + k * (rs - 1) + r - 1] = cx<double>{std::cos(a), -std::sin(a)};
      }
    off += ns * (rs - 1);
    ns *= rs;
    rem /= rs;
  }
}

void twiddles(int N, int PPT, std::vector<cx<float>>& f, std::vector<cx<double>>& d) {
  stage_twiddles(N, PPT, d);
  f.resize(N);
  for (int m = 0; m < N; ++m) f[m] = cx<float>{(float)d[m].x, (float)d[m].y};
}

void dct_table(int N, std::vector<cx<float>>& ew) {
  ew.resize(N);
  for (int k = 0; k < N; ++k) {
    double a = M_PI * (double)k / (2.0 * N);
    ew[k] = cx<float>{(float)std::cos(a), (float)(-std::sin(a))};
  }
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Patch dictionary tables: D (nv x na, row-major) and
// M1 = D^T (rho I + D D^T)^-1 (na x nv), formed in double precision with a
// Cholesky factorisation of the nv x nv matrix rho I + D D^T, both rounded to
// BF16 for the MFMA operands.
void patch_dictionary_tables(const std::vector<float>& D, int nv, int na, double rho,
                             std::vector<uint16_t>& dbf, std::vector<uint16_t>& m1bf) {
  std::vector<double> G((size_t)nv * nv, 0.0);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j <= i; ++j) {
      double acc = 0.0;
      for (int a = 0; a < na; ++a) acc += (double)D[(size_t)i * na + a] * D[(size_t)j * na + a];
      G[(size_t)i * nv + j] = G[(size_t)j * nv + i] = acc + (i == j ? rho : 0.0);
    }
  for (int j = 0; j < nv; ++j) {   // in-place Cholesky, lower triangle
    double d = G[(size_t)j * nv + j];
    for (int k = 0; k < j; ++k) d -= G[(size_t)j * nv + k] * G[(size_t)j * nv + k];
    d = std::sqrt(d);
    G[(size_t)j * nv + j] = d;
    for (int i = j + 1; i < nv; ++i) {
      double v = G[(size_t)i * nv + j];
      for (int k = 0; k < j; ++k) v -= G[(size_t)i * nv + k] * G[(size_t)j * nv + k];
      G[(size_t)i * nv + j] = v / d;
    }
  }
  // X = (rho I + D D^T)^-1 D  (nv x na); M1 = X^T
  std::vector<double> X((size_t)nv * na);
  for (int a = 0; a < na; ++a) {
    std::vector<double> y(nv);
    for (int i = 0; i < nv; ++i) {
      double v = D[(size_t)i * na + a];
      for (int k = 0; k < i; ++k) v -= G[(size_t)i * nv + k] * y[k];
      y[i] = v / G[(size_t)i * nv + i];
    }
    for (int i = nv - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nv; ++k) v -= G[(size_t)k * nv + i] * X[(size_t)k * na + a];
      X[(size_t)i * na + a] = v / G[(size_t)i * nv + i];
    }
  }
  dbf.resize((size_t)nv * na);
  m1bf.resize((size_t)na * nv);
  for (size_t i = 0; i < dbf.size(); ++i) dbf[i] = bf16_rne(D[i]);
  for (int a = 0; a < na; ++a)
    for (int i = 0; i < nv; ++i) m1bf[(size_t)a * nv + i] = bf16_rne((float)X[(size_t)i * na + a]);
}

}  // namespace

// ---------------------------------------------------------------- C ABI
namespace {

// Iterations 2 .. iters of Algorithm 1 (row pass, column pass), all on the
// plan's own buffers.
hipError_t loop_kernels(cip_plan_t p, int iters, hipStream_t st) {
  for (int l = 1; l < iters; ++l) {
    hipError_t e = admm_row(p, l, st);
    if (e != hipSuccess) return e;
    e = admm_col(p, 0, l < iters - 1 ? 1 : 0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The loop launched directly, or, from the second solve in a row with the
// same iteration count, replayed from a hipGraph captured once (the loop's
// kernels read and write only plan buffers, so the graph stays valid for
// every later solve with that count). A stream that is itself being
// captured (a batch graph) gets the kernels directly.
int analysis_loop(cip_plan_t p, int iters, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs));
  const bool repeat = p->last_iters == iters;
  p->last_iters = iters;
  if (cs != hipStreamCaptureStatusNone || !repeat) {
    HIP_TRY(loop_kernels(p, iters, st));
    return CIP_OK;
  }
  if (p->loop_iters != iters) {
    p->drop_loop_graph();
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    hipError_t e2 = e == hipSuccess ? loop_kernels(p, iters, cap) : hipSuccess;
    hipGraph_t g = nullptr;
    hipError_t e3 = e == hipSuccess ? hipStreamEndCapture(cap, &g) : hipSuccess;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      HIP_TRY(loop_kernels(p, iters, st));   // fall back to direct launches
      return CIP_OK;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      HIP_TRY(loop_kernels(p, iters, st));
      return CIP_OK;
    }
    p->loop_graph = g;
    p->loop_exec = x;
    p->loop_iters = iters;
  }
  HIP_TRY(hipGraphLaunch(p->loop_exec, st));
  return CIP_OK;
}

}  // namespace

extern "C" {

const char* cip_last_error(void) { return g_last_error.c_str(); }

int cip_plan_workspace_bytes(int K, int S, int N1, int N2, const cip_prior_desc* prior,
                             size_t* bytes) {
  int rc = validate(K, S, N1, N2, prior);
  if (rc) return rc;
  if (!bytes) return fail(CIP_EINVAL, "bytes is NULL");
  *bytes = make_layout(K, S, N1, N2, prior).total;
  return CIP_OK;
}

int cip_plan_create(int K, int S, int N1, int N2, const float* d_psf, const cip_prior_desc* prior,
                    double rho, double lambda, void* d_workspace, size_t ws_bytes, void* stream,
                    cip_plan_t* out) {
  int rc = validate(K, S, N1, N2, prior);
  if (rc) return rc;
  if (!d_psf || !d_workspace || !out) return fail(CIP_EINVAL, "NULL pointer argument");
  if (!(rho > 0.0) || !(lambda >= 0.0)) return fail(CIP_EINVAL, "need rho > 0 and lambda >= 0");
  if ((prior->kind == CIP_PRIOR_ITV2D || prior->kind == CIP_PRIOR_ITV3D) && !(lambda > 0.0))
    return fail(CIP_EINVAL, "isotropic TV: lambda must be > 0");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(CIP_EINVAL, "workspace must be 256-byte aligned");
  if (prior->kind == CIP_PRIOR_PATCH && !prior->dict)
    return fail(CIP_EINVAL, "patch prior needs a dictionary");
  if ((prior->kind == CIP_PRIOR_CONV2D || prior->kind == CIP_PRIOR_CONV3D) && !prior->filters)
    return fail(CIP_EINVAL, "conv prior needs filters");
  Layout L = make_layout(K, S, N1, N2, prior);
  if (ws_bytes < L.total) return fail(CIP_ENOSPC, "workspace too small");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  cip_plan_s* p = new cip_plan_s();
  p->K = K;
  p->S = S;
  p->N1 = N1;
  p->N2 = N2;
  p->H2 = N2 / 2 + 1;
  p->kind = prior->kind;
  p->n_atoms = prior->kind == CIP_PRIOR_PATCH ? prior->n_atoms : 0;
  p->n_filters =
      (prior->kind == CIP_PRIOR_CONV2D || prior->kind == CIP_PRIOR_CONV3D) ? prior->n_filters : 0;
  p->beta = prior->beta;
  p->rho = rho;
  p->lambda = lambda;
  p->ws = reinterpret_cast<unsigned char*>(d_workspace);
  p->sws = p->ws + L.tables;
  p->L = L;
  p->solved_once = false;
  p->attached = false;
  p->adaptive = (prior->flags & CIP_PLAN_ADAPTIVE) != 0;
  p->learn = (prior->kind == CIP_PRIOR_CONV3D || prior->kind == CIP_PRIOR_CONV2D ||
              prior->kind == CIP_PRIOR_PATCH) &&
             (prior->flags & CIP_PLAN_DICT_UPDATE) != 0;
  p->mu = prior->mu;
  // default sigma: the paper's settings (1 for the patch dictionary, 10 for
  // the convolutional one)
  p->sigma = prior->sigma > 0.0 ? prior->sigma : (prior->kind == CIP_PRIOR_PATCH ? 1.0 : 10.0);
  p->filt_l = prior->filt_l;
  p->row_np = PAIRS;
  p->row_ppt = ppt_row_n(N2);
  p->tv_inner = (prior->kind == CIP_PRIOR_ITV2D || prior->kind == CIP_PRIOR_ITV3D)
                    ? (prior->tv_inner > 0 ? prior->tv_inner : 20)
                    : 0;
  p->wt_levels =
      prior->kind == CIP_PRIOR_WDCT3D ? (prior->wt_levels > 0 ? prior->wt_levels : 3) : 0;

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

  std::vector<cx<float>> t1f, t2f, fw;
  std::vector<cx<double>> t1d, t2d;
  twiddles(N1, ppt_col_n(N1), t1f, t1d);   // column transforms (length N1)
  twiddles(N2, ppt_row_n(N2), t2f, t2d);   // row transforms (length N2)
  if (L.twN2f8) {
    std::vector<cx<float>> t8f;
    std::vector<cx<double>> t8d;
    twiddles(N2, 8, t8f, t8d);
    PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN2f8), t8f.data(), N2 * 8, hipMemcpyHostToDevice, st));
    PLAN_HIP(hipStreamSynchronize(st));
  }
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN1f), t1f.data(), N1 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN2f), t2f.data(), N2 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN1d), t1d.data(), N1 * 16, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.twN2d), t2d.data(), N2 * 16, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipStreamSynchronize(st));
  if (L.band || L.wband) {   // orthonormal DCT-II along the bands, C[k][s] = a_k cos(pi (2s+1) k / 2S)
    std::vector<float> cs((size_t)S * S);
    for (int k = 0; k < S; ++k)
      for (int j = 0; j < S; ++j)
        cs[(size_t)k * S + j] = (float)((k == 0 ? std::sqrt(1.0 / S) : std::sqrt(2.0 / S)) *
                                        std::cos(M_PI * (2.0 * j + 1.0) * k / (2.0 * S)));
    PLAN_HIP(hipMemcpyAsync(p->at<void>(L.band ? L.band : L.wband), cs.data(), cs.size() * 4,
                            hipMemcpyHostToDevice, st));
    PLAN_HIP(hipStreamSynchronize(st));
  }
  dct_table(N1, fw);
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.ew1), fw.data(), N1 * 8, hipMemcpyHostToDevice, st));
  PLAN_HIP(hipStreamSynchronize(st));
  dct_table(N2, fw);
  PLAN_HIP(hipMemcpyAsync(p->at<void>(L.ew2), fw.data(), N2 * 8, hipMemcpyHostToDevice, st));
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
  if (p->kind == CIP_PRIOR_CONV2D && !p->learn) {
    // filter spectra theta_m in FP64 (same transform path as the kernels)
    const int M = prior->n_filters, Lf = prior->filt_l;
    double* d_pl = p->at<double>(L.pl64);
    for (int m = 0; m < M; ++m) {
      PLAN_HIP(conv_place_filter(prior->filters + (size_t)m * Lf * Lf, d_pl, Lf, N1, N2, st));
      PLAN_HIP(row_r2c<double>(d_pl, p->at<cx<double>>(L.rt64), 1, N1, N2,
                               p->at<const cx<double>>(L.twN2d), st));
      PLAN_HIP((col_op<double, OP_SPEC>(p->at<const cx<double>>(L.rt64), p->at<void>(L.th64), 1, 1,
                                        N1, p->H2, p->at<const cx<double>>(L.twN1d), nullptr, m,
                                        st)));
    }
    PLAN_HIP(conv_tables(p->at<const cx<double>>(L.th64), p->at<cx<float>>(L.th32),
                         p->at<float>(L.gam), p->at<float>(L.eta), M, (size_t)N1 * p->H2, rho,
                         prior->mu, N1, N2, st));
  }
  if (p->kind == CIP_PRIOR_CONV3D) {
    // band DFT matrix bw[k][s] = exp(-2 pi i k s / S), formed in FP64
    std::vector<cx<float>> bw((size_t)S * S);
    for (int k = 0; k < S; ++k)
      for (int s2 = 0; s2 < S; ++s2) {
        const double a = -2.0 * kPi * (double)((k * s2) % S) / (double)S;
        bw[(size_t)k * S + s2] = cx<float>{(float)std::cos(a), (float)std::sin(a)};
      }
    PLAN_HIP(hipMemcpyAsync(p->at<void>(L.bw), bw.data(), bw.size() * sizeof(cx<float>),
                            hipMemcpyHostToDevice, st));
    PLAN_HIP(hipStreamSynchronize(st));   // bw is a host temporary
  }
  if (p->learn) {
    // the tables are formed from these filters at the start of every solve
    const size_t planes = (size_t)prior->n_filters * (p->kind == CIP_PRIOR_CONV3D ? S : 1);
    PLAN_HIP(hipMemcpyAsync(p->at<void>(L.filt0), prior->filters,
                            planes * prior->filt_l * prior->filt_l * 4, hipMemcpyDeviceToDevice,
                            st));
  }
  if (p->kind == CIP_PRIOR_CONV3D && !p->learn) {
    // 2D spectra of every filter slice (m, s') in FP64 -> band DFT -> theta_m(w, k)
    const int M = prior->n_filters, Lf = prior->filt_l;
    double* d_pl = p->at<double>(L.pl64);
    for (int m = 0; m < M; ++m) {
      for (int sp = 0; sp < S; ++sp) {
        PLAN_HIP(conv_place_filter(prior->filters + ((size_t)m * S + sp) * Lf * Lf, d_pl, Lf, N1,
                                   N2, st));
        PLAN_HIP(row_r2c<double>(d_pl, p->at<cx<double>>(L.rt64), 1, N1, N2,
                                 p->at<const cx<double>>(L.twN2d), st));
        PLAN_HIP((col_op<double, OP_SPEC>(p->at<const cx<double>>(L.rt64), p->at<void>(L.th64), 1,
                                          1, N1, p->H2, p->at<const cx<double>>(L.twN1d), nullptr,
                                          m * S + sp, st)));
      }
    }
    PLAN_HIP(conv_tables3(p->at<const cx<double>>(L.th64), p->at<cx<float>>(L.th32),
                          p->at<float>(L.gam), M, S, (size_t)N1 * p->H2, rho, st));
    PLAN_HIP(hipStreamSynchronize(st));
  }
  if (p->kind == CIP_PRIOR_PATCH) {
    // M1 = D^T (rho I + D D^T)^-1 in FP64 on the host; D and M1 stored as BF16
    const int nv = 64 * S, na = prior->n_atoms;
    std::vector<float> D((size_t)nv * na);
    PLAN_HIP(hipMemcpyAsync(D.data(), prior->dict, D.size() * 4, hipMemcpyDeviceToHost, st));
    PLAN_HIP(hipStreamSynchronize(st));
    std::vector<uint16_t> dbf, m1bf;
    patch_dictionary_tables(D, nv, na, rho, dbf, m1bf);
    PLAN_HIP(hipMemcpyAsync(p->at<void>(p->learn ? L.dbf0 : L.dbf), dbf.data(), dbf.size() * 2,
                            hipMemcpyHostToDevice, st));
    PLAN_HIP(hipMemcpyAsync(p->at<void>(p->learn ? L.m1bf0 : L.m1bf), m1bf.data(),
                            m1bf.size() * 2, hipMemcpyHostToDevice, st));
    if (p->learn)
      PLAN_HIP(hipMemcpyAsync(p->at<void>(L.pd0), D.data(), D.size() * 4, hipMemcpyHostToDevice,
                              st));
    PLAN_HIP(hipStreamSynchronize(st));
    if (p->adaptive) p->dict_host = std::move(D);
  }
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
  if (p->kind == CIP_PRIOR_PATCH || p->kind == CIP_PRIOR_CONV2D || p->kind == CIP_PRIOR_CONV3D ||
      p->kind == CIP_PRIOR_WDCT3D) {
    if (p->kind == CIP_PRIOR_PATCH) HIP_TRY(solve_patch(p, iters, d_x, st));
    else if (p->kind == CIP_PRIOR_WDCT3D) HIP_TRY(solve_wdct(p, iters, d_x, st));
    else HIP_TRY(solve_conv(p, iters, d_x, st));
    p->solved_once = true;
    return CIP_OK;
  }
  // iteration 1 (t = u = 0): column pass only
  HIP_TRY(admm_col(p, 1, iters > 1 ? 1 : 0, st));
  if (iters > 1) {
    int rc = analysis_loop(p, iters, st);
    if (rc) return rc;
  }
  HIP_TRY(admm_row_dct(p, ROW_FINAL, st, d_x));
  p->solved_once = true;
  return CIP_OK;
}

int cip_plan_dictionary(cip_plan_t p, float* d_filters, void* stream) {
  if (!p || !d_filters) return fail(CIP_EINVAL, "NULL argument");
  if (!p->learn) return fail(CIP_EINVAL, "the plan does not learn its dictionary");
  if (!p->solved_once) return fail(CIP_EINVAL, "run cip_solve on this plan first");
  if (p->kind == CIP_PRIOR_PATCH) {
    HIP_TRY(hipMemcpyAsync(d_filters, p->at<const void>(p->L.pg),
                           (size_t)64 * p->S * p->n_atoms * 4, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    return CIP_OK;
  }
  const size_t planes = (size_t)p->n_filters * (p->kind == CIP_PRIOR_CONV3D ? p->S : 1);
  const size_t bytes = planes * p->filt_l * p->filt_l * 4;
  HIP_TRY(hipMemcpyAsync(d_filters, p->at<const void>(p->L.gtap), bytes, hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(stream)));
  return CIP_OK;
}

int cip_plan_destroy(cip_plan_t p) {
  delete p;
  return CIP_OK;
}

// Algorithm 1 with an isotropic TV prior and the penalty rule of Eq. paramS
// (T = I). At a checked iteration l < iters, after the t-update:
//   r = ||x^l - t^l||,  s = rho ||t^l - t^(l-1)||,  stop on the iterate change,
//   else rho <- tau rho if r > mu s, rho / tau if s > mu r;
// on a change the closing row pass runs again with c = rho / rho' (the scaled
// dual rescaled, the spectrum of t - u' re-emitted), Psi^+ and x_hat0 are
// rebuilt, and Chambolle's dual stays as the next warm start. x^l comes from
// the prep pass (kept at the checks and the iterations before them), t^(l-1)
// from the norm pass of the iteration before a check.
int solve_itv_adaptive(cip_plan_t p, const float* d_y, const cip_adaptive_params* prm,
                       float* d_x, hipStream_t st, cip_solve_info& out) {
  const Layout& L = p->L;
  const int iters = prm->max_iters, every = prm->every;
  const double rho0 = p->rho;
  double rho = rho0;
  const size_t n = (size_t)p->S * p->N1 * p->N2;
  float* xb0 = p->at<float>(L.xbuf);
  float* xb1 = xb0 + n;
  auto xbuf = [&](int l) { return (l & 1) ? xb1 : xb0; };
  float* tprev = p->at<float>(L.tprev);
  const ItvState sv = itv_state(p);
  const int groups = p->S * (p->N1 / RT);
  std::vector<float> sums((size_t)groups * 4);
  auto xhat0 = [&]() -> hipError_t {
    // Alg. 1 step 2 with the current tables: x_hat0 = Psi^+ beta Lambda^H F y / (N1 N2)
    hipError_t e = row_r2c<float>(d_y, p->at<cx<float>>(L.bufB), p->K, p->N1, p->N2,
                                  p->at<const cx<float>>(L.twN2f), st);
    if (e != hipSuccess) return e;
    return col_op<float, OP_XHAT0>(p->at<const cx<float>>(L.bufB), p->at<void>(L.xh0), p->K, p->S,
                                   p->N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                   p->at<const cx<float>>(L.Mm), 0, st);
  };
  auto body = [&]() -> int {
    HIP_TRY(xhat0());
    HIP_TRY(admm_col(p, 1, 0, st));   // x^1 (t = u = 0)
    for (int l = 1;; ++l) {
      if (l == iters) {   // the last iterate is returned without a check
        out.iters = l;
        HIP_TRY(admm_row_dct(p, ROW_FINAL, st, d_x));
        break;
      }
      const bool check = l % every == 0;
      const bool store = (l + 1) % every == 0;   // keep x^l and t^l for the next check
      float* xo = (check || store) ? xbuf(l) : nullptr;
      HIP_TRY(itv_row(p, l, st, rho, xo));
      double next = rho;
      bool stop = false;
      if (check || store) {
        HIP_TRY(launch(k_itv_norm, groups, 256, 0, st, sv.f, sv.u, xo, tprev,
                       check && l > 1 ? xbuf(l - 1) : nullptr, RT * p->N2, l == 1 ? 1 : 0,
                       store ? 1 : 0, p->at<float>(L.sums)));
        if (check) {
          HIP_TRY(hipMemcpyAsync(sums.data(), p->at<float>(L.sums), sums.size() * 4,
                                 hipMemcpyDeviceToHost, st));
          HIP_TRY(hipStreamSynchronize(st));
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          for (int b = 0; b < groups; ++b)
            for (int i = 0; i < 4; ++i) acc[i] += (double)sums[(size_t)b * 4 + i];
          const double r = std::sqrt(acc[0]), sres = rho * std::sqrt(acc[1]);
          out.r_norm = r;
          out.s_norm = sres;
          if (l > 1) {
            out.rel_change = acc[3] > 0.0 ? std::sqrt(acc[2] / acc[3]) : 0.0;
            stop = out.rel_change < prm->tol;
          }
          if (!stop) {
            if (r > prm->mu * sres) next = prm->tau * rho;
            else if (sres > prm->mu * r) next = rho / prm->tau;
          }
        }
      }
      if (stop) {   // x^l: its spectrum is still the column-pass output
        out.iters = l;
        HIP_TRY(admm_row_dct(p, ROW_FINAL, st, d_x));
        break;
      }
      if (next != rho) {
        HIP_TRY(itv_finish(p, l, (float)(p->lambda / rho), (float)(rho / next), st));
        HIP_TRY(gram(p, st, next));
        HIP_TRY(xhat0());
        rho = next;
        ++out.rho_changes;
      }
      HIP_TRY(admm_col(p, 0, 0, st));
    }
    return CIP_OK;
  };
  int rc = body();
  out.rho = rho;
  if (rho != rho0) {   // leave the plan's tables at its own penalty
    hipError_t e = gram(p, st, rho0);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess && rc == CIP_OK)
      rc = fail(CIP_EHIP, std::string("restoring the tables: ") + hipGetErrorString(e));
  }
  return rc;
}

int cip_solve_adaptive(cip_plan_t p, const float* d_y, const cip_adaptive_params* prm, float* d_x,
                       void* stream, cip_solve_info* info) {
  if (!p || !d_y || !d_x || !prm) return fail(CIP_EINVAL, "NULL argument");
  if (!p->adaptive) return fail(CIP_EINVAL, "plan was not created with CIP_PLAN_ADAPTIVE");
  if (p->attached) return fail(CIP_EINVAL, "an adaptive solve rewrites the tables: not on an attached plan");
  const bool synthesis = p->kind == CIP_PRIOR_PATCH || p->kind == CIP_PRIOR_CONV2D ||
                         p->kind == CIP_PRIOR_CONV3D;
  if (prm->adapt_sigma && !p->learn)
    return fail(CIP_EUNSUPPORTED, "adapt_sigma: the plan does not learn its dictionary");
  if (prm->max_iters < 1 || prm->every < 1 || !(prm->tau > 1.0) || !(prm->mu > 1.0) ||
      !(prm->tol >= 0.0))
    return fail(CIP_EINVAL, "need max_iters >= 1, every >= 1, tau > 1, mu > 1, tol >= 0");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (synthesis) {
    // Alg. 2 step 2: x_hat0 = Psi^-1 beta Lambda^H F y / (N1 N2)
    HIP_TRY(row_r2c<float>(d_y, p->at<cx<float>>(p->L.bufA), p->K, p->N1, p->N2,
                           p->at<const cx<float>>(p->L.twN2f), st));
    HIP_TRY((col_op<float, OP_XHAT0>(p->at<const cx<float>>(p->L.bufA), p->at<void>(p->L.xh0),
                                     p->K, p->S, p->N1, p->H2,
                                     p->at<const cx<float>>(p->L.twN1f),
                                     p->at<const cx<float>>(p->L.Mm), 0, st)));
    cip_solve_info out{};
    out.rel_change = -1.0;
    const int rc = p->kind == CIP_PRIOR_PATCH ? solve_patch_adaptive(p, prm, d_x, st, out)
                                              : solve_conv_adaptive(p, prm, d_x, st, out);
    p->solved_once = true;
    if (info) *info = out;
    return rc;
  }
  if (is_itv(p) || p->kind == CIP_PRIOR_WDCT3D) {
    cip_solve_info out{};
    out.rel_change = -1.0;
    const int rc = is_itv(p) ? solve_itv_adaptive(p, d_y, prm, d_x, st, out)
                             : solve_wdct_adaptive(p, d_y, prm, d_x, st, out);
    p->solved_once = true;
    if (info) *info = out;
    return rc;
  }
  const Layout& L = p->L;
  const int iters = prm->max_iters, every = prm->every;
  const double rho0 = p->rho;
  double rho = rho0;
  cip_solve_info out{};
  out.rel_change = -1.0;
  std::vector<float> sums;
  float* xb0 = p->at<float>(L.xbuf);
  float* xb1 = xb0 + (size_t)p->S * p->N1 * p->N2;
  auto xbuf = [&](int l) { return (l & 1) ? xb1 : xb0; };
  auto xhat0 = [&]() -> hipError_t {
    // Alg. 1 step 2 with the current tables: x_hat0 = Psi^+ beta Lambda^H F y / (N1 N2)
    hipError_t e = row_r2c<float>(d_y, p->at<cx<float>>(L.bufB), p->K, p->N1, p->N2,
                                  p->at<const cx<float>>(L.twN2f), st);
    if (e != hipSuccess) return e;
    return col_op<float, OP_XHAT0>(p->at<const cx<float>>(L.bufB), p->at<void>(L.xh0), p->K, p->S,
                                   p->N1, p->H2, p->at<const cx<float>>(L.twN1f),
                                   p->at<const cx<float>>(L.Mm), 0, st);
  };
  int rc = CIP_OK;
  auto body = [&]() -> int {
    HIP_TRY(xhat0());
    HIP_TRY(admm_col(p, 1, iters > 1 ? 1 : 0, st));   // x^1 (t = u = 0)
    for (int l = 1;; ++l) {
      const bool check = l % every == 0 && l < iters;   // the last iterate is returned anyway
      const bool store = (l + 1) % every == 0 && l < iters;   // keep x^l for the next check
      double next = rho;
      bool stop = false;
      if (check || store) {
        int groups = 0;
        HIP_TRY(norm_pass(p, l, rho, store ? xbuf(l) : nullptr,
                          check && l > 1 ? xbuf(l - 1) : nullptr, st, &groups));
        if (check) {
          sums.resize((size_t)groups * 4);
          HIP_TRY(hipMemcpyAsync(sums.data(), p->at<float>(L.sums), sums.size() * 4,
                                 hipMemcpyDeviceToHost, st));
          HIP_TRY(hipStreamSynchronize(st));
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          for (int b = 0; b < groups; ++b)
            for (int i = 0; i < 4; ++i) acc[i] += (double)sums[(size_t)b * 4 + i];
          const double r = std::sqrt(acc[0]), sres = rho * std::sqrt(acc[1]);
          out.r_norm = r;
          out.s_norm = sres;
          if (l > 1) {
            out.rel_change = acc[3] > 0.0 ? std::sqrt(acc[2] / acc[3]) : 0.0;
            stop = out.rel_change < prm->tol;
          }
          if (!stop) {
            if (r > prm->mu * sres) next = prm->tau * rho;
            else if (sres > prm->mu * r) next = rho / prm->tau;
          }
        }
      }
      if (stop || l == iters) {
        out.iters = l;
        if (stop && is_dct(p) && l < iters) {
          // the column pass of this iteration applied the column DCT for the
          // next row pass: redo it without (its input, bufA, is intact)
          HIP_TRY(admm_col(p, 0, 0, st));
        }
        HIP_TRY(admm_row_dct(p, ROW_FINAL, st, d_x));
        break;
      }
      HIP_TRY(admm_row(p, l, st, rho, (float)(rho / next), check || store));
      if (next != rho) {
        HIP_TRY(gram(p, st, next));
        HIP_TRY(xhat0());
        rho = next;
        ++out.rho_changes;
      }
      HIP_TRY(admm_col(p, 0, l + 1 < iters ? 1 : 0, st));
    }
    return CIP_OK;
  };
  rc = body();
  out.rho = rho;
  if (rho != rho0) {   // leave the plan's tables at its own penalty
    hipError_t e = gram(p, st, rho0);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess && rc == CIP_OK)
      rc = fail(CIP_EHIP, std::string("restoring the tables: ") + hipGetErrorString(e));
  }
  p->solved_once = true;
  if (info) *info = out;
  return rc;
}

int cip_plan_state_bytes(cip_plan_t p, size_t* bytes) {
  if (!p || !bytes) return fail(CIP_EINVAL, "NULL argument");
  *bytes = p->L.state_bytes;
  return CIP_OK;
}

int cip_plan_attach(cip_plan_t base, void* d_state, size_t bytes, cip_plan_t* out) {
  if (!base || !d_state || !out) return fail(CIP_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(d_state) % 256)
    return fail(CIP_EINVAL, "state buffer must be 256-byte aligned");
  if (bytes < base->L.state_bytes) return fail(CIP_ENOSPC, "state buffer too small");
  cip_plan_s* p = new cip_plan_s(*base);
  // the copy must not share the base plan's captured loop (it holds the
  // base's state addresses)
  p->loop_graph = nullptr;
  p->loop_exec = nullptr;
  p->loop_iters = 0;
  p->last_iters = 0;
  p->sws = reinterpret_cast<unsigned char*>(d_state);
  p->solved_once = false;
  p->attached = true;
  *out = p;
  return CIP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
// Many independent solves fanned out over internal streams (fork / join on
// the caller's stream with events), either launched directly or captured
// once into a hipGraph and replayed with a single launch. Problems are
// assigned to streams largest-first onto the least-loaded stream.
struct cip_batch_s {
  std::vector<cip_plan_t> plans;
  std::vector<const float*> y;
  std::vector<float*> x;
  std::vector<int> iters;
  std::vector<std::vector<int>> lanes;   // problem indices per stream
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Fork / join of the solves over `streams`: lanes[i] lists the problems of
// stream i.
int fork_join(const std::vector<std::vector<int>>& lanes, const std::vector<hipStream_t>& streams,
              hipEvent_t fork, const std::vector<hipEvent_t>& join, const cip_plan_t* plans,
              const float* const* y, const int* iters, float* const* x, hipStream_t origin) {
  HIP_TRY(hipEventRecord(fork, origin));
  for (size_t i = 0; i < lanes.size(); ++i) {
    HIP_TRY(hipStreamWaitEvent(streams[i], fork, 0));
    for (int j : lanes[i]) {
      int rc = cip_solve(plans[j], y[j], iters[j], x[j], streams[i]);
      if (rc) return rc;
    }
    HIP_TRY(hipEventRecord(join[i], streams[i]));
    HIP_TRY(hipStreamWaitEvent(origin, join[i], 0));
  }
  return CIP_OK;
}

int batch_enqueue(cip_batch_s* b, hipStream_t origin) {
  return fork_join(b->lanes, b->streams, b->fork, b->join, b->plans.data(), b->y.data(),
                   b->iters.data(), b->x.data(), origin);
}

// Problems spread largest-first (cost ~ N1 N2 (S + K) iters) onto the
// least-loaded of ns lanes.
std::vector<std::vector<int>> assign_lanes(int n, const cip_plan_t* plans, const int* iters,
                                           int ns) {
  std::vector<std::vector<int>> lanes(ns);
  std::vector<double> load(ns, 0.0), cost(n);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    const cip_plan_t p = plans[i];
    cost[i] = (double)p->N1 * p->N2 * (p->S + p->K) * iters[i];
  }
  std::sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  for (int i : order) {
    int best = 0;
    for (int k = 1; k < ns; ++k)
      if (load[k] < load[best]) best = k;
    lanes[best].push_back(i);
    load[best] += cost[i];
  }
  return lanes;
}

int check_batch_args(int n, const cip_plan_t* plans, const float* const* d_y, const int* iters,
                     float* const* d_x) {
  if (n < 1 || !plans || !d_y || !iters || !d_x) return fail(CIP_EINVAL, "bad argument");
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || !d_y[i] || !d_x[i] || iters[i] < 1) return fail(CIP_EINVAL, "bad problem entry");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(CIP_EINVAL, "a plan may appear once per batch");
  }
  return CIP_OK;
}

// Internal streams and events of cip_batch_solve, per device, created at the
// first call on that device and kept until the process ends.
constexpr int kPoolStreams = 4;
struct StreamPool {
  bool ready = false;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
};
std::mutex g_pool_mu;
StreamPool g_pool[64];

void batch_free(cip_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto s : b->streams) (void)hipStreamDestroy(s);
  delete b;
}

}  // namespace

extern "C" {

int cip_batch_solve(int n, const cip_plan_t* plans, const float* const* d_y, const int* iters,
                    float* const* d_x, void* stream) {
  int rc = check_batch_args(n, plans, d_y, iters, d_x);
  if (rc) return rc;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(CIP_EHIP, "cip_batch_solve: no usable current device");
  std::lock_guard<std::mutex> lock(g_pool_mu);
  StreamPool& P = g_pool[dev];
  if (!P.ready) {
    P.streams.assign(kPoolStreams, nullptr);
    P.join.assign(kPoolStreams, nullptr);
    for (int k = 0; k < kPoolStreams; ++k) {
      HIP_TRY(hipStreamCreateWithFlags(&P.streams[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&P.join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&P.fork, hipEventDisableTiming));
    P.ready = true;
  }
  const int ns = n < kPoolStreams ? n : kPoolStreams;
  const std::vector<hipStream_t> streams(P.streams.begin(), P.streams.begin() + ns);
  const std::vector<hipEvent_t> join(P.join.begin(), P.join.begin() + ns);
  return fork_join(assign_lanes(n, plans, iters, ns), streams, P.fork, join, plans, d_y, iters,
                   d_x, reinterpret_cast<hipStream_t>(stream));
}

int cip_batch_create(int n, const cip_plan_t* plans, const float* const* d_y, const int* iters,
                     float* const* d_x, int n_streams, int use_graph, cip_batch_t* out) {
  if (!out) return fail(CIP_EINVAL, "bad argument");
  if (n_streams < 1 || n_streams > 64) return fail(CIP_EINVAL, "n_streams must be in [1, 64]");
  int crc = check_batch_args(n, plans, d_y, iters, d_x);
  if (crc) return crc;
  if (use_graph)
    for (int i = 0; i < n; ++i)
      if (plans[i]->learn)
        return fail(CIP_EUNSUPPORTED, "dictionary-learning plans are not captured into a graph");
  cip_batch_s* b = new cip_batch_s();
  b->plans.assign(plans, plans + n);
  b->y.assign(d_y, d_y + n);
  b->x.assign(d_x, d_x + n);
  b->iters.assign(iters, iters + n);
  const int ns = n_streams < n ? n_streams : n;
  b->lanes = assign_lanes(n, plans, iters, ns);
  auto bail = [&](int code, const std::string& m) {
    batch_free(b);
    return fail(code, m);
  };
  b->streams.resize(ns, nullptr);
  b->join.resize(ns, nullptr);
  for (int k = 0; k < ns; ++k) {
    if (hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking) != hipSuccess)
      return bail(CIP_EHIP, "hipStreamCreate failed");
    if (hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) != hipSuccess)
      return bail(CIP_EHIP, "hipEventCreate failed");
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    return bail(CIP_EHIP, "hipEventCreate failed");
  if (use_graph) {
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return bail(CIP_EHIP, "hipStreamCreate failed");
    int rc = CIP_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) != hipSuccess) rc = CIP_EHIP;
    if (!rc) rc = batch_enqueue(b, cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      std::string m = g_last_error;
      return bail(rc, "graph capture failed: " + m);
    }
    if (e != hipSuccess || !g) return bail(CIP_EHIP, "hipStreamEndCapture failed");
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
      return bail(CIP_EHIP, "hipGraphInstantiate failed");
  }
  *out = b;
  return CIP_OK;
}

int cip_batch_launch(cip_batch_t b, void* stream) {
  if (!b) return fail(CIP_EINVAL, "NULL batch");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (b->exec) {
    HIP_TRY(hipGraphLaunch(b->exec, st));
    for (auto p : b->plans) p->solved_once = true;
    return CIP_OK;
  }
  return batch_enqueue(b, st);
}

int cip_batch_destroy(cip_batch_t b) {
  if (b) batch_free(b);
  return CIP_OK;
}

int cip_plan_autotune(cip_plan_t p, int reps, void* stream, cip_tuning* out) {
  if (!p || reps < 1) return fail(CIP_EINVAL, "bad argument");
  if (!p->solved_once) return fail(CIP_EINVAL, "run cip_solve on this plan first");
  if (p->kind == CIP_PRIOR_PATCH || p->kind == CIP_PRIOR_CONV2D || p->kind == CIP_PRIOR_CONV3D ||
      is_itv(p) || p->kind == CIP_PRIOR_WDCT3D)
    return fail(CIP_EUNSUPPORTED, "autotuning covers the l1 analysis row passes");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool dct = is_dct(p);
  const int pd = ppt_row_n(p->N2);
  const bool has8 = is_pow2(p->N2) && pd != 8 && (dct || p->N2 <= 1024);
  struct Cand { int np, ppt; };
  std::vector<Cand> cands = {{PAIRS, pd}};
  if (has8) cands.push_back({PAIRS, 8});
  {   // half-tile row passes (all l1 analysis priors)
    cands.push_back({2, pd});
    if (has8) cands.push_back({2, 8});
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = 1e300, first = 0.0;
  Cand pick = cands[0];
  for (size_t c = 0; c < cands.size(); ++c) {
    p->row_np = cands[c].np;
    p->row_ppt = cands[c].ppt;
    for (int r = 0; r < 2; ++r) HIP_TRY(admm_row(p, 2 + (r & 1), st));   // warm-up
    HIP_TRY(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIP_TRY(admm_row(p, 2 + (r & 1), st));
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    const double us = 1e3 * ms / reps;
    if (c == 0) first = us;
    if (us < best) {
      best = us;
      pick = cands[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->row_np = pick.np;
  p->row_ppt = pick.ppt;
  if (out) {
    out->row_np = pick.np;
    out->row_ppt = pick.ppt;
    out->row_us = best;
    out->default_us = first;
    out->candidates = (int)cands.size();
  }
  return CIP_OK;
}

int cip_plan_set_tuning(cip_plan_t p, int row_np, int row_ppt) {
  if (!p) return fail(CIP_EINVAL, "NULL plan");
  const bool dct = is_dct(p);
  const int pd = ppt_row_n(p->N2);
  const bool has8 = is_pow2(p->N2) && pd != 8 && (dct || p->N2 <= 1024);
  if (p->kind == CIP_PRIOR_PATCH || p->kind == CIP_PRIOR_CONV2D || p->kind == CIP_PRIOR_CONV3D ||
      is_itv(p) || p->kind == CIP_PRIOR_WDCT3D)
    return fail(CIP_EUNSUPPORTED, "tuning covers the l1 analysis row passes");
  if (!(row_np == PAIRS || row_np == 2)) return fail(CIP_EINVAL, "row_np must be 4 or 2");
  if (!(row_ppt == pd || (has8 && row_ppt == 8)))
    return fail(CIP_EINVAL, "row_ppt must be the default or 8 (power-of-two N2)");
  if (p->row_np != row_np || p->row_ppt != row_ppt) p->drop_loop_graph();
  p->row_np = row_np;
  p->row_ppt = row_ppt;
  return CIP_OK;
}

int cip_time_kernel(cip_plan_t p, int which, int reps, void* stream, double* avg_us) {
  if (!p || !avg_us || reps < 1) return fail(CIP_EINVAL, "bad argument");
  if (!p->solved_once) return fail(CIP_EINVAL, "run cip_solve on this plan first");
  if (which < 0 || which > 2) return fail(CIP_EINVAL, "which must be 0, 1 or 2");
  const bool conv = p->kind == CIP_PRIOR_CONV2D || p->kind == CIP_PRIOR_CONV3D,
             patch = p->kind == CIP_PRIOR_PATCH;
  if (which == 2 && !patch && !conv)
    return fail(CIP_EINVAL, "which = 2 needs the patch or convolutional prior");
  if ((patch || p->kind == CIP_PRIOR_WDCT3D) && which == 0)
    return fail(CIP_EINVAL, "this prior has no fused row pass");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) {
    const Layout& L = p->L;
    const size_t F = (size_t)p->N1 * p->H2;
    if (conv) {
      const int P = p->n_filters * p->S;
      if (which == 0)
        HIP_TRY(conv_row(p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.rtc), p->at<float>(L.vconv),
                         P, p->N1, p->N2, p->at<const cx<float>>(L.twN2f),
                         (float)(p->lambda / p->rho), (float)(1.0 / ((double)p->N1 * p->N2)), 0, st));
      else if (which == 1)
        HIP_TRY(conv_col_fft(1, p->at<const cx<float>>(L.rtc), p->at<cx<float>>(L.gv), P, p->N1,
                             p->H2, p->at<const cx<float>>(L.twN1f), st));
      else
        HIP_TRY(conv_freq_pass(p, 0, 0, 1, st));
      continue;
    }
    if (which == 0) HIP_TRY(admm_row(p, 2 + (r & 1), st));
    else if (which == 1) HIP_TRY(admm_col(p, 0, 1, st));
    else HIP_TRY(patch_z_launch(p->S, p->n_atoms, p->at<const float>(p->L.rimg),
                                p->at<float>(p->L.vpatch), p->at<float>(p->L.tbuf),
                                p->at<const uint16_t>(p->L.dbf), p->at<const uint16_t>(p->L.m1bf),
                                p->N1, p->N2, (float)(p->lambda / p->rho), 0, st));
  }
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_us = 1000.0 * ms / reps;
  return CIP_OK;
}

}  // extern "C"
