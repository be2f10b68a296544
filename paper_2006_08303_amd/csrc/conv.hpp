// Convolutional-dictionary synthesis prior, 2D-correlation form (a common set
// of M filters d_m for every plane: plane s ~ sum_m d_m * z_{m,s}; P = I),
// and the 3D form (k_conv_tables3, k_conv_freq3 below).
//
// One ADMM iteration of Algorithm 2, with all operators diagonal in the 2D
// DFT domain (Section IV-B):
//   x-update (Eq. solx_synt_DFT, c_P = 1): x^ = Psi^+ (b^ + d^), d^_s = sum_m theta_m z^_{m,s};
//   z-update (Eqs. solz_DFT, solz_DFT_SM) per frequency and plane: with
//     a = conj(theta) (M-vector), g^ = F(t - u),
//     v = g^ + a (x^_s - a^H g^) gamma,  gamma = 1 / (rho + |a|^2),
//   which equals Sherman-Morrison's rho^-1 (c - a a^H c gamma) for
//   c = a x^_s + rho g^ but has no 1/rho (stable in FP32 for small rho);
//   z = F^-1 v; soft threshold and dual update in space (Eq. softADMM).
// The state per code voxel is V = z + u_prev (t = soft(V), u = clip(V),
// t - u = 2 soft(V) - V). Transforms are unnormalised; the x^ tables carry no
// 1/(N1 N2), which the inverse transforms apply.
//
// Layouts: RT and FL as in kernels.hpp; code planes p = m * S + s.
#pragma once
#include "kernels.hpp"

namespace cip {

// Filter m (L x L, row-major) placed on the N1 x N2 torus with tap (a, b) at
// offset (a - L/2, b - L/2), promoted to double (plan time).
__global__ void k_place_filter(const float* __restrict__ filt, double* __restrict__ dst, int L,
                               int N1, int N2) {
  const size_t n = (size_t)N1 * N2;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int n1 = (int)(i / N2), n2 = (int)(i % N2);
  const int a = (n1 + L / 2) % N1, b = (n2 + L / 2) % N2;
  dst[i] = (a < L && b < L) ? (double)filt[a * L + b] : 0.0;
}

// theta (FP32) and, formed in FP64 at FL frequency f = k2 N1 + k1, with the
// code-gradient (Tikhonov) weight mu and the symbol of sum_i R_i^H R_i
// (circular forward differences along both axes),
//   psi = (2 - 2 cos w1) + (2 - 2 cos w2),  c = rho + mu psi,
//   gamma = 1 / (c + sum_m |theta_m|^2),     eta = rho / c.
__global__ void k_conv_tables(const cx<double>* __restrict__ th64, cx<float>* __restrict__ th32,
                              float* __restrict__ gam, float* __restrict__ eta, int M, size_t F,
                              double rho, double mu, int N1, int N2) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  double s = 0.0;
  for (int m = 0; m < M; ++m) {
    cx<double> t = th64[(size_t)m * F + f];
    s += t.x * t.x + t.y * t.y;
    th32[(size_t)m * F + f] = cx<float>{(float)t.x, (float)t.y};
  }
  double c = rho;
  if (mu > 0.0) {
    const int k2 = (int)(f / N1), k1 = (int)(f % N1);
    const double w1 = 2.0 * kPi * (double)k1 / (double)N1;
    const double w2 = 2.0 * kPi * (double)k2 / (double)N2;
    c += mu * ((2.0 - 2.0 * cos(w1)) + (2.0 - 2.0 * cos(w2)));
  }
  gam[f] = (float)(1.0 / (c + s));
  eta[f] = (float)(rho / c);
}

constexpr int CONV_PC = 4;   // planes per work-group in the batched column FFT

// Batched column FFT, one work-group per (column k2, chunk of CONV_PC planes).
// DIR = +1: RT -> FL (forward); DIR = -1: FL -> RT (inverse, unnormalised).
template <int N1, int DIR>
__global__ void k_col_fft_batch(const cx<float>* __restrict__ in, cx<float>* __restrict__ out, int P,
                                int H2, const cx<float>* __restrict__ twg) {
  constexpr int PPT = ppt_col<N1>();
  constexpr int T = N1 / PPT;
  constexpr int PL = padded_len(N1);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  cx<float>* cb = tw + N1 + (threadIdx.x / T) * PL;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int k2 = b % H2, chunk = b / H2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int p = chunk * CONV_PC + g;
  const bool live = p < P;
  lds_load_table(tw, twg, N1);
  cx<float> v[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int k1 = t + T * q;
    if (!live) v[q] = cx<float>{0.f, 0.f};
    else if (DIR > 0) v[q] = in[rt_idx(p, k1, k2, N1, H2)];
    else v[q] = in[fl_idx(p, k1, k2, N1, H2)];
  }
  __syncthreads();
  fft_group<N1, PPT, DIR>(v, cb, t, tw);
  if (live) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int k1 = t + T * q;
      if (DIR > 0) out[fl_idx(p, k1, k2, N1, H2)] = v[q];
      else out[rt_idx(p, k1, k2, N1, H2)] = v[q];
    }
  }
}

// Frequency pass, one thread per frequency f (FL order):
//   x^ = xh0 + A d^ (S x S, packed Hermitian A = Psi^+), stored to xhat;
//   if do_z: per plane s the stable Sherman-Morrison update of the M codes
//   (v overwrites g^ in gv) and the new d^_s = sum_m theta_m v_m. With the
//   Tikhonov term the diagonal is c = rho + mu psi(w) instead of rho, and
//   v = eta g^ + a (x^_s - a^H eta g^) gamma with eta = rho / c (eta = 1
//   without it).
// first: d^ = 0 (z = 0); zero_g: g^ = 0 (t = u = 0).
constexpr int CONV_MMAX = 32;   // filters per dictionary (at most)

// (S is a template parameter so that the per-plane arrays stay in registers.)
template <int S>
__global__ void __launch_bounds__(128)
k_conv_freq(cx<float>* __restrict__ gv, cx<float>* __restrict__ dhat,
            cx<float>* __restrict__ xhat, const cx<float>* __restrict__ xh0,
            const float* __restrict__ Adiag, const cx<float>* __restrict__ Aoff,
            const cx<float>* __restrict__ th, const float* __restrict__ gam,
            const float* __restrict__ eta, int M, size_t F, int first, int zero_g, int do_z) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  cx<float> d[S], xs[S];
#pragma unroll
  for (int s = 0; s < S; ++s) d[s] = first ? cx<float>{0.f, 0.f} : dhat[(size_t)s * F + f];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    cx<float> acc = xh0[(size_t)s * F + f];
    const float dg = Adiag[(size_t)s * F + f];
    acc.x += dg * d[s].x;
    acc.y += dg * d[s].y;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (j == s) continue;
      const cx<float> a = s < j ? Aoff[(size_t)pair_index(s, j, S) * F + f]
                                : conjx(Aoff[(size_t)pair_index(j, s, S) * F + f]);
      acc = acc + cmul(a, d[j]);
    }
    xs[s] = acc;
    xhat[(size_t)s * F + f] = acc;
  }
  if (!do_z) return;
  // the loads of all filter slots are unconditional (slots m >= M read slot
  // M - 1, finite values, and are multiplied by 0), so that they are issued
  // together rather than one per branch
  cx<float> t[CONV_MMAX];
#pragma unroll
  for (int m = 0; m < CONV_MMAX; ++m) {
    const cx<float> tm = th[(size_t)(m < M ? m : M - 1) * F + f];
    const float w = m < M ? 1.f : 0.f;
    t[m] = cx<float>{w * tm.x, w * tm.y};
  }
  const float gm = gam[f], et = eta[f];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    cx<float> g[CONV_MMAX];
    cx<float> ag = {0.f, 0.f};   // a^H g = sum_m theta_m g_m
    if (zero_g) {
#pragma unroll
      for (int m = 0; m < CONV_MMAX; ++m) g[m] = cx<float>{0.f, 0.f};
    } else {
#pragma unroll
      for (int m = 0; m < CONV_MMAX; ++m) {
        const cx<float> gg = gv[((size_t)(m < M ? m : M - 1) * S + s) * F + f];
        const float em = m < M ? et : 0.f;
        g[m] = cx<float>{em * gg.x, em * gg.y};
      }
    }
#pragma unroll
    for (int m = 0; m < CONV_MMAX; ++m)
      if (m < M) ag = ag + cmul(t[m], g[m]);
    const cx<float> r = {(xs[s].x - ag.x) * gm, (xs[s].y - ag.y) * gm};
    cx<float> dn = {0.f, 0.f};
#pragma unroll
    for (int m = 0; m < CONV_MMAX; ++m) {
      if (m < M) {
        const cx<float> vm = g[m] + cmulc(r, t[m]);   // g + conj(theta) r
        gv[((size_t)m * S + s) * F + f] = vm;
        dn = dn + cmul(t[m], vm);
      }
    }
    dhat[(size_t)s * F + f] = dn;
  }
}

// 3D form (filters and codes circular along the S planes too; every operator
// is diagonal in the 3D DFT over (band, n1, n2)). theta_m(w, k) for band
// frequency k = 1D DFT over the band taps of the 2D spectra of the filter
// slices; formed in FP64 at plan time, stored [M][k][F] in FP32, with
// gamma(w, k) = 1 / (rho + sum_m |theta_m(w, k)|^2) stored [k][F].
__global__ void k_conv_tables3(const cx<double>* __restrict__ th64, cx<float>* __restrict__ th32,
                               float* __restrict__ gam, int M, int S, size_t F, double rho) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  for (int k = 0; k < S; ++k) {
    double sum = 0.0;
    for (int m = 0; m < M; ++m) {
      cx<double> acc = {0.0, 0.0};
      for (int sp = 0; sp < S; ++sp) {
        // exp(-2 pi i k s' / S)
        double sn, cs;
        sincospi(-2.0 * (double)((k * sp) % S) / (double)S, &sn, &cs);
        acc = acc + cmul(th64[((size_t)m * S + sp) * F + f], cx<double>{cs, sn});
      }
      th32[((size_t)m * S + k) * F + f] = cx<float>{(float)acc.x, (float)acc.y};
      sum += acc.x * acc.x + acc.y * acc.y;
    }
    gam[(size_t)k * F + f] = (float)(1.0 / (rho + sum));
  }
}

// Frequency pass of the 3D form, one thread per 2D frequency f (FL order),
// all S planes and M codes:
//   x^ = xh0 + A d^ as in the 2D form (d^_s from the previous code update);
//   band DFTs (unnormalised, bw[k][s] = exp(-2 pi i k s / S)):
//     X(k) = sum_s x^_s bw[k][s],   G_m(k) = sum_s g^_{m,s} bw[k][s];
//   Sherman-Morrison per band frequency k (Eq. solz_DFT_SM at every 3D
//   frequency): r(k) = (X(k) - sum_m theta_m(k) G_m(k)) gamma(k),
//     V_m(k) = G_m(k) + conj(theta_m(k)) r(k);
//   v_{m,s} = (1/S) sum_k V_m(k) conj(bw[k][s])  (overwrites g^ in gv),
//   d^_s = (1/S) sum_k (sum_m theta_m(k) V_m(k)) conj(bw[k][s]).
// Two passes over the codes (first the r(k), then V) keep the registers to
// O(S). first: d^ = 0; zero_g: g^ = 0.
template <int S>
__global__ void __launch_bounds__(128)
k_conv_freq3(cx<float>* __restrict__ gv, cx<float>* __restrict__ dhat, cx<float>* __restrict__ xhat,
             const cx<float>* __restrict__ xh0, const float* __restrict__ Adiag,
             const cx<float>* __restrict__ Aoff, const cx<float>* __restrict__ th,
             const float* __restrict__ gam, const cx<float>* __restrict__ bw, int M, size_t F,
             int first, int zero_g, int do_z) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  cx<float> d[S], xs[S];
#pragma unroll
  for (int s = 0; s < S; ++s) d[s] = first ? cx<float>{0.f, 0.f} : dhat[(size_t)s * F + f];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    cx<float> acc = xh0[(size_t)s * F + f];
    const float dg = Adiag[(size_t)s * F + f];
    acc.x += dg * d[s].x;
    acc.y += dg * d[s].y;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (j == s) continue;
      const cx<float> a = s < j ? Aoff[(size_t)pair_index(s, j, S) * F + f]
                                : conjx(Aoff[(size_t)pair_index(j, s, S) * F + f]);
      acc = acc + cmul(a, d[j]);
    }
    xs[s] = acc;
    xhat[(size_t)s * F + f] = acc;
  }
  if (!do_z) return;
  cx<float> X[S], ag[S], r[S], dn[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    X[k] = cx<float>{0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S; ++s) X[k] = X[k] + cmul(xs[s], bw[k * S + s]);
    ag[k] = cx<float>{0.f, 0.f};
    dn[k] = cx<float>{0.f, 0.f};
  }
  // the codes are visited in chunks of CH filters whose loads are issued
  // together (slots past M read filter M - 1 and are multiplied by 0)
  constexpr int CH = S <= 2 ? 8 : (S <= 4 ? 4 : 2);
  if (!zero_g) {
    for (int m0 = 0; m0 < M; m0 += CH) {
      cx<float> g[CH][S], t[CH][S];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const size_t m = (size_t)(m0 + c < M ? m0 + c : M - 1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          g[c][s] = gv[(m * S + s) * F + f];
          t[c][s] = th[(m * S + s) * F + f];
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const float w = m0 + c < M ? 1.f : 0.f;
#pragma unroll
        for (int k = 0; k < S; ++k) {
          cx<float> G = {0.f, 0.f};
#pragma unroll
          for (int s = 0; s < S; ++s) G = G + cmul(g[c][s], bw[k * S + s]);
          ag[k] = ag[k] + cmul(cx<float>{w * t[c][k].x, w * t[c][k].y}, G);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float gm = gam[(size_t)k * F + f];
    r[k] = cx<float>{(X[k].x - ag[k].x) * gm, (X[k].y - ag[k].y) * gm};
  }
  const float invS = 1.f / (float)S;
  for (int m0 = 0; m0 < M; m0 += CH) {
    cx<float> g[CH][S], t[CH][S];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const size_t m = (size_t)(m0 + c < M ? m0 + c : M - 1);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        g[c][s] = zero_g ? cx<float>{0.f, 0.f} : gv[(m * S + s) * F + f];
        t[c][s] = th[(m * S + s) * F + f];
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int m = m0 + c;
      const float w = m < M ? 1.f : 0.f;
      cx<float> V[S];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        cx<float> G = {0.f, 0.f};
#pragma unroll
        for (int s = 0; s < S; ++s) G = G + cmul(g[c][s], bw[k * S + s]);
        const cx<float> tk = {w * t[c][k].x, w * t[c][k].y};
        V[k] = G + cmulc(r[k], tk);   // G + conj(theta) r
        dn[k] = dn[k] + cmul(tk, V[k]);
      }
      if (m < M) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          cx<float> acc = {0.f, 0.f};
#pragma unroll
          for (int k = 0; k < S; ++k) acc = acc + cmulc(V[k], bw[k * S + s]);
          gv[((size_t)m * S + s) * F + f] = cx<float>{acc.x * invS, acc.y * invS};
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < S; ++k) acc = acc + cmulc(dn[k], bw[k * S + s]);
    dhat[(size_t)s * F + f] = cx<float>{acc.x * invS, acc.y * invS};
  }
}

// ---------------------------------------------------------------- 3D dictionary update
// Online update of the 3D dictionary (Eqs. d_admm, sold_3D, g_admm, h_admm),
// one d, g, e step per outer iteration after the code update. d and e are
// full-size (M codes of S planes, N1 x N2), g lives on the L x L x S filter
// support (taps gtap [M][S][L][L]); spectra are unnormalised 2D DFTs per
// plane (FL order), the band axis transformed inside the kernels.

// d-update, one thread per 2D frequency: with Z_m(k), X(k), GE_m(k) the 3D
// spectra of the codes, of x and of g - e, Eq. sold_3D at every 3D frequency
// is (sigma I + a a^H) d = a X + sigma GE with a = conj(Z) (rank one plus
// sigma I); Sherman-Morrison in the form without 1/sigma (as for the codes),
//   r = (X - sum_m Z_m GE_m) / (sigma + sum_m |Z_m|^2),   d_m = GE_m + conj(Z_m) r,
// returned as plane spectra (inverse band DFT) plus the dual's, d^ + e^, in
// dsp [M][S][F] (what the projection needs; d^ itself is not kept).
template <int S>
__global__ void __launch_bounds__(128)
k_cdl_dfreq(const cx<float>* __restrict__ xhat, const cx<float>* __restrict__ zh,
            const cx<float>* __restrict__ gehat, const cx<float>* __restrict__ ehat,
            cx<float>* __restrict__ dsp, const cx<float>* __restrict__ bw, int M, size_t F,
            float sigma) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  cx<float> xs[S], X[S], ag[S];
  float aa[S];
#pragma unroll
  for (int s = 0; s < S; ++s) xs[s] = xhat[(size_t)s * F + f];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    X[k] = cx<float>{0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S; ++s) X[k] = X[k] + cmul(xs[s], bw[k * S + s]);
    ag[k] = cx<float>{0.f, 0.f};
    aa[k] = 0.f;
  }
  for (int m = 0; m < M; ++m) {
    cx<float> z[S], ge[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      z[s] = zh[((size_t)m * S + s) * F + f];
      ge[s] = gehat[((size_t)m * S + s) * F + f];
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      cx<float> Z = {0.f, 0.f}, G = {0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        Z = Z + cmul(z[s], bw[k * S + s]);
        G = G + cmul(ge[s], bw[k * S + s]);
      }
      ag[k] = ag[k] + cmul(Z, G);
      aa[k] += Z.x * Z.x + Z.y * Z.y;
    }
  }
  cx<float> r[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const float w = 1.f / (sigma + aa[k]);
    r[k] = cx<float>{(X[k].x - ag[k].x) * w, (X[k].y - ag[k].y) * w};
  }
  const float invS = 1.f / (float)S;
  for (int m = 0; m < M; ++m) {
    cx<float> z[S], ge[S], D[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      z[s] = zh[((size_t)m * S + s) * F + f];
      ge[s] = gehat[((size_t)m * S + s) * F + f];
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      cx<float> Z = {0.f, 0.f}, G = {0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        Z = Z + cmul(z[s], bw[k * S + s]);
        G = G + cmul(ge[s], bw[k * S + s]);
      }
      D[k] = G + cmul(conjx(Z), r[k]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      cx<float> acc = {0.f, 0.f};
#pragma unroll
      for (int k = 0; k < S; ++k) acc = acc + cmulc(D[k], bw[k * S + s]);
      const size_t o = ((size_t)m * S + s) * F + f;
      dsp[o] = cx<float>{acc.x * invS, acc.y * invS} + ehat[o];
    }
  }
}

// d-update of the 2D form (common filters): per 2D frequency the normal
// equation (sigma I + A A^H) d = A X + sigma GE with A = [a_1 .. a_S],
// a_s = conj(Z_{.,s}) (rank S plus sigma I; the sum over the planes noted in
// Section IV-B). Solved through the Woodbury identity in the form without
// 1/sigma,  d = GE + A y,  (sigma I_S + A^H A) y = X - A^H GE,
// with an S x S complex Cholesky factorisation per frequency. The condition
// number of sigma I_S + A^H A is about ||A||^2 / sigma (1e5 .. 1e9 for small
// sigma and strong codes), so the products, the factorisation and the solves
// run in FP64 on the FP32 operands; only d^ + e^ is rounded to FP32.
// zh [M][S][F] (codes), xhat [S][F], gehat, ehat and dsp [M][F]; dsp
// receives d^ + e^. B holds the upper triangle of A^H A packed by rows,
// element (s, t), t >= s, at tri(s, t); the factor L overwrites it in the
// transposed position, L(i, j) at tri(j, i).
template <int S>
__device__ __forceinline__ constexpr int tri(int s, int t) {
  return s * S - s * (s - 1) / 2 + (t - s);
}

template <int S>
__global__ void __launch_bounds__(128)
k_cdl_dfreq2(const cx<float>* __restrict__ xhat, const cx<float>* __restrict__ zh,
             const cx<float>* __restrict__ gehat, const cx<float>* __restrict__ ehat,
             cx<float>* __restrict__ dsp, int M, size_t F, float sigma) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  constexpr int NT = S * (S + 1) / 2;
  cx<double> B[NT], w[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const cx<float> xv = xhat[(size_t)s * F + f];
    w[s] = cx<double>{(double)xv.x, (double)xv.y};
  }
#pragma unroll
  for (int i = 0; i < NT; ++i) B[i] = cx<double>{0.0, 0.0};
  for (int m = 0; m < M; ++m) {
    cx<double> z[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cx<float> zv = zh[((size_t)m * S + s) * F + f];
      z[s] = cx<double>{(double)zv.x, (double)zv.y};
    }
    const cx<float> gf = gehat[(size_t)m * F + f];
    const cx<double> ge = {(double)gf.x, (double)gf.y};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      w[s] = w[s] - cmul(z[s], ge);                                       // X - A^H GE
#pragma unroll
      for (int t = s; t < S; ++t) B[tri<S>(s, t)] = B[tri<S>(s, t)] + cmulc(z[s], z[t]);
    }
  }
  // Cholesky sigma I + A^H A = L L^H. Every pivot is at least sigma (a Schur
  // complement of a PSD matrix plus sigma I): a smaller computed pivot is
  // rounding and is raised to sigma.
  const double sg = (double)sigma;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    double djj = B[tri<S>(j, j)].x + sg;
#pragma unroll
    for (int k = 0; k < j; ++k) {
      const cx<double> l = B[tri<S>(k, j)];
      djj -= l.x * l.x + l.y * l.y;
    }
    djj = djj > sg ? djj : sg;
    const double ljj = sqrt(djj), il = 1.0 / ljj;
    B[tri<S>(j, j)] = cx<double>{ljj, 0.0};
#pragma unroll
    for (int i = j + 1; i < S; ++i) {
      cx<double> a = conjx(B[tri<S>(j, i)]);   // (A^H A)_{i,j} = conj((A^H A)_{j,i})
#pragma unroll
      for (int k = 0; k < j; ++k) a = a - cmulc(B[tri<S>(k, i)], B[tri<S>(k, j)]);
      B[tri<S>(j, i)] = cx<double>{a.x * il, a.y * il};
    }
  }
  // L u = w, then L^H y = u
#pragma unroll
  for (int i = 0; i < S; ++i) {
    cx<double> a = w[i];
#pragma unroll
    for (int k = 0; k < i; ++k) a = a - cmul(B[tri<S>(k, i)], w[k]);
    const double d = B[tri<S>(i, i)].x;
    w[i] = cx<double>{a.x / d, a.y / d};
  }
#pragma unroll
  for (int i = S - 1; i >= 0; --i) {
    cx<double> a = w[i];
#pragma unroll
    for (int k = i + 1; k < S; ++k) a = a - cmul(conjx(B[tri<S>(i, k)]), w[k]);
    const double d = B[tri<S>(i, i)].x;
    w[i] = cx<double>{a.x / d, a.y / d};
  }
  for (int m = 0; m < M; ++m) {
    const cx<float> gf = gehat[(size_t)m * F + f];
    cx<double> d = {(double)gf.x, (double)gf.y};
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cx<float> zv = zh[((size_t)m * S + s) * F + f];
      d = d + cmul(cx<double>{(double)zv.x, -(double)zv.y}, w[s]);
    }
    const cx<float> ev = ehat[(size_t)m * F + f];
    dsp[(size_t)m * F + f] = cx<float>{(float)(d.x + (double)ev.x), (float)(d.y + (double)ev.y)};
  }
}

// Filter tables of the 2D form from FP32 spectra (theta already in th):
// gamma = 1 / (c + sum_m |theta_m|^2), eta = rho / c, c = rho + mu psi(w).
__global__ void k_conv_tables2f(const cx<float>* __restrict__ th, float* __restrict__ gam,
                                float* __restrict__ eta, int M, size_t F, double rho, double mu,
                                int N1, int N2) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  float sum = 0.f;
  for (int m = 0; m < M; ++m) {
    const cx<float> t = th[(size_t)m * F + f];
    sum += t.x * t.x + t.y * t.y;
  }
  double c = rho;
  if (mu > 0.0) {
    const int k2 = (int)(f / N1), k1 = (int)(f % N1);
    c += mu * ((2.0 - 2.0 * cospi(2.0 * (double)k1 / (double)N1)) +
               (2.0 - 2.0 * cospi(2.0 * (double)k2 / (double)N2)));
  }
  gam[f] = (float)(1.0 / (c + (double)sum));
  eta[f] = (float)(rho / c);
}

// d^_s = sum_m theta_m z^_{m,s} (2D form), after a dictionary change.
__global__ void k_conv_dhat2(const cx<float>* __restrict__ zh, const cx<float>* __restrict__ th,
                             cx<float>* __restrict__ dhat, int M, int S, size_t F) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  for (int s = 0; s < S; ++s) {
    cx<float> acc = {0.f, 0.f};
    for (int m = 0; m < M; ++m)
      acc = acc + cmul(th[(size_t)m * F + f], zh[((size_t)m * S + s) * F + f]);
    dhat[(size_t)s * F + f] = acc;
  }
}

// Support test of the filter grid placement: pixel (n1, n2) carries tap
// (a, b) = ((n1 + L/2) mod N1, (n2 + L/2) mod N2) when a, b < L.
__device__ __forceinline__ bool cdl_tap(int n1, int n2, int N1, int N2, int L, int& a, int& b) {
  a = (n1 + L / 2) % N1;
  b = (n2 + L / 2) % N2;
  return a < L && b < L;
}

// g-update: per filter m (one work-group each), w = d + e on the support,
// gtap = w / ||w||. dpl, e: [M][S][N1][N2]; e may be null (dpl then holds
// d + e).
__global__ void __launch_bounds__(256)
k_cdl_project(const float* __restrict__ dpl, const float* __restrict__ e, float* __restrict__ gtap,
              int S, int N1, int N2, int L) {
  const int m = blockIdx.x;
  const int taps = S * L * L;
  const size_t plane = (size_t)N1 * N2;
  __shared__ float red[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < taps; i += blockDim.x) {
    const int sp = i / (L * L), a = (i / L) % L, b = i % L;
    const int n1 = (a - L / 2 + N1) % N1, n2 = (b - L / 2 + N2) % N2;
    const size_t o = ((size_t)m * S + sp) * plane + (size_t)n1 * N2 + n2;
    const float w = dpl[o] + (e ? e[o] : 0.f);
    acc += w * w;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const float inv = red[0] > 0.f ? 1.f / __builtin_sqrtf(red[0]) : 0.f;
  for (int i = threadIdx.x; i < taps; i += blockDim.x) {
    const int sp = i / (L * L), a = (i / L) % L, b = i % L;
    const int n1 = (a - L / 2 + N1) % N1, n2 = (b - L / 2 + N2) % N2;
    const size_t o = ((size_t)m * S + sp) * plane + (size_t)n1 * N2 + n2;
    gtap[(size_t)m * taps + i] = (dpl[o] + (e ? e[o] : 0.f)) * inv;
  }
}

// The dual e is kept as plane spectra (the transforms are linear): with
// s = d^ + e^ (from the d-update) and g^ the spectra of the placed g,
// elementwise over [P][F]:
//   e^ <- e^ + d^ - g^ = s - g^,  ge <- g^ - e^ (the next right-hand side),
//   gs <- g^.
// (e is the scaled dual of the penalty sigma/2 ||d - g + e||^2 of Eqs.
// d_admm and g_admm, so it moves by the split residual d - g; the sign
// printed with Eq. h_admm makes e double every step and the solve diverge.)
// ge holds g^ on entry; gs may alias sd (s is read first).
__global__ void k_cdl_fdual(cx<float>* __restrict__ e, cx<float>* ge, const cx<float>* sd,
                            cx<float>* gs, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cx<float> g = ge[i], sv = sd[i];
  const cx<float> en = sv - g;
  e[i] = en;
  ge[i] = g - en;
  gs[i] = g;
}

// k_cdl_fdual at a check of the dictionary penalty (the rule of Section IV-C
// applied to sigma): the same updates, grid-stride over the work-groups, and
// per work-group b
//   part[2 b] = sum w |e^_new - e^_old|^2 = sum w |d^ - g^|^2, w = 1 on the
//     half-spectrum columns k2 = 0 and N2 / 2 and 2 elsewhere, so that the
//     total is N1 N2 ||D - G||^2 (Parseval, unnormalised transforms);
//   part[2 b + 1] = sum (gtap - gprev)^2 over the ntaps filter taps
//     (= ||G - G_prev||^2).
__global__ void __launch_bounds__(256)
k_cdl_fdual_res(cx<float>* __restrict__ e, cx<float>* ge, const cx<float>* sd, cx<float>* gs,
                size_t n, size_t F, int N1, int N2, const float* __restrict__ gtap,
                const float* __restrict__ gprev, size_t ntaps, float* __restrict__ part) {
  __shared__ float red[2][4];
  const size_t stride = (size_t)gridDim.x * 256;
  float a = 0.f, b = 0.f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const cx<float> g = ge[i], sv = sd[i], eo = e[i];
    const cx<float> en = sv - g;
    e[i] = en;
    ge[i] = g - en;
    gs[i] = g;
    const int k2 = (int)((i % F) / (size_t)N1);
    const float w = (k2 == 0 || 2 * k2 == N2) ? 1.f : 2.f;
    const float dx = en.x - eo.x, dy = en.y - eo.y;
    a += w * (dx * dx + dy * dy);
  }
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < ntaps; i += stride) {
    const float d = gtap[i] - gprev[i];
    b += d * d;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// A change sigma -> sigma' of the dictionary penalty: the scaled dual
// e^ <- c e^ (c = sigma / sigma'), and the next right-hand side ge = g^ - e^
// formed again from gs = g^.
__global__ void k_cdl_rescale_dual(cx<float>* __restrict__ e, cx<float>* __restrict__ ge,
                                   const cx<float>* __restrict__ gs, size_t n, float c) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cx<float> en = cx<float>{c * e[i].x, c * e[i].y};
  e[i] = en;
  ge[i] = gs[i] - en;
}

// e^ = 0 (start of a solve)
__global__ void k_cdl_fzero(cx<float>* __restrict__ e, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) e[i] = cx<float>{0.f, 0.f};
}

// Grid placement of the taps gtap [M][S][L][L] -> planes [M][S][N1][N2]:
// thread (n2, n1, plane) of a 3D grid (no index division).
__global__ void k_cdl_place(const float* __restrict__ gtap, float* __restrict__ out, int N1, int N2,
                            int L) {
  const int n2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (n2 >= N2) return;
  const int n1 = blockIdx.y;
  const size_t p = blockIdx.z;
  int a, b;
  out[(p * N1 + n1) * N2 + n2] = cdl_tap(n1, n2, N1, N2, L, a, b) ? gtap[(p * L + a) * L + b] : 0.f;
}

// Filter tables from the plane spectra th2 [M][S][F] of the placed taps
// (FP32 form of k_conv_tables3): theta_m(k) = sum_s' th2_{m,s'} bw[k][s'],
// gamma(k) = 1 / (rho + sum_m |theta_m(k)|^2).
template <int S>
__global__ void k_conv_tables3f(const cx<float>* __restrict__ th2, cx<float>* __restrict__ th32,
                                float* __restrict__ gam, const cx<float>* __restrict__ bw, int M,
                                size_t F, float rho) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  float sum[S];
#pragma unroll
  for (int k = 0; k < S; ++k) sum[k] = 0.f;
  for (int m = 0; m < M; ++m) {
    cx<float> t[S];
#pragma unroll
    for (int s = 0; s < S; ++s) t[s] = th2[((size_t)m * S + s) * F + f];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      cx<float> acc = {0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S; ++s) acc = acc + cmul(t[s], bw[k * S + s]);
      th32[((size_t)m * S + k) * F + f] = acc;
      sum[k] += acc.x * acc.x + acc.y * acc.y;
    }
  }
#pragma unroll
  for (int k = 0; k < S; ++k) gam[(size_t)k * F + f] = 1.f / (rho + sum[k]);
}

// d^_s = sum_m theta_m z^_m per 3D frequency, back to plane spectra (after a
// dictionary change, for the next x-update).
template <int S>
__global__ void k_conv_dhat3(const cx<float>* __restrict__ zh, const cx<float>* __restrict__ th,
                             cx<float>* __restrict__ dhat, const cx<float>* __restrict__ bw, int M,
                             size_t F) {
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  cx<float> dn[S];
#pragma unroll
  for (int k = 0; k < S; ++k) dn[k] = cx<float>{0.f, 0.f};
  for (int m = 0; m < M; ++m) {
    cx<float> z[S];
#pragma unroll
    for (int s = 0; s < S; ++s) z[s] = zh[((size_t)m * S + s) * F + f];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      cx<float> Z = {0.f, 0.f};
#pragma unroll
      for (int s = 0; s < S; ++s) Z = Z + cmul(z[s], bw[k * S + s]);
      dn[k] = dn[k] + cmul(th[((size_t)m * S + k) * F + f], Z);
    }
  }
  const float invS = 1.f / (float)S;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < S; ++k) acc = acc + cmulc(dn[k], bw[k * S + s]);
    dhat[(size_t)s * F + f] = cx<float>{acc.x * invS, acc.y * invS};
  }
}

// Row pass of the conv prior (pairs of rows of one code plane per group):
// inverse row FFT of v (z = scale * result), state update V = z + clip(V),
// w = 2 soft(V) - V, forward row FFT of w -> RT. first: V_prev = 0.
// rs (optional): the residuals of the split z = t, per wave of the group,
//   rs[2 i] = sum (z - t)^2 = sum (clip(V) - clip(V_prev))^2,
//   rs[2 i + 1] = sum (t - t_prev)^2 = sum (soft(V) - soft(V_prev))^2,
// i = blockIdx.x * waves + wave (conv_row_residual_floats entries in all).
template <int N2>
__global__ void __launch_bounds__(PAIRS * (N2 / ppt_row<N2>()), 2)
k_conv_row(const cx<float>* __restrict__ Vin, cx<float>* __restrict__ Gout, float* __restrict__ V,
           int N1, const cx<float>* __restrict__ twg, float kappa, float zscale, int first,
           float* __restrict__ rs) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  constexpr int NT = PAIRS * T;
  static_assert(NT % 64 == 0 || 64 % NT == 0, "waves of the row pass must be whole or one");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int p = b / tiles, row0 = (b % tiles) * RT;
  const int ra = row0 + 2 * g;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  lds_load_table(tw, twg, N2);
  tile_to_staging(Vin + rt_tile_base(p, row0, N1, H2), stg, H2 * RT);
  float* va = V + ((size_t)p * N1 + ra) * N2;
  float* vb = va + N2;
  float oa[PPT], ob[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    oa[q] = first ? 0.f : va[t + T * q];
    ob[q] = first ? 0.f : vb[t + T * q];
  }
  __syncthreads();
  cx<float> v[PPT];
  staging_to_pair<N2, PPT>(v, stg, g, t);
  __syncthreads();
  fft_group<N2, PPT, -1>(v, cb, t, tw);
  float r2 = 0.f, s2 = 0.f;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int k = t + T * q;
    const float na = zscale * v[q].x + clip_f(oa[q], kappa);
    const float nb = zscale * v[q].y + clip_f(ob[q], kappa);
    va[k] = na;
    vb[k] = nb;
    const float ta = soft_f(na, kappa), tb = soft_f(nb, kappa);
    v[q] = cx<float>{2.f * ta - na, 2.f * tb - nb};
    if (rs) {
      const float ra = clip_f(na, kappa) - clip_f(oa[q], kappa);
      const float rb = clip_f(nb, kappa) - clip_f(ob[q], kappa);
      const float da = ta - soft_f(oa[q], kappa), db = tb - soft_f(ob[q], kappa);
      r2 += ra * ra + rb * rb;
      s2 += da * da + db * db;
    }
  }
  if (rs) {   // fixed-order reduction over the lanes of each wave
    constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1) {
      r2 += __shfl_xor(r2, off, W);
      s2 += __shfl_xor(s2, off, W);
    }
    if ((threadIdx.x & (W - 1)) == 0) {
      const int i = blockIdx.x * (NT / W) + threadIdx.x / W;
      rs[2 * i] = r2;
      rs[2 * i + 1] = s2;
    }
  }
  fft_group<N2, PPT, +1>(v, cb, t, tw);
  pair_to_staging<N2, PPT>(v, cb, stg, g, t);
  __syncthreads();
  staging_to_tile(Gout + rt_tile_base(p, row0, N1, H2), stg, H2 * RT);
}

// A change of the penalty rho -> rho' between iterations (Section IV-C):
// the state V (t = soft(V, kappa), u = clip(V, kappa)) is re-expressed as
// V' = t + sc u with sc = rho / rho' (kappa' = lambda / rho' bounds sc u), and
// W = t - sc u = 2 soft(V', kappa') - V' is written for the forward
// transforms that rebuild g^ = F(t - u').
__global__ void k_conv_reemit(float* __restrict__ V, float* __restrict__ W, size_t n, float kappa,
                              float kappa_new, float sc) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float v = V[i];
    const float vn = soft_f(v, kappa) + sc * clip_f(v, kappa);
    V[i] = vn;
    W[i] = 2.f * soft_f(vn, kappa_new) - vn;
  }
}

}  // namespace cip
