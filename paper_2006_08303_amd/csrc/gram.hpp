// FP64 per-frequency Gram precompute (Algorithm 1/2, step 2).
//
// At every 2D frequency w the x-update of Eq. solx_Trans_DFT needs
//   Psi(w) = wgt * tau(w) I (+ wgt * L_band) + beta Lambda(w)^H Lambda(w),
// an S x S Hermitian matrix (below Eq. solx_Trans_DFT: its blocks are the
// diagonal matrices Psi_{i,j}). Where the kernel spectra nearly vanish and the
// weight is small, Psi is badly conditioned, so it is formed and inverted in
// FP64 (cyclic complex Jacobi eigen-decomposition; eigenvalues below rcond
// times the largest are dropped, giving the pseudo-inverse), and only the
// finished products are rounded to FP32:
//   A(w) = coefA * scale * Psi^+          (packed Hermitian: diag + upper)
//   M(w) = beta * scale * Psi^+ Lambda^H  (S x K), so that x_hat0 = M F y
// The paper proposes a recursive 2x2 block inversion (Eq. recinv) for this
// step; a small dense eigen-solve per lane serves here because it also yields
// the pseudo-inverse of singular blocks.
#pragma once
#include "fft.hpp"

namespace cip {

struct GramArgs {
  int K, N1, N2, H2;
  double wgt;       // rho (analysis) or c_P (synthesis): weight of the identity/symbol
  int tv_symbol;    // 1: tau(w) = (2 - 2 cos w1) + (2 - 2 cos w2); 0: tau = 1
  int band_lap;     // 1: add wgt * path-graph Laplacian over the S planes
  double beta;
  double coefA;     // rho (analysis: the x-update multiplies T^H(t-u) by rho) or 1
  double scale;     // 1 / (N1 N2)
  double rcond;
};

template <typename R> __device__ __forceinline__ cx<R> cconjmul(cx<R> a, cx<R> b) {  // conj(a) * b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

template <int S>
__global__ void k_gram(const cx<double>* __restrict__ lam64, GramArgs a, float* __restrict__ Adiag,
                       cx<float>* __restrict__ Aoff, cx<float>* __restrict__ Mm,
                       cx<float>* __restrict__ lam32) {
  const size_t F = (size_t)a.N1 * a.H2;
  const size_t f = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int k2 = (int)(f / a.N1), k1 = (int)(f % a.N1);
  cx<double> P[S][S];
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) P[i][j] = cx<double>{0.0, 0.0};
  for (int k = 0; k < a.K; ++k) {
    cx<double> L[S];
    for (int s = 0; s < S; ++s) {
      L[s] = lam64[(size_t)(k * S + s) * F + f];
      lam32[(size_t)(k * S + s) * F + f] = cx<float>{(float)L[s].x, (float)L[s].y};
    }
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) {
        cx<double> p = cconjmul(L[i], L[j]);
        P[i][j].x += a.beta * p.x;
        P[i][j].y += a.beta * p.y;
      }
  }
  double tau = 1.0;
  if (a.tv_symbol) {
    double w1 = 2.0 * kPi * (double)k1 / (double)a.N1;
    double w2 = 2.0 * kPi * (double)k2 / (double)a.N2;
    tau = (2.0 - 2.0 * cos(w1)) + (2.0 - 2.0 * cos(w2));
  }
  for (int i = 0; i < S; ++i) P[i][i].x += a.wgt * tau;
  if (a.band_lap) {
    for (int s = 0; s + 1 < S; ++s) {
      P[s][s].x += a.wgt;
      P[s + 1][s + 1].x += a.wgt;
      P[s][s + 1].x -= a.wgt;
      P[s + 1][s].x -= a.wgt;
    }
  }
  for (int i = 0; i < S; ++i) P[i][i].y = 0.0;

  // cyclic Jacobi: P <- U^H P U, V <- V U
  cx<double> V[S][S];
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) V[i][j] = cx<double>{i == j ? 1.0 : 0.0, 0.0};
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < S; ++i) {
      dia += P[i][i].x * P[i][i].x;
      for (int j = i + 1; j < S; ++j) off += P[i][j].x * P[i][j].x + P[i][j].y * P[i][j].y;
    }
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < S - 1; ++p)
      for (int q = p + 1; q < S; ++q) {
        cx<double> apq = P[p][q];
        double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
        if (mag == 0.0) continue;
        cx<double> e = {apq.x / mag, -apq.y / mag};   // exp(-i phi)
        double theta = (P[q][q].x - P[p][p].x) / (2.0 * mag);
        double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(tt * tt + 1.0), sn = tt * c;
        // U on the (p, q) plane: Upp = c, Upq = sn, Uqp = -sn e, Uqq = c e
        cx<double> Upp = {c, 0.0}, Upq = {sn, 0.0};
        cx<double> Uqp = {-sn * e.x, -sn * e.y}, Uqq = {c * e.x, c * e.y};
        for (int r = 0; r < S; ++r) {  // P U (columns)
          cx<double> rp = P[r][p], rq = P[r][q];
          P[r][p] = cmul(rp, Upp) + cmul(rq, Uqp);
          P[r][q] = cmul(rp, Upq) + cmul(rq, Uqq);
          cx<double> vp = V[r][p], vq = V[r][q];
          V[r][p] = cmul(vp, Upp) + cmul(vq, Uqp);
          V[r][q] = cmul(vp, Upq) + cmul(vq, Uqq);
        }
        for (int r = 0; r < S; ++r) {  // U^H (P U) (rows)
          cx<double> pr = P[p][r], qr = P[q][r];
          P[p][r] = cconjmul(Upp, pr) + cconjmul(Uqp, qr);
          P[q][r] = cconjmul(Upq, pr) + cconjmul(Uqq, qr);
        }
        P[p][q] = cx<double>{0.0, 0.0};
        P[q][p] = cx<double>{0.0, 0.0};
        P[p][p].y = 0.0;
        P[q][q].y = 0.0;
      }
  }
  double mu[S], mumax = 0.0;
  for (int i = 0; i < S; ++i) {
    mu[i] = P[i][i].x;
    mumax = fmax(mumax, fabs(mu[i]));
  }
  double inv[S];
  for (int i = 0; i < S; ++i) inv[i] = (mu[i] > a.rcond * mumax) ? 1.0 / mu[i] : 0.0;
  // Psi^+ = sum_i inv_i v_i v_i^H  (reuse P)
  for (int r = 0; r < S; ++r)
    for (int cc = 0; cc < S; ++cc) {
      cx<double> acc = {0.0, 0.0};
      for (int i = 0; i < S; ++i) {
        cx<double> t = cmul(V[r][i], conjx(V[cc][i]));
        acc.x += inv[i] * t.x;
        acc.y += inv[i] * t.y;
      }
      P[r][cc] = acc;
    }
  const double sA = a.coefA * a.scale;
  int pi = 0;
  for (int i = 0; i < S; ++i) {
    Adiag[(size_t)i * F + f] = (float)(sA * P[i][i].x);
    for (int j = i + 1; j < S; ++j, ++pi)
      Aoff[(size_t)pi * F + f] = cx<float>{(float)(sA * P[i][j].x), (float)(sA * P[i][j].y)};
  }
  const double sM = a.beta * a.scale;
  for (int k = 0; k < a.K; ++k) {
    cx<double> L[S];
    for (int s = 0; s < S; ++s) L[s] = lam64[(size_t)(k * S + s) * F + f];
    for (int s = 0; s < S; ++s) {
      cx<double> acc = {0.0, 0.0};
      for (int j = 0; j < S; ++j) acc = acc + cmul(P[s][j], conjx(L[j]));
      Mm[(size_t)(s * a.K + k) * F + f] = cx<float>{(float)(sM * acc.x), (float)(sM * acc.y)};
    }
  }
}

}  // namespace cip
