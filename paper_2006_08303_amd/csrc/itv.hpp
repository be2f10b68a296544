// Isotropic TV prior (Section III-A: Phi(Tx) = TV(x) with T = I), either one
// 2D TV per plane or one TV of the whole cube whose gradient also has the
// forward difference along the planes (none after the last plane). The
// x-update is that of a unitary T (tau = 1); the t-update is the TV proximal
// map of f = x + u with weight mu = lambda / rho, computed with Chambolle's
// projection algorithm (circular forward differences along the image axes),
// whose dual p is kept in the state and warm-starts the next ADMM iteration:
//   q = div p - f / mu,   p <- (p + tau grad q) / (1 + tau |grad q|),
//   t = f - mu div p,     u <- u + x - t = f - t,
// with div p = (p0[n1] - p0[n1-1]) + (p1[n2] - p1[n2-1]) [+ p2[s] - p2[s-1]]
// (the negative adjoint of the forward differences; p2 of the last plane is
// 0). The step is 1/8 per plane and 1/12 along the planes (the squared norm
// of div is at most 8, resp. 12). Per ADMM iteration: k_itv_prep (inverse
// row FFT, f = x + u), ceil(inner / KB) launches of k_itv_chambolle or
// k_itv3_chambolle (up to KB iterations each, in LDS), k_itv_finish (t, u,
// forward row FFT of t - u for the next column pass).
// State planes [S][N1][N2] each: u, dual buffer A (p0, p1[, p2]), dual
// buffer B (p0, p1[, p2]), f.
#pragma once
#include "kernels.hpp"

namespace cip {

// Inverse row FFT of the column-pass output (x rows), f = x + u; on the
// first iteration u = 0 and the dual starts at p = 0 (p2 is null per plane).
// x is also written to xo when given (the iterate of an adaptive check).
template <int N2>
__global__ void __launch_bounds__(PAIRS * (N2 / ppt_row<N2>()))
k_itv_prep(const cx<float>* __restrict__ Yin, const float* __restrict__ u, float* __restrict__ f,
           float* __restrict__ p0, float* __restrict__ p1, float* __restrict__ p2,
           float* __restrict__ xo, int N1, const cx<float>* __restrict__ twg, int first) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int s = b / tiles, row0 = (b % tiles) * RT;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  const size_t oa = ((size_t)s * N1 + row0 + 2 * g) * N2, ob = oa + N2;
  // the dual of both rows, loaded before the transform so that the loads
  // overlap it
  float ua[PPT], ub[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = t + T * q;
    ua[q] = first ? 0.f : u[oa + n];
    ub[q] = first ? 0.f : u[ob + n];
  }
  lds_load_table(tw, twg, N2);
  tile_to_staging(Yin + rt_tile_base(s, row0, N1, H2), stg, H2 * RT);
  __syncthreads();
  cx<float> v[PPT];
  staging_to_pair<N2, PPT>(v, stg, g, t);
  __syncthreads();
  fft_group<N2, PPT, -1>(v, cb, t, tw);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int n = t + T * q;
    f[oa + n] = v[q].x + ua[q];
    f[ob + n] = v[q].y + ub[q];
    if (xo) {
      xo[oa + n] = v[q].x;
      xo[ob + n] = v[q].y;
    }
    if (first) {
      p0[oa + n] = p0[ob + n] = 0.f;
      p1[oa + n] = p1[ob + n] = 0.f;
      if (p2) p2[oa + n] = p2[ob + n] = 0.f;
    }
  }
}

// Up to KB Chambolle iterations on one TS x TS tile of one plane, in LDS
// (temporal blocking). The tile is loaded with a halo of KB pixels on every
// side (circular wrap): one iteration makes p at a pixel depend on p within
// one pixel in each direction, so after m <= KB iterations only the cells
// within m pixels of the region border are stale, and the TS x TS interior
// equals what m global iterations give. Reads the dual from
// (pi0, pi1) and writes the interior to (po0, po1): two buffers, because
// neighbouring tiles read the halo of the input. Per iteration:
//   q = div p - f / mu                 at region rows, cols >= 1
//   p <- (p + tau grad q) / (1 + tau |grad q|)   at rows, cols in [1, W - 2]
// (no cell reads outside the region; the cells left out never reach the
// interior). One work-group per (plane, tile).
template <int TS, int KB>
__global__ void __launch_bounds__(256)
k_itv_chambolle(const float* __restrict__ f, const float* __restrict__ pi0,
                const float* __restrict__ pi1, float* __restrict__ po0, float* __restrict__ po1,
                int N1, int N2, int iters, float inv_mu, float tau) {
  constexpr int W = TS + 2 * KB;
  constexpr int R = W * W;
  // every cell's own values stay in registers (slot k of this thread holds
  // cell e = threadIdx.x + 256 k); LDS carries what the neighbours read
  constexpr int NSLOT = (R + 255) / 256;
  __shared__ float P0[R], P1[R], Q[R];
  const int tx = N2 / TS, ty = N1 / TS;
  const int s = blockIdx.x / (tx * ty), rem = blockIdx.x % (tx * ty);
  const int r0 = (rem / tx) * TS - KB, c0 = (rem % tx) * TS - KB;
  const size_t pl = (size_t)s * N1 * N2;
  float rp0[NSLOT], rp1[NSLOT], rf[NSLOT], rq[NSLOT];
  // every slot's loads first (all in flight together), then the LDS copies
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    const int e = threadIdx.x + 256 * k;
    rp0[k] = rp1[k] = rf[k] = rq[k] = 0.f;
    if (e < R) {
      // r0 + a lies in [-KB, N1 + KB) and KB < N1 (likewise for columns)
      int gr = r0 + e / W, gc = c0 + e % W;
      gr += gr < 0 ? N1 : (gr >= N1 ? -N1 : 0);
      gc += gc < 0 ? N2 : (gc >= N2 ? -N2 : 0);
      const size_t i = pl + (size_t)gr * N2 + gc;
      rp0[k] = pi0[i];
      rp1[k] = pi1[i];
      rf[k] = f[i];
    }
  }
  // which cells take part in the q and p updates
  unsigned qm = 0, pm = 0;
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    const int e = threadIdx.x + 256 * k;
    const int a = e / W, c = e % W;
    if (e < R) {
      P0[e] = rp0[k];
      P1[e] = rp1[k];
      if (a >= 1 && c >= 1) {
        qm |= 1u << k;
        if (a <= W - 2 && c <= W - 2) pm |= 1u << k;
      }
    }
  }
  for (int it = 0; it < iters; ++it) {
    __syncthreads();   // P0, P1 hold the current dual
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
      const int e = threadIdx.x + 256 * k;
      if ((qm >> k) & 1u) {
        rq[k] = (rp0[k] - P0[e - W]) + (rp1[k] - P1[e - 1]) - rf[k] * inv_mu;
        Q[e] = rq[k];
      }
    }
    __syncthreads();   // Q complete; P0, P1 no longer read this iteration
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
      const int e = threadIdx.x + 256 * k;
      if ((pm >> k) & 1u) {
        const float g0 = Q[e + W] - rq[k], g1 = Q[e + 1] - rq[k];
        // hardware square root and reciprocal (about 1 ulp each)
        const float inv = __builtin_amdgcn_rcpf(
            1.f + tau * __builtin_amdgcn_sqrtf(g0 * g0 + g1 * g1));
        rp0[k] = (rp0[k] + tau * g0) * inv;
        rp1[k] = (rp1[k] + tau * g1) * inv;
        P0[e] = rp0[k];
        P1[e] = rp1[k];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TS * TS; e += 256) {
    const int a = e / TS, c = e % TS;
    const int l = (a + KB) * W + c + KB;
    const size_t i = pl + (size_t)(r0 + KB + a) * N2 + (c0 + KB + c);
    po0[i] = P0[l];
    po1[i] = P1[l];
  }
}

// Band-coupled form: one work-group per TS x TS tile holds every plane, and
// each thread keeps the S values of its pixel columns in registers, so the
// band differences of div and grad are register arithmetic; LDS carries the
// in-plane neighbours as in k_itv_chambolle, whose halo argument holds
// unchanged (the coupling along the planes does not widen the spatial
// dependence). Per iteration, at every plane s:
//   q = (p0 - p0[n1-1]) + (p1 - p1[n2-1]) + (p2[s] - p2[s-1]) - f / mu
//   g = (q[n1+1] - q, q[n2+1] - q, q[s+1] - q), the last plane's g2 = 0
//   p <- (p + tau g) / (1 + tau |g|)
// with p2[-1] = 0; p2 of the last plane starts at 0, so it stays 0 and is
// written as 0. The interior is written from registers.
template <int S, int TS, int KB, int NT>
__global__ void __launch_bounds__(NT)
k_itv3_chambolle(const float* __restrict__ f, const float* __restrict__ pi0,
                 const float* __restrict__ pi1, const float* __restrict__ pi2,
                 float* __restrict__ po0, float* __restrict__ po1, float* __restrict__ po2,
                 int N1, int N2, int iters, float inv_mu, float tau) {
  constexpr int W = TS + 2 * KB;
  constexpr int R = W * W;
  constexpr int NSLOT = (R + NT - 1) / NT;
  static_assert(3 * S * R * 4 <= 65536, "tile does not fit in 64 KiB of LDS");
  __shared__ float P0[S * R], P1[S * R], Q[S * R];
  const int tx = N2 / TS;
  const int r0 = ((int)blockIdx.x / tx) * TS - KB, c0 = ((int)blockIdx.x % tx) * TS - KB;
  const size_t pn = (size_t)N1 * N2;
  float rp0[NSLOT][S], rp1[NSLOT][S], rp2[NSLOT][S], rf[NSLOT][S], rq[NSLOT][S];
  size_t gi[NSLOT];
  unsigned qm = 0, pm = 0, om = 0;
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    const int e = threadIdx.x + NT * k;
    const int a = e / W, c = e % W;
    gi[k] = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) rp0[k][s] = rp1[k][s] = rp2[k][s] = rf[k][s] = rq[k][s] = 0.f;
    if (e < R) {
      // r0 + a lies in [-KB, N1 + KB) and KB < N1 (likewise for columns)
      int gr = r0 + a, gc = c0 + c;
      gr += gr < 0 ? N1 : (gr >= N1 ? -N1 : 0);
      gc += gc < 0 ? N2 : (gc >= N2 ? -N2 : 0);
      gi[k] = (size_t)gr * N2 + gc;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const size_t i = s * pn + gi[k];
        rp0[k][s] = pi0[i];
        rp1[k][s] = pi1[i];
        if (s < S - 1) rp2[k][s] = pi2[i];
        rf[k][s] = f[i];
        P0[s * R + e] = rp0[k][s];
        P1[s * R + e] = rp1[k][s];
      }
      if (a >= 1 && c >= 1) {
        qm |= 1u << k;
        if (a <= W - 2 && c <= W - 2) pm |= 1u << k;
      }
      if (a >= KB && a < KB + TS && c >= KB && c < KB + TS) om |= 1u << k;
    }
  }
  for (int it = 0; it < iters; ++it) {
    __syncthreads();   // P0, P1 hold the current dual
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
      const int e = threadIdx.x + NT * k;
      if ((qm >> k) & 1u) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float b = s > 0 ? rp2[k][s] - rp2[k][s - 1] : rp2[k][s];
          rq[k][s] = (rp0[k][s] - P0[s * R + e - W]) + (rp1[k][s] - P1[s * R + e - 1]) + b -
                     rf[k][s] * inv_mu;
          Q[s * R + e] = rq[k][s];
        }
      }
    }
    __syncthreads();   // Q complete; P0, P1 no longer read this iteration
#pragma unroll
    for (int k = 0; k < NSLOT; ++k) {
      const int e = threadIdx.x + NT * k;
      if ((pm >> k) & 1u) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const float g0 = Q[s * R + e + W] - rq[k][s], g1 = Q[s * R + e + 1] - rq[k][s];
          const float g2 = s < S - 1 ? rq[k][s + 1] - rq[k][s] : 0.f;
          // hardware square root and reciprocal (about 1 ulp each)
          const float inv = __builtin_amdgcn_rcpf(
              1.f + tau * __builtin_amdgcn_sqrtf(g0 * g0 + g1 * g1 + g2 * g2));
          rp0[k][s] = (rp0[k][s] + tau * g0) * inv;
          rp1[k][s] = (rp1[k][s] + tau * g1) * inv;
          if (s < S - 1) rp2[k][s] = (rp2[k][s] + tau * g2) * inv;
          P0[s * R + e] = rp0[k][s];
          P1[s * R + e] = rp1[k][s];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    if ((om >> k) & 1u) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const size_t i = s * pn + gi[k];
        po0[i] = rp0[k][s];
        po1[i] = rp1[k][s];
        po2[i] = rp2[k][s];
      }
    }
  }
}

// t = f - mu div p, u = c (f - t), and the forward row FFT of t - u (two
// rows per group) -> RT tile of the next column pass. c = 1, or
// rho / rho' when an adaptive solve changes the penalty after this
// iteration's t-update (the scaled dual is rescaled; f and p are unchanged,
// so the pass can run again with the new c). BAND: div has the band term
// p2[s] - p2[s-1] (no p2[S-1] term); both loads are made on every plane (at
// in-range addresses) and the terms selected, so they issue with the others.
template <int N2, bool BAND>
__global__ void __launch_bounds__(PAIRS * (N2 / ppt_row<N2>()))
k_itv_finish(const float* __restrict__ f, const float* __restrict__ p0,
             const float* __restrict__ p1, const float* __restrict__ p2, int S,
             float* __restrict__ u, cx<float>* __restrict__ Gout,
             int N1, const cx<float>* __restrict__ twg, float mu, float c) {
  constexpr int PPT = ppt_row<N2>();
  constexpr int T = N2 / PPT;
  constexpr int H2 = N2 / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<float>* tw = reinterpret_cast<cx<float>*>(smem_raw);
  float* lds = reinterpret_cast<float*>(smem_raw) + 2 * N2;
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  const int tiles = N1 / RT;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int s = b / tiles, row0 = (b % tiles) * RT;
  cx<float>* cb = reinterpret_cast<cx<float>*>(lds) + g * padded_len(N2);
  cx<float>* stg = reinterpret_cast<cx<float>*>(lds);
  lds_load_table(tw, twg, N2);
  const int ra = row0 + 2 * g, rup = ra == 0 ? N1 - 1 : ra - 1;
  const size_t pn = (size_t)N1 * N2, pl = (size_t)s * pn;
  const bool has_next = s < S - 1, has_prev = s > 0;
  cx<float> v[PPT];
  // QC points of both rows at a time: every load of a chunk is issued before
  // its arithmetic (p0 of the row above the pair once; the second row's
  // "above" is the first row's own p0)
  constexpr int QC = 4;
  static_assert(PPT % QC == 0, "points per thread must be a multiple of the chunk");
#pragma unroll
  for (int q0 = 0; q0 < PPT; q0 += QC) {
    float fv[QC][2], a0[QC][3], a1[QC][2], a1l[QC][2], b2[QC][2], b2p[QC][2];
#pragma unroll
    for (int k = 0; k < QC; ++k) {
      const int n = t + T * (q0 + k), nl = n == 0 ? N2 - 1 : n - 1;
      a0[k][0] = p0[pl + (size_t)rup * N2 + n];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const size_t i = pl + (size_t)(ra + r) * N2 + n;
        fv[k][r] = f[i];
        a0[k][r + 1] = p0[i];
        a1[k][r] = p1[i];
        a1l[k][r] = p1[pl + (size_t)(ra + r) * N2 + nl];
        if constexpr (BAND) {
          b2[k][r] = p2[i];
          b2p[k][r] = p2[has_prev ? i - pn : i];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < QC; ++k) {
      const int n = t + T * (q0 + k);
      float o[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const size_t i = pl + (size_t)(ra + r) * N2 + n;
        float dv = (a0[k][r + 1] - a0[k][r]) + (a1[k][r] - a1l[k][r]);
        if constexpr (BAND) {
          dv += has_next ? b2[k][r] : 0.f;
          dv -= has_prev ? b2p[k][r] : 0.f;
        }
        const float fi = fv[k][r];
        const float ti = fi - mu * dv;
        const float ui = c * (fi - ti);
        u[i] = ui;
        o[r] = ti - ui;
      }
      v[q0 + k] = cx<float>{o[0], o[1]};
    }
  }
  __syncthreads();   // twiddle table ready
  fft_group<N2, PPT, +1>(v, cb, t, tw);
  pair_to_staging<N2, PPT>(v, cb, stg, g, t);
  __syncthreads();
  staging_to_tile(Gout + rt_tile_base(s, row0, N1, H2), stg, H2 * RT);
}

}  // namespace cip
