// LDS-resident Stockham FFT building blocks for gfx950 (wave64).
//
// A length-N transform is carried by a group of T = N / PPT threads; thread t
// holds PPT complex values in registers. On entry and on exit of `fft_group`,
// register slot q of thread t holds element t + T*q (input x, output X), so
// global loads and stores in that order are coalesced. The first radix is
// PPT (taken straight from registers), middle stages exchange through LDS
// (real and imaginary parts in separate padded float arrays to avoid bank
// conflicts), and a last, smaller radix finishes lengths that are not a power
// of PPT. Twiddles come from a per-length table W_N^m = exp(-2 pi i m / N)
// computed on the host in double precision.
//
// The in-register DFT kernels use compile-time twiddles (constexpr cos/sin).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cip {

template <typename R> struct cx { R x, y; };
template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R> __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R> __device__ __forceinline__ cx<R> conjx(cx<R> a) { return {a.x, -a.y}; }
template <typename R> __device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <int DIR, typename R> __device__ __forceinline__ cx<R> mul_mi(cx<R> a) {
  if constexpr (DIR > 0) return {a.y, -a.x};   // -i * a
  else return {-a.y, a.x};                     // +i * a
}

// ---------------------------------------------------------------- constexpr trig
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double cexpr_sin_series(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cexpr_cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi k / n, exact symmetry handling for the common angles
constexpr double ccos2pi(int k, int n) {
  k = ((k % n) + n) % n;
  if (4 * k == n) return 0.0;
  if (4 * k == 3 * n) return 0.0;
  if (2 * k == n) return -1.0;
  if (k == 0) return 1.0;
  double a = 2.0 * kPi * double(k) / double(n);
  if (a > kPi) a -= 2.0 * kPi;
  return cexpr_cos_series(a);
}
constexpr double csin2pi(int k, int n) {
  k = ((k % n) + n) % n;
  if (k == 0 || 2 * k == n) return 0.0;
  if (4 * k == n) return 1.0;
  if (4 * k == 3 * n) return -1.0;
  double a = 2.0 * kPi * double(k) / double(n);
  if (a > kPi) a -= 2.0 * kPi;
  return cexpr_sin_series(a);
}

// Multiply by W_n^k (DIR = +1: exp(-2 pi i k / n); DIR = -1: conjugate),
// with trivial angles special-cased at compile time.
template <int DIR, int K, int NN, typename R>
__device__ __forceinline__ cx<R> twc(cx<R> a) {
  constexpr int k = ((K % NN) + NN) % NN;
  if constexpr (k == 0) return a;
  else if constexpr (4 * k == NN) return mul_mi<DIR>(a);
  else if constexpr (2 * k == NN) return {-a.x, -a.y};
  else if constexpr (4 * k == 3 * NN) return mul_mi<-DIR>(a);
  else {
    constexpr double c = ccos2pi(k, NN);
    constexpr double s = -double(DIR) * csin2pi(k, NN);
    return {a.x * R(c) - a.y * R(s), a.x * R(s) + a.y * R(c)};
  }
}

// ---------------------------------------------------------------- in-register DFTs
template <int P> struct smallest_factor {
  static constexpr int value = (P % 4 == 0 && P > 4) ? 4 : (P % 2 == 0 ? 2 : (P % 3 == 0 ? 3 : P));
};

// 3-point DFT: X1,2 = a - (b + c)/2 -+ DIR * i * sin(pi/3) * (b - c)
template <int DIR, typename R> __device__ __forceinline__ void dft3(cx<R>& a, cx<R>& b, cx<R>& c) {
  constexpr double s3 = 0.86602540378443864676372317075294;
  cx<R> t1 = b + c;
  cx<R> t2 = {a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y};
  cx<R> d = b - c;
  // t3 = -DIR * i * s3 * d = (DIR * s3 * d.y, -DIR * s3 * d.x)
  cx<R> t3 = {R(double(DIR) * s3) * d.y, R(-double(DIR) * s3) * d.x};
  a = a + t1;
  b = t2 + t3;
  c = t2 - t3;
}

template <int K, int M, int F, int MM, int P, int DIR, typename R, int STRIDE>
__device__ __forceinline__ void static_for_k(cx<R> (&sub)[F][MM], cx<R>* v);

// DFT of length P, in place, natural order in and out (stride-1 array).
template <int P, int DIR, typename R, int STRIDE = 1>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (P == 1) {
    return;
  } else if constexpr (P == 2) {
    cx<R> a = v[0], b = v[STRIDE];
    v[0] = a + b;
    v[STRIDE] = a - b;
  } else if constexpr (P == 3) {
    dft3<DIR>(v[0], v[STRIDE], v[2 * STRIDE]);
  } else if constexpr (P == 4) {
    cx<R> a = v[0], b = v[STRIDE], c = v[2 * STRIDE], d = v[3 * STRIDE];
    cx<R> s0 = a + c, s1 = a - c, s2 = b + d, s3 = mul_mi<DIR>(b - d);
    v[0] = s0 + s2;
    v[2 * STRIDE] = s0 - s2;
    v[STRIDE] = s1 + s3;
    v[3 * STRIDE] = s1 - s3;
  } else {
    // decimation in time by factor F: P = F * M
    constexpr int F = smallest_factor<P>::value;
    constexpr int M = P / F;
    cx<R> sub[F][M];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int m = 0; m < M; ++m) sub[f][m] = v[(m * F + f) * STRIDE];
#pragma unroll
    for (int f = 0; f < F; ++f) dft<M, DIR, R, 1>(sub[f]);
    // combine: X[k + M*r] = sum_f W_P^{f (k + M r)} Sub_f[k]
    //        = sum_f W_F^{f r} (W_P^{f k} Sub_f[k])
    static_for_k<0, M, F, M, P, DIR, R, STRIDE>(sub, v);
  }
}

template <int F, int K, int P, int DIR, typename R, int f = 0>
__device__ __forceinline__ void twiddle_col_impl(cx<R>* col) {
  if constexpr (f < F) {
    col[f] = twc<DIR, f * K, P>(col[f]);
    twiddle_col_impl<F, K, P, DIR, R, f + 1>(col);
  }
}

template <int K, int M, int F, int MM, int P, int DIR, typename R, int STRIDE>
__device__ __forceinline__ void static_for_k(cx<R> (&sub)[F][MM], cx<R>* v) {
  if constexpr (K < M) {
    cx<R> col[F];
#pragma unroll
    for (int f = 0; f < F; ++f) col[f] = sub[f][K];
    twiddle_col_impl<F, K, P, DIR, R>(col);
    dft<F, DIR, R, 1>(col);
#pragma unroll
    for (int r = 0; r < F; ++r) v[(K + M * r) * STRIDE] = col[r];
    static_for_k<K + 1, M, F, MM, P, DIR, R, STRIDE>(sub, v);
  }
}

// ---------------------------------------------------------------- LDS layout
// Padded index: one spare slot every 16 entries. Strides that are multiples of
// 16 stay affine (pad(a + 16 c) = pad(a) + 17 c), so unrolled accesses fold
// into immediate LDS offsets, and power-of-two strides spread over banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

// Synchronise the threads of one transform group. WS (wave-scope sync) may be
// set by kernels whose groups never share LDS with another group between
// their own explicit work-group barriers; a group of at most 64 threads then
// lies inside one wavefront (T divides 64), whose LDS operations are
// performed in order, so ordering its LDS accesses needs only a wavefront-
// scope release fence, the wave barrier and an acquire fence (the fences
// keep the compiler from moving LDS accesses across the barrier, which the
// bare wave barrier does not). Otherwise the work-group barrier is used.
template <int T, bool WS = false> __device__ __forceinline__ void group_sync() {
  if constexpr (WS && T <= 64 && 64 % T == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ---------------------------------------------------------------- group FFT
// Stockham radix sequence: PPT (first stage, from registers), then radices
// R_1, R_2, ... each dividing PPT, chosen greedily as the largest divisor of
// PPT that divides what remains of N / PPT (N = 1024, PPT = 16: 16, 16, 4;
// N = 384, PPT = 12: 12, 4, 4, 2). Twiddles of every stage after the first
// are stored per stage as [k in 0..Ns)[r in 1..Rs) = W_{Ns Rs}^{r k}
// (forward sign), Ns the product of the earlier radices, so a thread reads
// its Rs - 1 twiddles at consecutive addresses.
constexpr int next_radix(int rem, int ppt) {
  for (int d = ppt; d > 1; --d)
    if (ppt % d == 0 && rem % d == 0) return d;
  return 0;
}
template <int N, int PPT> struct fft_shape {
  static constexpr int T = N / PPT;
  static constexpr int nstages() {
    int rem = N / PPT, c = 0;
    while (rem > 1) {
      const int r = next_radix(rem, PPT);
      if (r == 0) return -1;
      rem /= r;
      ++c;
    }
    return c;
  }
  static constexpr int NST = nstages();   // stages after the first
  static constexpr int radix(int s) {      // radix of stage s = 1 .. NST
    int rem = N / PPT, r = 0;
    for (int i = 1; i <= s; ++i) {
      r = next_radix(rem, PPT);
      rem /= r;
    }
    return r;
  }
  static constexpr int ns(int s) {         // product of the radices before stage s
    int p = PPT;
    for (int i = 1; i < s; ++i) p *= radix(i);
    return p;
  }
  static constexpr int stage_off(int s) {  // twiddle-table offset of stage s
    int off = 0;
    for (int i = 1; i < s; ++i) off += ns(i) * (radix(i) - 1);
    return off;
  }
  static constexpr int TW_ENTRIES = stage_off(NST + 1);
  static_assert(N % PPT == 0, "N must be a multiple of PPT");
  static_assert(NST >= 0, "N / PPT must factor into divisors of PPT");
};

// One Stockham stage with radix RS on the group's LDS array buf, after
// radices with product NS have been applied.
template <int N, int PPT, int RS, int NS, int TWOFF, int DIR, bool LASTSTAGE, typename R,
          bool WS = false>
__device__ __forceinline__ void stage_lds(cx<R>* buf, int t, const cx<R>* tws, cx<R>* v) {
  constexpr int T = N / PPT;
  constexpr int NB = PPT / RS;   // butterflies per thread
  constexpr int STR = N / RS;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + T * b;
    if constexpr (STR % 16 == 0) {
      const int pj = pad(j);
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int idx = pj + r * (STR + STR / 16);
        v[b * RS + r] = buf[idx];
      }
    } else {
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int idx = pad(j + r * STR);
        v[b * RS + r] = buf[idx];
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + T * b;
    const int k = j % NS;
    const cx<R>* w = tws + TWOFF + k * (RS - 1) - 1;
#pragma unroll
    for (int r = 1; r < RS; ++r) {
      cx<R> ww = w[r];
      if (DIR < 0) ww.y = -ww.y;
      v[b * RS + r] = cmul(v[b * RS + r], ww);
    }
    dft<RS, DIR, R>(&v[b * RS]);
  }
  group_sync<T, WS>();
  if constexpr (!LASTSTAGE) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + T * b;
      const int k = j % NS;
      const int base = (j / NS) * NS * RS + k;
      if constexpr (NS % 16 == 0) {
        const int pb = pad(base);
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int idx = pb + r * (NS + NS / 16);
          buf[idx] = v[b * RS + r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int idx = pad(base + r * NS);
          buf[idx] = v[b * RS + r];
        }
      }
    }
    group_sync<T, WS>();
  }
}

template <int N, int PPT, int DIR, typename R, int S, bool WS = false>
__device__ __forceinline__ void later_stages(cx<R>* buf, int t, const cx<R>* tws, cx<R>* reg) {
  using SH = fft_shape<N, PPT>;
  if constexpr (S <= SH::NST) {
    constexpr bool last = S == SH::NST;
    stage_lds<N, PPT, SH::radix(S), SH::ns(S), SH::stage_off(S), DIR, last, R, WS>(buf, t, tws,
                                                                                  reg);
    later_stages<N, PPT, DIR, R, S + 1, WS>(buf, t, tws, reg);
  }
}

// Full transform of a group. In: reg[q] = x[t + T q]. Out: reg[q] = X[t + T q].
// buf: this group's LDS scratch of padded_len(N) complex values; tws: the
// stage twiddle table (LDS). The routine starts with a group barrier before
// its first LDS write, so callers may still have been reading buf.
// DIR = +1: forward (exp(-2 pi i jk/N)); DIR = -1: inverse, unnormalised.
// WS: wave-scope group synchronisation (see group_sync).
template <int N, int PPT, int DIR, typename R, bool WS = false>
__device__ __forceinline__ void fft_group(cx<R>* reg, cx<R>* buf, int t, const cx<R>* tws) {
  using SH = fft_shape<N, PPT>;
  constexpr int T = SH::T;
  if constexpr (N == 1) return;
  dft<PPT, DIR, R>(reg);   // first radix (Ns = 1, no twiddles)
  if constexpr (SH::NST == 0) {
    return;   // N == PPT
  } else {
    group_sync<T, WS>();
    if constexpr (16 % PPT == 0) {   // t * PPT + r stays within one padding block
      const int pb = pad(t * PPT);
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        buf[pb + r] = reg[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < PPT; ++r) {
        buf[pad(t * PPT + r)] = reg[r];
      }
    }
    group_sync<T, WS>();
    later_stages<N, PPT, DIR, R, 1, WS>(buf, t, tws, reg);
    // last stage: butterfly b, output r -> element t + T (b + r NB), where
    // registers hold [b][r]; reorder to reg[q] = X[t + T q]
    constexpr int RL = SH::radix(SH::NST);
    if constexpr (RL < PPT) {
      constexpr int NB = PPT / RL;
      cx<R> tmp[PPT];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < RL; ++r) tmp[b + r * NB] = reg[b * RL + r];
#pragma unroll
      for (int q = 0; q < PPT; ++q) reg[q] = tmp[q];
    }
  }
}

}  // namespace cip
