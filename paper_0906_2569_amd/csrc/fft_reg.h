// Register-resident 1D transforms of length L = 4 * LS, one quad of lanes per
// transform.  Each lane keeps LS complex values in VGPRs; the transform is a
// per-lane LS-point DFT (compile-time mixed radix 2/3/4/5, fully unrolled,
// with its twiddles folded to constants), a twiddle, and a 4-point DFT across
// the quad through DPP quad permutes.
//
//  inverse ("to real space", sign s = +1), decimation in time:
//    lane q holds x[q + 4 j] (j < LS)  ->  lane q holds X[k + LS p] (k < LS)
//  forward (sign s = -1), decimation in frequency:
//    lane q holds y[k + LS p] (k < LS) ->  lane q holds Y[q + 4 m] (m < LS)
//  with p = quad_block(q), the bit-reversed lane index of the radix-2^2
//  network across the quad.
//
// so the output layout of one direction is the input layout of the other,
// and a pointwise product between them needs no data exchange.
// The lane twiddles come from a table tw[m] = exp(+2 pi i m / L), m < L (LDS).
#pragma once
#include "fft.h"

// cos(2 pi m / N) and sin(2 pi m / N) at compile time: the angle is reduced on
// the integer m to [0, pi/4] by octant symmetry, then summed as a Taylor
// series (error below 2.5e-16 in float64).
namespace croot {
constexpr double kPi4 = 0.78539816339744830962;
constexpr double sin_poly(double x) {
  const double x2 = x * x;
  double t = 1.0;
  for (int k = 13; k >= 1; --k) t = 1.0 - t * x2 / ((2.0 * k) * (2.0 * k + 1.0));
  return x * t;
}
constexpr double cos_poly(double x) {
  const double x2 = x * x;
  double t = 1.0;
  for (int k = 13; k >= 1; --k) t = 1.0 - t * x2 / ((2.0 * k - 1.0) * (2.0 * k));
  return t;
}
struct CS {
  double c, s;
};
// 8 m = o N + r: octant o, angle (pi/4)(o + r/N)
constexpr CS root(long m, long N) {
  m %= N;
  if (m < 0) m += N;
  const long a = 8 * m, o = a / N, r = a - o * N;
  const double f = (o % 2 == 0) ? kPi4 * (double)r / (double)N : kPi4 * (double)(N - r) / (double)N;
  const double c0 = cos_poly(f), s0 = sin_poly(f);
  switch (o) {
    case 0: return {c0, s0};
    case 1: return {s0, c0};
    case 2: return {-s0, c0};
    case 3: return {-c0, s0};
    case 4: return {-c0, -s0};
    case 5: return {-s0, -c0};
    case 6: return {s0, -c0};
    default: return {c0, -s0};
  }
}
template <int N>
struct Roots {
  double c[N], s[N];
  constexpr Roots() : c(), s() {
    for (int m = 0; m < N; ++m) {
      const CS w = root(m, N);
      c[m] = w.c;
      s[m] = w.s;
    }
  }
};
// indexed with compile-time offsets only, so every entry folds to a constant
template <int N>
struct RootTab {
  static constexpr Roots<N> v{};
};
}  // namespace croot

namespace regfft {

template <int N>
struct SmallFactor {
  static constexpr int value = (N % 4 == 0 && N > 4) ? 4
                             : (N % 3 == 0 && N > 3) ? 3
                             : (N % 2 == 0 && N > 2) ? 2
                             : (N % 5 == 0 && N > 5) ? 5
                                                     : N;
};

template <typename T>
__device__ __forceinline__ cpx<T> twid(const cpx<T>* tw, int idx, T s) {
  cpx<T> w = tw[idx];
  w.y *= s;
  return w;
}

template <typename T>
__device__ __forceinline__ T tfma(T a, T b, T c);
template <>
__device__ __forceinline__ double tfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float tfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// In-place N-point DFT of x[0..N) in registers, X_k = sum_n x_n W^(s n k),
// W = exp(2 pi i / N); the twiddles are compile-time constants.
template <int N, typename T, int F = SmallFactor<N>::value>
struct RDft {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) {
    constexpr int N1 = F, N2 = N / F;
    cpx<T> a[N];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      cpx<T> t[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) t[n1] = x[N2 * n1 + n2];
      Dft<N1, T>::run(t, s);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        cpx<T> v = t[k1];
        if ((n2 * k1) % N != 0) {
          const int m = (n2 * k1) % N;
          const cpx<T> w{(T)croot::RootTab<N>::v.c[m], s * (T)croot::RootTab<N>::v.s[m]};
          v = cmul(v, w);
        }
        a[n2 * N1 + k1] = v;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      cpx<T> t[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) t[n2] = a[n2 * N1 + k1];
      RDft<N2, T>::run(t, s);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) x[k1 + N1 * k2] = t[k2];
    }
  }
};

template <int N, typename T>
struct RDft<N, T, N> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) { Dft<N, T>::run(x, s); }
};

template <typename T>
struct RDft<1, T, 1> {
  static __device__ __forceinline__ void run(cpx<T>*, T) {}
};

// value of lane (q ^ D) of the quad, through a DPP quad permute
template <int D>
__device__ __forceinline__ float qx(float v) {
  constexpr int ctrl = D == 1 ? 0xB1 : (D == 2 ? 0x4E : 0x1B);
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, true));
}
template <int D>
__device__ __forceinline__ double qx(double v) {
  constexpr int ctrl = D == 1 ? 0xB1 : (D == 2 ? 0x4E : 0x1B);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int D, typename T>
__device__ __forceinline__ cpx<T> qxc(cpx<T> v) { return cpx<T>{qx<D>(v.x), qx<D>(v.y)}; }

// Radix-2^2 network across the quad, lane q = q0 + 2 q1.  Each stage
// exchanges with one partner lane (DPP) and forms partner + sign * self with
// one FMA per component (sign = -1 on the upper lane of the pair, an exact
// product, so the sums round as plain additions would).
template <typename T>
struct QuadLane {
  T sg1, sg2;   // -1 where q0 = 1, resp. q1 = 1, else +1
  T mr, mi;     // internal twiddle W_4^(q0 p0): (0, 1) on lane 3, else (1, 0)
};

template <typename T>
__device__ __forceinline__ QuadLane<T> quad_lane(int q) {
  QuadLane<T> l;
  l.sg1 = (q & 1) ? T(-1) : T(1);
  l.sg2 = (q & 2) ? T(-1) : T(1);
  l.mr = q == 3 ? T(0) : T(1);
  l.mi = q == 3 ? T(1) : T(0);
  return l;
}

template <int D, typename T>
__device__ __forceinline__ cpx<T> bfly(cpx<T> self, T sg) {
  const cpx<T> o = qxc<D>(self);
  return cpx<T>{tfma(sg, self.x, o.x), tfma(sg, self.y, o.y)};
}

// b * (mr + i s mi): the identity on lanes 0..2, i s on lane 3.  float64 uses
// exact FMAs against the lane constants; float32 selects (cheaper there).
template <typename T>
__device__ __forceinline__ cpx<T> quad_twiddle(cpx<T> b, const QuadLane<T>& l, T s) {
  const T mi = s * l.mi;
  return cpx<T>{tfma(b.x, l.mr, -b.y * mi), tfma(b.x, mi, b.y * l.mr)};
}
template <>
__device__ __forceinline__ cpx<float> quad_twiddle<float>(cpx<float> b, const QuadLane<float>& l, float s) {
  const bool rot = l.mi != 0.0f;
  return cpx<float>{rot ? -s * b.y : b.x, rot ? s * b.x : b.y};
}

// block index held by lane q after inv_dit (bit-reversed 2-bit lane index)
__device__ __forceinline__ int quad_block(int q) { return ((q & 1) << 1) | (q >> 1); }

// lane q holds b_q; returns X_p = sum_q b_q W_4^(s q p) for p = quad_block(q)
template <typename T>
__device__ __forceinline__ cpx<T> quad_dit(cpx<T> b, const QuadLane<T>& l, T s) {
  b = bfly<2>(b, l.sg2);           // sum over q1: (-1)^(q1 p0), p0 = q1
  b = quad_twiddle(b, l, s);       // W_4^(s q0 p0)
  return bfly<1>(b, l.sg1);        // sum over q0: (-1)^(q0 p1), p1 = q0
}

// lane q holds y_p for p = quad_block(q); returns B_q = sum_p y_p W_4^(s p q)
template <typename T>
__device__ __forceinline__ cpx<T> quad_dif(cpx<T> y, const QuadLane<T>& l, T s) {
  y = bfly<1>(y, l.sg1);           // sum over p1 = q0: (-1)^(p1 q'0)
  y = quad_twiddle(y, l, s);       // W_4^(s p0 q'0)
  return bfly<2>(y, l.sg2);        // sum over p0 = q1: (-1)^(p0 q'1)
}

// inverse direction (s = +1): lane q holds x[q + 4 j]  ->  X[k + LS p], p = quad_block(q)
template <int LS, typename T>
__device__ __forceinline__ void inv_dit(cpx<T> (&x)[LS], int q, const QuadLane<T>& l, const cpx<T>* tw) {
  const T s = T(1);
  RDft<LS, T>::run(x, s);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    if (k != 0) x[k] = cmul(x[k], twid(tw, q * k, s));   // q k < 4 LS
    x[k] = quad_dit(x[k], l, s);
  }
}

// forward direction (s = -1): lane q holds y[k + LS p], p = quad_block(q)  ->  Y[q + 4 m]
template <int LS, typename T>
__device__ __forceinline__ void fwd_dif(cpx<T> (&x)[LS], int q, const QuadLane<T>& l, const cpx<T>* tw) {
  const T s = T(-1);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    x[k] = quad_dif(x[k], l, s);
    if (k != 0) x[k] = cmul(x[k], twid(tw, q * k, s));
  }
  RDft<LS, T>::run(x, s);
}

}  // namespace regfft
