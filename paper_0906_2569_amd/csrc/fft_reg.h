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

// ---------------------------------------------------------------------------
// Groups of G = 8 or 16 lanes: N = G LS, lane g (0..G-1) of a group of G
// consecutive lanes (inside one DPP row) holds x[g + G j], j < LS.  The same
// four-step factorization as the quad form: an LS-point DFT in each lane, the
// twiddle W_N^(s g k), then the G-point DFT across the lanes as log2(G)
// radix-2 stages (DPP exchanges with lanes g ^ 8, g ^ 4, g ^ 2, g ^ 1).
// ---------------------------------------------------------------------------

// value of lane g ^ 4 and of lane g ^ 8: one ds_swizzle each in its
// bit-mask mode (and 0x1F, or 0, xor 4 resp. 8 within groups of 32 lanes),
// through the LDS crossbar without touching LDS memory; two DPP row
// permutations would each take a vector ALU slot
__device__ __forceinline__ int lx4_b32(int v) { return __builtin_amdgcn_ds_swizzle(v, (4 << 10) | 0x1F); }
__device__ __forceinline__ int lx8_b32(int v) { return __builtin_amdgcn_ds_swizzle(v, (8 << 10) | 0x1F); }
template <int D>
__device__ __forceinline__ int lx_b32(int v) {
  if constexpr (D == 8) return lx8_b32(v);
  else if constexpr (D == 4) return lx4_b32(v);
  else return __builtin_amdgcn_mov_dpp(v, D == 1 ? 0xB1 : 0x4E, 0xF, 0xF, true);
}
template <int D>
__device__ __forceinline__ float lx(float v) { return __int_as_float(lx_b32<D>(__float_as_int(v))); }
template <int D>
__device__ __forceinline__ double lx(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lx_b32<D>((int)(b & 0xffffffffll));
  const int hi = lx_b32<D>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// partner + sg * self, partner = lane g ^ D
template <int D, typename T>
__device__ __forceinline__ cpx<T> gbfly(cpx<T> self, T sg) {
  const cpx<T> o{lx<D>(self.x), lx<D>(self.y)};
  return cpx<T>{tfma(sg, self.x, o.x), tfma(sg, self.y, o.y)};
}

// per-lane constants of the cross-lane stages (for s = +1; s = -1 conjugates)
template <typename T>
struct GLane {
  T sg1, sg2, sg4, sg8;   // -1 where bit 0, 1, 2, 3 of g is set, else +1
  T w2r, w2i;             // W_4^(g mod 2) where bit 1 is set, else 1
  T w4r, w4i;             // W_8^(g mod 4) where bit 2 is set, else 1
  T w8r, w8i;             // W_16^(g mod 8) where bit 3 is set, else 1
};

template <typename T>
__device__ __forceinline__ GLane<T> glane(int g) {
  // cos(pi m / 8), m = 0..4
  constexpr double c16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0};
  GLane<T> l;
  l.sg1 = (g & 1) ? T(-1) : T(1);
  l.sg2 = (g & 2) ? T(-1) : T(1);
  l.sg4 = (g & 4) ? T(-1) : T(1);
  l.sg8 = (g & 8) ? T(-1) : T(1);
  // W_16^m = (cos(pi m / 8), sin(pi m / 8)), m < 8; sin(pi m / 8) = cos(pi (4 - m) / 8)
  auto w16 = [&](int m, T& re, T& im) {
    re = (T)(m <= 4 ? c16[m] : -c16[8 - m]);
    im = (T)(m <= 4 ? c16[4 - m] : c16[m - 4]);
  };
  w16((g & 2) ? 4 * (g & 1) : 0, l.w2r, l.w2i);
  w16((g & 4) ? 2 * (g & 3) : 0, l.w4r, l.w4i);
  w16((g & 8) ? (g & 7) : 0, l.w8r, l.w8i);
  return l;
}

// b * (wr + i s wi)
template <typename T>
__device__ __forceinline__ cpx<T> grot(cpx<T> b, T wr, T wi, T s) {
  const T si = s * wi;
  return cpx<T>{tfma(b.x, wr, -b.y * si), tfma(b.x, si, b.y * wr)};
}

// decimation in frequency across the G lanes: lane g holds b_g; returns
// X_p = sum_g b_g W_G^(s g p) for p = the bit reversal of g (log2 G bits)
template <int G, typename T>
__device__ __forceinline__ cpx<T> g_dif(cpx<T> b, const GLane<T>& l, T s) {
  if constexpr (G == 16) {
    b = gbfly<8>(b, l.sg8);
    b = grot(b, l.w8r, l.w8i, s);
  }
  b = gbfly<4>(b, l.sg4);
  b = grot(b, l.w4r, l.w4i, s);
  b = gbfly<2>(b, l.sg2);
  b = grot(b, l.w2r, l.w2i, s);
  return gbfly<1>(b, l.sg1);
}

// decimation in time across the G lanes: lane g holds y_p for p = the bit
// reversal of g; returns Y_g = sum_p y_p W_G^(s p g)
template <int G, typename T>
__device__ __forceinline__ cpx<T> g_dit(cpx<T> y, const GLane<T>& l, T s) {
  y = gbfly<1>(y, l.sg1);
  y = grot(y, l.w2r, l.w2i, s);
  y = gbfly<2>(y, l.sg2);
  y = grot(y, l.w4r, l.w4i, s);
  y = gbfly<4>(y, l.sg4);
  if constexpr (G == 16) {
    y = grot(y, l.w8r, l.w8i, s);
    y = gbfly<8>(y, l.sg8);
  }
  return y;
}

// block index held by lane g after ginv (bit reversal of g, log2 G bits)
template <int G>
__device__ __forceinline__ int g_block(int g) {
  const int r3 = ((g & 1) << 2) | (g & 2) | ((g >> 2) & 1);
  return G == 8 ? r3 : ((r3 << 1) | ((g >> 3) & 1));
}

// Twiddles W_N^(g k), k = 1, 2, ...: float64 forms them by the recurrence
// w_k = w_(k-1) w_1 from one table entry (rounding grows by about one unit
// per step, far below float64 tolerances, and no table entries occupy
// registers); float32 reads each from the table.
template <typename T>
struct GTw {
  cpx<T> w1, w;
  const cpx<T>* __restrict__ tw;
  int g;
  __device__ __forceinline__ GTw(const cpx<T>* __restrict__ t, int gg) : tw(t), g(gg) {
    if constexpr (sizeof(T) == 8) { w1 = t[gg]; w = w1; }
  }
  __device__ __forceinline__ cpx<T> next(int k) {
    if constexpr (sizeof(T) == 8) {
      const cpx<T> r = w;
      w = cmul(w, w1);
      return r;
    } else {
      return tw[g * k];
    }
  }
};

// inverse direction (s = +1): lane g holds x[g + G j]  ->  X[k + LS p], p = g_block<G>(g).
// tw[m] = exp(+2 pi i m / N) in global memory (g k < N)
template <int G, int LS, typename T>
__device__ __forceinline__ void ginv(cpx<T> (&x)[LS], int g, const GLane<T>& l, const cpx<T>* __restrict__ tw) {
  const T s = T(1);
  RDft<LS, T>::run(x, s);
  GTw<T> t(tw, g);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    if (k != 0) x[k] = cmul(x[k], t.next(k));
    x[k] = g_dif<G>(x[k], l, s);
  }
}

// forward direction (s = -1): lane g holds y[k + LS p], p = g_block<G>(g)  ->  Y[g + G m]
template <int G, int LS, typename T>
__device__ __forceinline__ void gfwd(cpx<T> (&x)[LS], int g, const GLane<T>& l, const cpx<T>* __restrict__ tw) {
  const T s = T(-1);
  GTw<T> t(tw, g);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    x[k] = g_dit<G>(x[k], l, s);
    if (k != 0) {
      cpx<T> w = t.next(k);
      w.y = -w.y;
      x[k] = cmul(x[k], w);
    }
  }
  RDft<LS, T>::run(x, s);
}

}  // namespace regfft
