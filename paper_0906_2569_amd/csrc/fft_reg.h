// Register-resident 1D transforms of length L = 4 * LS, one quad of lanes per
// transform.  Each lane keeps LS complex values in VGPRs; the transform is a
// per-lane LS-point DFT (compile-time mixed radix 2/3/4/5, fully unrolled),
// a twiddle, and a 4-point DFT across the quad through DPP quad permutes.
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
// Twiddles come from a table tw[m] = exp(+2 pi i m / L), m < L (LDS).
#pragma once
#include "fft.h"

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

// In-place N-point DFT of x[0..N) in registers, X_k = sum_n x_n W^(s n k),
// W = exp(2 pi i / N); W_N^j is tw[j * tstep].
template <int N, typename T, int F = SmallFactor<N>::value>
struct RDft {
  static __device__ __forceinline__ void run(cpx<T>* x, T s, const cpx<T>* tw, int tstep) {
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
        if ((n2 * k1) % N != 0) v = cmul(v, twid(tw, ((n2 * k1) % N) * tstep, s));
        a[n2 * N1 + k1] = v;
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      cpx<T> t[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) t[n2] = a[n2 * N1 + k1];
      RDft<N2, T>::run(t, s, tw, tstep * N1);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) x[k1 + N1 * k2] = t[k2];
    }
  }
};

template <int N, typename T>
struct RDft<N, T, N> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s, const cpx<T>*, int) { Dft<N, T>::run(x, s); }
};

template <typename T>
struct RDft<1, T, 1> {
  static __device__ __forceinline__ void run(cpx<T>*, T, const cpx<T>*, int) {}
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
// exchanges with one partner lane (DPP) and forms partner + sgn * self.
template <int D, typename T>
__device__ __forceinline__ cpx<T> bfly(cpx<T> self, bool upper) {
  const cpx<T> o = qxc<D>(self);
  return upper ? cpx<T>{o.x - self.x, o.y - self.y} : cpx<T>{o.x + self.x, o.y + self.y};
}

// block index held by lane q after inv_dit (bit-reversed 2-bit lane index)
__device__ __forceinline__ int quad_block(int q) { return ((q & 1) << 1) | (q >> 1); }

// lane q holds b_q; returns X_p = sum_q b_q W_4^(s q p) for p = quad_block(q)
template <typename T>
__device__ __forceinline__ cpx<T> quad_dit(cpx<T> b, int q, T s) {
  const bool q0 = q & 1, q1 = q & 2;
  b = bfly<2>(b, q1);                        // sum over q1: (-1)^(q1 p0), p0 = q1
  if (q0 && q1) b = mul_is(b, s);            // W_4^(s q0 p0)
  return bfly<1>(b, q0);                     // sum over q0: (-1)^(q0 p1), p1 = q0
}

// lane q holds y_p for p = quad_block(q); returns B_q = sum_p y_p W_4^(s p q)
template <typename T>
__device__ __forceinline__ cpx<T> quad_dif(cpx<T> y, int q, T s) {
  const bool q0 = q & 1, q1 = q & 2;
  y = bfly<1>(y, q0);                        // sum over p1 = q0: (-1)^(p1 q'0)
  if (q0 && q1) y = mul_is(y, s);            // W_4^(s p0 q'0)
  return bfly<2>(y, q1);                     // sum over p0 = q1: (-1)^(p0 q'1)
}

// inverse direction (s = +1): lane q holds x[q + 4 j]  ->  X[k + LS p], p = quad_block(q)
template <int LS, typename T>
__device__ __forceinline__ void inv_dit(cpx<T> (&x)[LS], int q, const cpx<T>* tw) {
  const T s = T(1);
  RDft<LS, T>::run(x, s, tw, 4);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    if (k != 0) x[k] = cmul(x[k], twid(tw, q * k, s));   // q k < 4 LS
    x[k] = quad_dit(x[k], q, s);
  }
}

// forward direction (s = -1): lane q holds y[k + LS p], p = quad_block(q)  ->  Y[q + 4 m]
template <int LS, typename T>
__device__ __forceinline__ void fwd_dif(cpx<T> (&x)[LS], int q, const cpx<T>* tw) {
  const T s = T(-1);
#pragma unroll
  for (int k = 0; k < LS; ++k) {
    x[k] = quad_dif(x[k], q, s);
    if (k != 0) x[k] = cmul(x[k], twid(tw, q * k, s));
  }
  RDft<LS, T>::run(x, s, tw, 4);
}

}  // namespace regfft
