// Batched 1D complex FFTs inside one workgroup (LDS ping-pong, mixed radix
// 2/3/4/5/8, Stockham autosort).  Used by the three passes of the
// sphere <-> grid transform of H.psi.
//
// A length-L transform is a sequence of radix-R stages.  With Ns the product
// of the radices of the earlier stages, butterfly j (0 <= j < L/R) of a stage
// reads x_t = in[j + t L/R] (t < R), multiplies x_t by w^(t k L/(Ns R)) with
// k = j mod Ns and w = exp(s 2 pi i / L), takes an R-point DFT with sign s and
// writes y_q to out[(j / Ns) Ns R + k + q Ns].  After the last stage the
// result is in natural order, unscaled:  y_m = sum_j x_j exp(s 2 pi i j m / L).
//
// The first stage reads its inputs through a `load(b, i)` functor and the
// last stage writes through `store(b, i, v)`, so gathers, zero padding,
// pointwise products and scatters fuse into the transform.  Intermediate
// stages ping-pong between two LDS buffers p0 / p1 with `stride` elements per
// transform: stage s < nst-1 writes p0 when s is even, p1 when s is odd.
#pragma once
#include "common.h"

#define FFT_MAX_STAGES 8

struct FftDesc {
  int L;
  int nst;
  int radix[FFT_MAX_STAGES];
};

// Factor L into radices 8, 4, 5, 3, 2 (largest first).  Returns false if L
// has a prime factor above 5.
inline bool fft_factor(int L, FftDesc& d) {
  d.L = L;
  d.nst = 0;
  int m = L;
  const int pref[5] = {8, 4, 5, 3, 2};
  while (m > 1) {
    bool found = false;
    for (int r : pref) {
      if (m % r == 0) {
        if (d.nst >= FFT_MAX_STAGES) return false;
        d.radix[d.nst++] = r;
        m /= r;
        found = true;
        break;
      }
    }
    if (!found) return false;
  }
  if (d.nst == 0) {  // L == 1: a single trivial radix-1 stage is not supported
    return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// R-point DFT codelets, y_q = sum_t x_t exp(s 2 pi i t q / R), in place.
// ---------------------------------------------------------------------------
template <int R, typename T>
struct Dft;

template <typename T>
struct Dft<2, T> {
  static __device__ __forceinline__ void run(cpx<T>* x, T) {
    cpx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};

template <typename T>
struct Dft<3, T> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) {
    const T c = T(-0.5);
    const T sn = T(0.86602540378443864676) * s;  // sin(2 pi / 3)
    cpx<T> t1 = x[1] + x[2];
    cpx<T> t2 = x[0] + t1 * c;
    cpx<T> t3 = mul_is(x[1] - x[2], sn);
    x[0] = x[0] + t1;
    x[1] = t2 + t3;
    x[2] = t2 - t3;
  }
};

template <typename T>
struct Dft<4, T> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) {
    cpx<T> a = x[0] + x[2], b = x[0] - x[2];
    cpx<T> c = x[1] + x[3], d = mul_is(x[1] - x[3], s);
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + d;
    x[3] = b - d;
  }
};

template <typename T>
struct Dft<5, T> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) {
    const T c1 = T(0.30901699437494742410);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi/5)
    cpx<T> a1 = x[1] + x[4], b1 = x[1] - x[4];
    cpx<T> a2 = x[2] + x[3], b2 = x[2] - x[3];
    cpx<T> x0 = x[0];
    cpx<T> r1 = x0 + a1 * c1 + a2 * c2;
    cpx<T> r2 = x0 + a1 * c2 + a2 * c1;
    cpx<T> i1 = mul_is(b1 * s1 + b2 * s2, s);
    cpx<T> i2 = mul_is(b1 * s2 - b2 * s1, s);
    x[0] = x0 + a1 + a2;
    x[1] = r1 + i1;
    x[4] = r1 - i1;
    x[2] = r2 + i2;
    x[3] = r2 - i2;
  }
};

template <typename T>
struct Dft<8, T> {
  static __device__ __forceinline__ void run(cpx<T>* x, T s) {
    const T h = T(0.70710678118654752440);
    // DFT-4 of the even and of the odd samples
    cpx<T> e[4] = {x[0], x[2], x[4], x[6]};
    cpx<T> o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, T>::run(e, s);
    Dft<4, T>::run(o, s);
    // o_q *= exp(s 2 pi i q / 8)
    cpx<T> o1 = o[1], o3 = o[3];
    o[1] = mk<T>((o1.x - s * o1.y) * h, (o1.y + s * o1.x) * h);    // (1 + i s)/sqrt2
    o[2] = mul_is(o[2], s);                                          // i s
    o[3] = mk<T>((-o3.x - s * o3.y) * h, (-o3.y + s * o3.x) * h);  // (-1 + i s)/sqrt2
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = e[q] + o[q];
      x[q + 4] = e[q] - o[q];
    }
  }
};

// One Stockham stage over `nbatch` transforms.  `bfast` selects the task
// order: batch index fastest (coalesced access across transforms at fixed i)
// or butterfly index fastest (coalesced along a transform).
template <int R, typename T, class Load, class Store>
__device__ __forceinline__ void fft_stage(int L, int Ns, int nbatch, T s, const cpx<T>* tw,
                                          const cpx<T>* in, cpx<T>* out, int stride, bool first,
                                          bool last, bool bfast, Load& load, Store& store) {
  const int Lr = L / R;
  const int total = nbatch * Lr;
  const int tstep = L / (Ns * R);
  for (int task = threadIdx.x; task < total; task += blockDim.x) {
    int b, j;
    if (bfast) {
      b = task % nbatch;
      j = task / nbatch;
    } else {
      b = task / Lr;
      j = task - b * Lr;
    }
    const int k = j % Ns;
    cpx<T> x[R];
    if (first) {
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = load(b, j + t * Lr);
    } else {
      const cpx<T>* src = in + b * stride + j;
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] = src[t * Lr];
    }
    if (Ns > 1) {
#pragma unroll
      for (int t = 1; t < R; ++t) {
        cpx<T> w = tw[t * k * tstep];  // t k tstep < L
        w.y *= s;
        x[t] = cmul(x[t], w);
      }
    }
    Dft<R, T>::run(x, s);
    const int base = (j / Ns) * Ns * R + k;
    if (last) {
#pragma unroll
      for (int q = 0; q < R; ++q) store(b, base + q * Ns, x[q]);
    } else {
      cpx<T>* dst = out + b * stride + base;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q * Ns] = x[q];
    }
  }
}

// Full transform; ends with a __syncthreads().  `tw` holds exp(+2 pi i m / L),
// m < L (LDS or global); s = +1 (to real space) or -1 (to reciprocal space).
template <typename T, class Load, class Store>
__device__ void fft_run(const FftDesc& d, int nbatch, T s, const cpx<T>* tw, cpx<T>* p0,
                        cpx<T>* p1, int stride, bool bfast_first, bool bfast_last, Load load,
                        Store store) {
  int Ns = 1;
  for (int st = 0; st < d.nst; ++st) {
    const int R = d.radix[st];
    const bool first = (st == 0), last = (st == d.nst - 1);
    const cpx<T>* in = (st & 1) ? p0 : p1;
    cpx<T>* out = (st & 1) ? p1 : p0;
    const bool bfast = first ? bfast_first : (last ? bfast_last : false);
    switch (R) {
      case 2: fft_stage<2, T>(d.L, Ns, nbatch, s, tw, in, out, stride, first, last, bfast, load, store); break;
      case 3: fft_stage<3, T>(d.L, Ns, nbatch, s, tw, in, out, stride, first, last, bfast, load, store); break;
      case 4: fft_stage<4, T>(d.L, Ns, nbatch, s, tw, in, out, stride, first, last, bfast, load, store); break;
      case 5: fft_stage<5, T>(d.L, Ns, nbatch, s, tw, in, out, stride, first, last, bfast, load, store); break;
      default: fft_stage<8, T>(d.L, Ns, nbatch, s, tw, in, out, stride, first, last, bfast, load, store); break;
    }
    Ns *= R;
    __syncthreads();
  }
}

// Which ping-pong buffer the last stage reads (0 = p0, 1 = p1); a store
// functor that writes into LDS must target the other one (or any buffer when
// nst == 1).
__host__ __device__ inline int fft_last_read(const FftDesc& d) {
  return d.nst >= 2 ? ((d.nst - 2) & 1) : -1;
}
