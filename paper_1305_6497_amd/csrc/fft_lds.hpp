// Mixed-radix (2, 3, 4, 5, 8) complex FFT of a batch of pencils held in LDS.
//
// The 2/3/5-smooth lengths follow the guide's grid-extension rule (§13,
// "Choice of FFT Algorithm": GPFA needs extents of the form 2^i 3^j 5^k).
// The transform is a Stockham autosort FFT: every stage reads R inputs spaced
// L/R apart, multiplies by twiddles, does a radix-R DFT and writes the outputs
// to their sorted places, so no bit-reversal pass is needed.  A block of kNT
// threads works on `npen` pencils of length L stored in LDS at
// buf[p * ps + m * es]; each stage reads everything into registers, waits at a
// barrier, and writes back in place.
//
// EPT (elements per thread) bounds npen * L <= EPT * kNT and sizes the
// register arrays at compile time; every index into them is a compile-time
// constant so they stay in VGPRs.
#pragma once

#include "dda_internal.hpp"

namespace dda {

// multiply by DIR * i  (DIR = -1: forward transform, +1: inverse)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> z) {
  if (DIR < 0) return {z.y, -z.x};
  return {-z.y, z.x};
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cpx<T> *a) {
  if constexpr (R == 2) {
    cpx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  } else if constexpr (R == 3) {
    const T h = T(0.86602540378443864676);
    cpx<T> t = a[1] + a[2];
    cpx<T> d = mul_i<DIR>(h * (a[1] - a[2]));
    cpx<T> m = a[0] - T(0.5) * t;
    a[0] = a[0] + t;
    a[1] = m + d;
    a[2] = m - d;
  } else if constexpr (R == 4) {
    cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    cpx<T> t2 = a[1] + a[3], t3 = mul_i<DIR>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    cpx<T> t1 = a[1] + a[4], t2 = a[2] + a[3];
    cpx<T> d1 = a[1] - a[4], d2 = a[2] - a[3];
    cpx<T> m1 = a[0] + c1 * t1 + c2 * t2;
    cpx<T> m2 = a[0] + c2 * t1 + c1 * t2;
    cpx<T> n1 = mul_i<DIR>(s1 * d1 + s2 * d2);
    cpx<T> n2 = mul_i<DIR>(s2 * d1 - s1 * d2);
    a[0] = a[0] + t1 + t2;
    a[1] = m1 + n1;
    a[4] = m1 - n1;
    a[2] = m2 + n2;
    a[3] = m2 - n2;
  } else if constexpr (R == 8) {
    const T r = T(0.70710678118654752440);
    cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
    dft_small<4, DIR>(e);
    dft_small<4, DIR>(o);
    // w8^q for q = 1, 2, 3 with w8 = exp(DIR * 2 pi i / 8)
    cpx<T> o1 = r * (o[1] + mul_i<DIR>(o[1]));
    cpx<T> o2 = mul_i<DIR>(o[2]);
    cpx<T> o3 = r * (mul_i<DIR>(o[3]) - o[3]);
    a[0] = e[0] + o[0];
    a[4] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[5] = e[1] - o1;
    a[2] = e[2] + o2;
    a[6] = e[2] - o2;
    a[3] = e[3] + o3;
    a[7] = e[3] - o3;
  }
}

// One Stockham stage of radix R over npen pencils (see file comment).
template <typename T, int R, int EPT, int DIR>
__device__ __forceinline__ void fft_stage(cpx<T> *buf, const cpx<T> *tw, int L, int Ns, int npen,
                                          int ps, int es, bool pen_fastest) {
  constexpr int NB = (EPT + R - 1) / R;
  const int Lr = L / R;
  const int nbf = npen * Lr;
  const int tstride = L / (Ns * R);
  const int tid = threadIdx.x;
  cpx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * kNT;
    if (b < nbf) {
      int p, j;
      if (pen_fastest) { p = b % npen; j = b / npen; }
      else { j = b % Lr; p = b / Lr; }
      const cpx<T> *src = buf + p * ps + j * es;
#pragma unroll
      for (int k = 0; k < R; ++k) v[i][k] = src[k * Lr * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * kNT;
    if (b < nbf) {
      int p, j;
      if (pen_fastest) { p = b % npen; j = b / npen; }
      else { j = b % Lr; p = b / Lr; }
      const int jm = j % Ns;
      if (jm != 0) {
#pragma unroll
        for (int k = 1; k < R; ++k) {
          cpx<T> w = tw[jm * k * tstride];
          if (DIR > 0) w.y = -w.y;
          v[i][k] = v[i][k] * w;
        }
      }
      dft_small<R, DIR>(v[i]);
      cpx<T> *dst = buf + p * ps + ((j - jm) * R + jm) * es;
#pragma unroll
      for (int k = 0; k < R; ++k) dst[k * Ns * es] = v[i][k];
    }
  }
  __syncthreads();
}

// Full transform of npen pencils in LDS.  Data must be visible to all threads
// on entry (callers put a barrier after filling buf); on exit a barrier has
// been passed.
template <typename T, int EPT, int DIR>
__device__ __forceinline__ void fft_lds(cpx<T> *buf, const cpx<T> *tw, const AxisPlan &pl, int npen,
                                        int ps, int es, bool pen_fastest) {
  int Ns = 1;
  for (int s = 0; s < pl.nstages; ++s) {
    const int R = pl.radix[s];
    switch (R) {
      case 2: fft_stage<T, 2, EPT, DIR>(buf, tw, pl.L, Ns, npen, ps, es, pen_fastest); break;
      case 3: fft_stage<T, 3, EPT, DIR>(buf, tw, pl.L, Ns, npen, ps, es, pen_fastest); break;
      case 4: fft_stage<T, 4, EPT, DIR>(buf, tw, pl.L, Ns, npen, ps, es, pen_fastest); break;
      case 5: fft_stage<T, 5, EPT, DIR>(buf, tw, pl.L, Ns, npen, ps, es, pen_fastest); break;
      default: fft_stage<T, 8, EPT, DIR>(buf, tw, pl.L, Ns, npen, ps, es, pen_fastest); break;
    }
    Ns *= R;
  }
}

// Copy a twiddle table into LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T> *dst, const cpx<T> *src, int L) {
  for (int i = threadIdx.x; i < L; i += kNT) dst[i] = src[i];
}

}  // namespace dda
