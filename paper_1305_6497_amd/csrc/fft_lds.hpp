// Mixed-radix (2, 3, 4, 5, 8) complex FFT of a batch of pencils held in LDS.
//
// The 2/3/5-smooth lengths follow the guide's grid-extension rule (§13,
// "Choice of FFT Algorithm": GPFA needs extents of the form 2^i 3^j 5^k).
// The transform is a Stockham autosort FFT: every stage reads R inputs spaced
// L/R apart, multiplies by twiddles, does a radix-R DFT and writes the outputs
// to their sorted places, so no bit-reversal pass is needed.  Each stage reads
// everything into registers, waits at a barrier, and writes back in place.
//
// Two layouts of a batch of npen pencils in LDS:
//   pen   element m of pencil p at buf[m * NPEN + p], NPEN = 2^LOGP fixed at
//         compile time (the tiled y and z passes: pencils are the W lanes of
//         a 128-byte row);
//   rows  element m of pencil p at buf[p * L + m] (the x passes).
// The length is either a template constant LC (the whole plan, every stride
// and every quotient folds into immediates and shifts) or, with LC = 0, read
// from an AxisPlan whose per-stage strides and divisors were prepared on the
// host (no divide sequences in the kernels).
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

// exp(DIR * 2 pi i m / R) as compile-time constants.  cos and sin come from
// their Taylor series on [0, pi/4] after reducing m / R by the symmetries of
// the circle; the points on the axes and the diagonals are exact.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}

constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 12; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}

struct Root {
  double c, s;
};

// cos and sin of 2 pi m / R.  The angle is held as a = 8 m (units of
// 2 pi / (8 R)) and folded into [0, R] (an angle in [0, pi/4]) with integer
// arithmetic, so only the final series sees rounding.
constexpr Root unit_root(int m, int R) {
  m %= R;
  if (m < 0) m += R;
  long a = 8L * m;
  double ss = 1.0, sc = 1.0;
  if (a > 4L * R) { a = 8L * R - a; ss = -1.0; }       // theta -> 2 pi - theta
  if (a > 2L * R) { a = 4L * R - a; sc = -1.0; }       // theta -> pi - theta
  bool swap = false;
  if (a > R) { a = 2L * R - a; swap = true; }          // theta -> pi/2 - theta
  const double x = kPi * double(a) / (4.0 * R);
  double c = taylor_cos(x), s = taylor_sin(x);
  if (a == 0) { c = 1.0; s = 0.0; }
  if (a == R) { c = 0.70710678118654752440; s = c; }
  if (swap) { const double t = c; c = s; s = t; }
  return {sc * c, ss * s};
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cpx<T> *a);

// v * exp(DIR * 2 pi i M / R), with the trivial rotations done without multiplies
template <int R, int M, int DIR, typename T>
__device__ __forceinline__ cpx<T> rotate(cpx<T> v) {
  constexpr int m = M % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (2 * m == R) {
    return {-v.x, -v.y};
  } else if constexpr (4 * m == R) {
    return DIR < 0 ? cpx<T>{v.y, -v.x} : cpx<T>{-v.y, v.x};
  } else if constexpr (4 * m == 3 * R) {
    return DIR < 0 ? cpx<T>{-v.y, v.x} : cpx<T>{v.y, -v.x};
  } else {
    constexpr Root w = unit_root(m, R);
    const T c = T(w.c), sn = T(DIR * w.s);
    return {v.x * c - v.y * sn, v.x * sn + v.y * c};
  }
}

// y[n1][k2] *= exp(DIR * 2 pi i n1 k2 / R) for n1 >= N1, k2 >= K2
template <int R, int A, int B, int DIR, int N1, int K2, typename T>
__device__ __forceinline__ void rotate_all(cpx<T> (&y)[A][B]) {
  if constexpr (N1 < A) {
    if constexpr (K2 < B) {
      y[N1][K2] = rotate<R, N1 * K2, DIR>(y[N1][K2]);
      rotate_all<R, A, B, DIR, N1, K2 + 1>(y);
    } else {
      rotate_all<R, A, B, DIR, N1 + 1, 1>(y);
    }
  }
}

// DFT of size R = A * B in registers (Cooley-Tukey): with n = n1 + A n2 and
// k = B k1 + k2, X[B k1 + k2] = sum_n1 w_A^(n1 k1) w_R^(n1 k2) Y[n1][k2], where
// Y[n1] is the size-B DFT of x[n1 + A n2] over n2.
template <int A, int B, int DIR, typename T>
__device__ __forceinline__ void dft_composite(cpx<T> *a) {
  constexpr int R = A * B;
  cpx<T> y[A][B];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) y[n1][n2] = a[n1 + A * n2];
    dft_small<B, DIR>(y[n1]);
  }
  rotate_all<R, A, B, DIR, 1, 1>(y);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    cpx<T> z[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) z[n1] = y[n1][k2];
    dft_small<A, DIR>(z);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) a[B * k1 + k2] = z[k1];
  }
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
  } else if constexpr (R == 6) {
    dft_composite<2, 3, DIR>(a);
  } else if constexpr (R == 9) {
    dft_composite<3, 3, DIR>(a);
  } else if constexpr (R == 10) {
    dft_composite<2, 5, DIR>(a);
  } else if constexpr (R == 12) {
    dft_composite<4, 3, DIR>(a);
  } else if constexpr (R == 15) {
    dft_composite<3, 5, DIR>(a);
  } else if constexpr (R == 16) {
    dft_composite<4, 4, DIR>(a);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// v * w for the forward transform, v * conj(w) for the inverse: the table
// holds exp(-2 pi i n / L), and the conjugate costs nothing extra.
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> twmul(cpx<T> v, cpx<T> w) {
  if (DIR < 0) return {v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
  return {v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
}

// Division by a compile-time constant (strength-reduced by the compiler).
template <int N>
struct ConstDiv {
  __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return x / N; }
};

__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

// Pen layout, one stage.  Butterfly b = j * NPEN + p reads buf[b + k * nbf],
// nbf = (L / R) * NPEN; with j = q * Ns + jm its outputs go to
// buf[b + q * Ns (R - 1) NPEN + k * Ns NPEN], which is the Stockham position
// ((j - jm) R + jm + k Ns) * NPEN + p.  pen_butterfly does the twiddles, the
// DFT and hands each output and its position to `put`.
template <typename T, int R, int DIR, int LOGP, typename DN, typename Put>
__device__ __forceinline__ void pen_butterfly(cpx<T> (&v)[R], int b, const cpx<T> *tw, int Ns, int twstep, DN nsd,
                                              Put &&put) {
  const int j = b >> LOGP;
  const int q = (int)nsd((uint32_t)j);
  if (Ns > 1) {
    const int st = mul24(j - mul24(q, Ns), twstep);
    int ti = st;
#pragma unroll
    for (int k = 1; k < R; ++k) {
      v[k] = twmul<DIR>(v[k], tw[ti]);
      ti += st;
    }
  }
  dft_small<R, DIR>(v);
  const int o = b + (mul24(q, mul24(Ns, R - 1)) << LOGP);
  const int ostr = Ns << LOGP;
#pragma unroll
  for (int k = 0; k < R; ++k) put(o + k * ostr, v[k]);
}

template <typename T, int R, int NB, int DIR, int LOGP, typename DN>
__device__ __forceinline__ void stage_pen(cpx<T> *buf, const cpx<T> *tw, int lr, int Ns, int twstep, DN nsd) {
  const int nbf = lr << LOGP;
  cpx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < nbf) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[i][k] = buf[b + k * nbf];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < nbf) pen_butterfly<T, R, DIR, LOGP>(v[i], b, tw, Ns, twstep, nsd, [&](int o, cpx<T> x) { buf[o] = x; });
  }
  __syncthreads();
}

// Rows layout, one stage.  Butterfly b = p * (L / R) + j reads
// buf[p L + j + k L / R] and writes buf[p L + (j - jm) R + jm + k Ns].
template <typename T, int R, int NB, int DIR, typename DL, typename DN>
__device__ __forceinline__ void stage_rows(cpx<T> *buf, const cpx<T> *tw, int L, int lr, int Ns, int twstep, DL lrd,
                                           DN nsd, int npen) {
  const int nbf = mul24(npen, lr);
  const int gap = L - lr;
  const int jump = mul24(Ns, R - 1);
  cpx<T> v[NB][R];
  int base[NB], jj[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < nbf) {
      const int p = (int)lrd((uint32_t)b);
      jj[i] = b - mul24(p, lr);
      base[i] = b + mul24(p, gap);
#pragma unroll
      for (int k = 0; k < R; ++k) v[i][k] = buf[base[i] + k * lr];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < nbf) {
      const int q = (int)nsd((uint32_t)jj[i]);
      if (Ns > 1) {
        const int st = mul24(jj[i] - mul24(q, Ns), twstep);
        int ti = st;
#pragma unroll
        for (int k = 1; k < R; ++k) {
          v[i][k] = twmul<DIR>(v[i][k], tw[ti]);
          ti += st;
        }
      }
      dft_small<R, DIR>(v[i]);
      cpx<T> *dst = buf + base[i] + mul24(q, jump);
#pragma unroll
      for (int k = 0; k < R; ++k) dst[k * Ns] = v[i][k];
    }
  }
  __syncthreads();
}

// The plan of a compile-time length.  Besides the radices of the run-time plan
// it may use the composite radices 6, 9, 10, 12, 15 and 16 (up to rmax): the
// plan with the fewest stages (each stage is one LDS round trip and two
// barriers) and, among those, the fewest flops, largest radix first (the
// first stage needs no twiddles).
struct StaticPlan {
  int n;
  int radix[kMaxStages];
  int ns[kMaxStages];
  double cost;
};

// real flops per element of a radix-R DFT, and of its R - 1 twiddle products
constexpr double radix_flops(int R) {
  switch (R) {
    case 2: return 2.0;
    case 3: return 5.3;
    case 4: return 4.0;
    case 5: return 8.8;
    case 6: return 9.3;
    case 8: return 7.0;
    case 9: return 13.3;
    case 10: return 12.4;
    case 12: return 12.3;
    case 15: return 17.3;
    default: return 10.9;     // 16
  }
}

constexpr StaticPlan search_plan(int L, int rmax) {
  StaticPlan best{};
  best.cost = 1e30;
  if (L == 1) {
    best.cost = 0.0;
    return best;
  }
  const int set[11] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  for (int i = 0; i < 11; ++i) {
    const int R = set[i];
    if (R > rmax || L % R != 0) continue;
    StaticPlan c = search_plan(L / R, rmax);
    if (c.cost >= 1e29 || c.n + 1 > kMaxStages) continue;
    c.radix[c.n++] = R;
    c.cost += radix_flops(R) + 6.0 * (R - 1) / R;
    if (best.cost >= 1e29 || c.n < best.n || (c.n == best.n && c.cost < best.cost)) best = c;
  }
  return best;
}

constexpr StaticPlan static_plan(int L, int rmax = 8) {
  StaticPlan p = search_plan(L, rmax);
  for (int i = 0; i < p.n; ++i)             // largest radix first
    for (int j = i + 1; j < p.n; ++j)
      if (p.radix[j] > p.radix[i]) {
        const int t = p.radix[i];
        p.radix[i] = p.radix[j];
        p.radix[j] = t;
      }
  int ns = 1;
  for (int i = 0; i < p.n; ++i) {
    p.ns[i] = ns;
    ns *= p.radix[i];
  }
  return p;
}

// The cheapest plan (by the cost model) with exactly n stages.
constexpr StaticPlan search_plan_n(int L, int rmax, int n) {
  StaticPlan best{};
  best.cost = 1e30;
  if (n == 0) {
    if (L == 1) best.cost = 0.0;
    return best;
  }
  const int set[11] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  for (int i = 0; i < 11; ++i) {
    const int R = set[i];
    if (R > rmax || L % R != 0) continue;
    StaticPlan c = search_plan_n(L / R, rmax, n - 1);
    if (c.cost >= 1e29) continue;
    c.radix[c.n++] = R;
    c.cost += radix_flops(R) + 6.0 * (R - 1) / R;
    if (c.cost < best.cost) best = c;
  }
  return best;
}

// Radices sorted (largest first, or smallest first) and their Ns filled in.
constexpr StaticPlan order_plan(StaticPlan p, bool largest_first) {
  for (int i = 0; i < p.n; ++i)
    for (int j = i + 1; j < p.n; ++j)
      if (largest_first ? p.radix[j] > p.radix[i] : p.radix[j] < p.radix[i]) {
        const int t = p.radix[i];
        p.radix[i] = p.radix[j];
        p.radix[j] = t;
      }
  int ns = 1;
  for (int i = 0; i < p.n; ++i) {
    p.ns[i] = ns;
    ns *= p.radix[i];
  }
  return p;
}

// Alternative plans of one length, for the plan autotuner:
//   0  the cost model's plan (static_plan with the caller's radix bound:
//      fewest stages, then fewest flops, largest radix first),
//   1  the same with radices up to 16 whatever the bound (fewer LDS stages
//      at the price of idle threads in the large-radix stages),
//   2  the cheapest plan with one stage more than 0 (smaller radices, fewer
//      registers per butterfly), largest radix first,
//   3  the radices of 0, smallest first.
// Variant 2 falls back to 0 where no such plan exists.
constexpr int kPlanVariants = 4;

constexpr StaticPlan plan_variant(int L, int rmax, int V) {
  const StaticPlan p0 = search_plan(L, rmax);
  if (V == 1) return order_plan(search_plan(L, 16), true);
  if (V == 2) {
    const StaticPlan p2 = p0.n + 1 <= kMaxStages ? search_plan_n(L, rmax, p0.n + 1) : p0;
    return order_plan(p2.cost < 1e29 ? p2 : p0, true);
  }
  return order_plan(p0, V != 3);
}

// Largest radix of a pen plan over 2^LOGP pencils: a radix-R stage keeps
// L NPEN / R butterflies, and at least half the threads should get one.
constexpr int pen_rmax(int L, int LOGP) {
  const int r = 2 * (L << LOGP) / kNT;
  return r < 8 ? 8 : (r > 16 ? 16 : r);
}

constexpr int cdiv_c(int a, int b) { return (a + b - 1) / b; }

template <typename T, int DIR, int LOGP, int L, int S, int SEND = 64, int V = 0>
__device__ __forceinline__ void fft_pen_c(cpx<T> *buf, const cpx<T> *tw) {
  constexpr StaticPlan P = plan_variant(L, pen_rmax(L, LOGP), V);
  if constexpr (S < P.n && S < SEND) {
    constexpr int R = P.radix[S], Ns = P.ns[S];
    constexpr int NB = cdiv_c((L / R) << LOGP, kNT);
    stage_pen<T, R, NB, DIR, LOGP>(buf, tw, L / R, Ns, L / (Ns * R), ConstDiv<Ns>{});
    fft_pen_c<T, DIR, LOGP, L, S + 1, SEND, V>(buf, tw);
  }
}

// First and last stage of a compile-time pen plan, for transforms whose input
// comes from (or whose output goes to) global memory directly.
template <int L, int LOGP, int V = 0>
struct PenEnds {
  static constexpr StaticPlan P = plan_variant(L, pen_rmax(L, LOGP), V);
  static constexpr int R0 = P.radix[0];                  // first stage
  static constexpr int NBF0 = (L / R0) << LOGP;          // its butterflies
  static constexpr int NB0 = cdiv_c(NBF0, kNT);          // ... per thread
  static constexpr int RL = P.radix[P.n - 1];            // last stage
  static constexpr int NBFL = (L / RL) << LOGP;
  static constexpr int NBL = cdiv_c(NBFL, kNT);
};

// Pen transform whose first-stage inputs are already in registers:
// v[i][k] = element b + k * NBF0 of the buffer for butterfly b = tid + i kNT.
// buf must be free on entry (no thread still reading it); on exit the result
// is in buf and a barrier has been passed.
template <typename T, int DIR, int LOGP, int L, int V = 0>
__device__ __forceinline__ void fft_pen_from_regs(cpx<T> *buf, const cpx<T> *tw,
                                                  cpx<T> (&v)[PenEnds<L, LOGP, V>::NB0][PenEnds<L, LOGP, V>::R0]) {
  using E = PenEnds<L, LOGP, V>;
#pragma unroll
  for (int i = 0; i < E::NB0; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < E::NBF0)
      pen_butterfly<T, E::R0, DIR, LOGP>(v[i], b, tw, 1, 0, ConstDiv<1>{}, [&](int o, cpx<T> x) { buf[o] = x; });
  }
  __syncthreads();
  fft_pen_c<T, DIR, LOGP, L, 1, 64, V>(buf, tw);
}

// Pen transform of buf whose last-stage outputs go to put(e, value), e the
// element index in the pen layout, instead of back to LDS.  Data must be
// visible to all threads on entry; no barrier follows the last stage, so the
// caller synchronises before writing buf again.
template <typename T, int DIR, int LOGP, int L, int V = 0, typename Put>
__device__ __forceinline__ void fft_pen_to_store(cpx<T> *buf, const cpx<T> *tw, Put &&put) {
  using E = PenEnds<L, LOGP, V>;
  constexpr int S = E::P.n - 1, R = E::RL, Ns = E::P.ns[S];
  fft_pen_c<T, DIR, LOGP, L, 0, S, V>(buf, tw);
  cpx<T> v[E::NBL][R];
#pragma unroll
  for (int i = 0; i < E::NBL; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < E::NBFL) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[i][k] = buf[b + k * E::NBFL];
    }
  }
#pragma unroll
  for (int i = 0; i < E::NBL; ++i) {
    const int b = threadIdx.x + i * kNT;
    if (b < E::NBFL) pen_butterfly<T, R, DIR, LOGP>(v[i], b, tw, Ns, L / (Ns * R), ConstDiv<Ns>{}, put);
  }
}

template <typename T, int EPT, int DIR, int LOGP>
__device__ __forceinline__ void fft_pen_rt(cpx<T> *buf, const cpx<T> *tw, const AxisPlan &pl) {
  for (int s = 0; s < pl.nstages; ++s) {
    const int lr = pl.lr[s], Ns = pl.ns[s], ts = pl.twstep[s];
    const FastDiv d = pl.ns_div[s];
    switch (pl.radix[s]) {
      case 2: stage_pen<T, 2, cdiv_c(EPT, 2), DIR, LOGP>(buf, tw, lr, Ns, ts, d); break;
      case 3: stage_pen<T, 3, cdiv_c(EPT, 3), DIR, LOGP>(buf, tw, lr, Ns, ts, d); break;
      case 4: stage_pen<T, 4, cdiv_c(EPT, 4), DIR, LOGP>(buf, tw, lr, Ns, ts, d); break;
      case 5: stage_pen<T, 5, cdiv_c(EPT, 5), DIR, LOGP>(buf, tw, lr, Ns, ts, d); break;
      default: stage_pen<T, 8, cdiv_c(EPT, 8), DIR, LOGP>(buf, tw, lr, Ns, ts, d); break;
    }
  }
}

// Transform the 2^LOGP interleaved pencils in buf (pen layout).  LC > 0: the
// length is LC and `pl` is not read.  Data must be visible to all threads on
// entry (callers put a barrier after filling buf); on exit a barrier has been
// passed.
template <typename T, int EPT, int DIR, int LOGP, int LC>
__device__ __forceinline__ void fft_pen(cpx<T> *buf, const cpx<T> *tw, const AxisPlan &pl) {
  if constexpr (LC > 0) fft_pen_c<T, DIR, LOGP, LC, 0>(buf, tw);
  else fft_pen_rt<T, EPT, DIR, LOGP>(buf, tw, pl);
}

// Plans of the rows layout (the x passes): 0 radices up to 8 (the cost
// model's bound for contiguous rows), 1 radices up to 16 (fewer LDS stages).
constexpr int kRowPlanVariants = 2;
static_assert(kRowPlanVariants == kRowPlanVariantsHost, "rows plan variant count");

constexpr StaticPlan rows_plan(int L, int V) { return static_plan(L, V == 1 ? 16 : 8); }

template <typename T, int EPT, int DIR, int L, int S, int V = 0>
__device__ __forceinline__ void fft_rows_c(cpx<T> *buf, const cpx<T> *tw, int npen) {
  constexpr StaticPlan P = rows_plan(L, V);
  if constexpr (S < P.n) {
    constexpr int R = P.radix[S], Ns = P.ns[S];
    stage_rows<T, R, cdiv_c(EPT, R), DIR>(buf, tw, L, L / R, Ns, L / (Ns * R), ConstDiv<L / R>{}, ConstDiv<Ns>{},
                                          npen);
    fft_rows_c<T, EPT, DIR, L, S + 1, V>(buf, tw, npen);
  }
}

template <typename T, int EPT, int DIR>
__device__ __forceinline__ void fft_rows_rt(cpx<T> *buf, const cpx<T> *tw, const AxisPlan &pl, int npen) {
  const int L = pl.L;
  for (int s = 0; s < pl.nstages; ++s) {
    const int lr = pl.lr[s], Ns = pl.ns[s], ts = pl.twstep[s];
    const FastDiv dl = pl.lr_div[s], dn = pl.ns_div[s];
    switch (pl.radix[s]) {
      case 2: stage_rows<T, 2, cdiv_c(EPT, 2), DIR>(buf, tw, L, lr, Ns, ts, dl, dn, npen); break;
      case 3: stage_rows<T, 3, cdiv_c(EPT, 3), DIR>(buf, tw, L, lr, Ns, ts, dl, dn, npen); break;
      case 4: stage_rows<T, 4, cdiv_c(EPT, 4), DIR>(buf, tw, L, lr, Ns, ts, dl, dn, npen); break;
      case 5: stage_rows<T, 5, cdiv_c(EPT, 5), DIR>(buf, tw, L, lr, Ns, ts, dl, dn, npen); break;
      default: stage_rows<T, 8, cdiv_c(EPT, 8), DIR>(buf, tw, L, lr, Ns, ts, dl, dn, npen); break;
    }
  }
}

// Transform npen contiguous pencils in buf (rows layout); npen * L <= EPT * kNT.
template <typename T, int EPT, int DIR, int LC, int V = 0>
__device__ __forceinline__ void fft_rows(cpx<T> *buf, const cpx<T> *tw, const AxisPlan &pl, int npen) {
  if constexpr (LC > 0) fft_rows_c<T, EPT, DIR, LC, 0, V>(buf, tw, npen);
  else fft_rows_rt<T, EPT, DIR>(buf, tw, pl, npen);
}

// Copy a twiddle table into LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T> *dst, const cpx<T> *src, int L) {
  for (int i = threadIdx.x; i < L; i += kNT) dst[i] = src[i];
}

// A twiddle table copied into LDS in two steps: issue() starts the loads into
// registers and commit() writes them to LDS, so a pass that issues its data
// loads in between waits for one round trip to memory instead of two.  With a
// compile-time length the loads are unconditional (indices past the table
// are clamped, their values dropped), which lets the compiler count them
// exactly.  FP64 tables (and run-time lengths) are copied by issue() at once:
// staged, the FP64 x-inverse was measured slower.
template <typename T, int LC>
struct TwiddleStage {
  static constexpr bool kStaged = LC > 0 && sizeof(T) == 4;
  static constexpr int N = kStaged ? cdiv_c(LC, kNT) : 1;
  cpx<T> v[N];
  __device__ __forceinline__ void issue(cpx<T> *dst, const cpx<T> *src, int len) {
    if constexpr (kStaged) {
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] = src[min((int)threadIdx.x + k * kNT, LC - 1)];
    } else {
      load_twiddles(dst, src, len);
    }
  }
  __device__ __forceinline__ void commit(cpx<T> *dst) const {
    if constexpr (kStaged) {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int i = threadIdx.x + k * kNT;
        if (i < LC) dst[i] = v[k];
      }
    }
  }
};

}  // namespace dda
