// The FFT convolution A P of the DDA (Goodman, Draine & Flatau 1990, cited in
// §1 and §13 of the DDSCAT 7.3 guide) as five LDS-tiled passes on gfx950:
//
//   x-forward   sites -> A      gather P through the cell->site map, zero-pad
//                               x to Mx, FFT along x             (ny*nz pencils)
//   y-forward   A -> B          zero-pad y to My, FFT along y    (Mx*nz pencils)
//   z-pass      B -> B          zero-pad z to Mz, FFT along z, 3x3 complex-
//                               symmetric product with the Green transform,
//                               inverse FFT along z, keep nz     (Mx*My pencils)
//   y-inverse   B -> A          inverse FFT along y, keep ny     (Mx*nz pencils)
//   x-inverse   A -> sites      inverse FFT along x, keep nx, subtract from
//                               the diagonal term ainv * P       (ny*nz pencils)
//
// Zero padding is never materialised: a pass only reads the rows that hold
// data and only writes the rows the next pass needs (pruned transforms).
// The tiled layouts of A and B (see Geometry) make every global access a run
// of W = 128 bytes / sizeof(complex) consecutive elements.
// The Green transform is stored for one octant of frequencies: each tensor
// component is even or odd in each lattice offset, so its transform has the
// same parity and the other seven octants follow by sign flips.

// Kernel templates and the launcher template; instantiated once per precision
// (matvec_f32.hip, matvec_f64.hip) so the two compile in parallel.
#pragma once

#include <algorithm>
#include <climits>
#include <type_traits>

#include "dda_internal.hpp"
#include "fft_lds.hpp"
#include "reduce.hpp"

namespace dda {


extern __shared__ __align__(16) unsigned char dda_smem[];

template <typename T>
__device__ __forceinline__ cpx<T> to_t(c64 v) { return {T(v.x), T(v.y)}; }

// Tile width in x of the intermediate layouts: 128 bytes of complex values.
template <typename T>
constexpr int kW = 128 / (int)sizeof(cpx<T>);
template <typename T>
constexpr int kLogW = sizeof(T) == 4 ? 4 : 3;

// Sizes of the passes with their divisors prepared on the host.
struct PassDims {
  int nx, ny, nz;
  int Mx, My;
  int nxt;                        // x tiles of W
  int nrows;                      // rows per block of the x passes
  int Mxh, Myh;                   // octant extents M/2 + 1 (Green table)
  int nrhs;                       // right-hand sides of the launch
  FastDiv d_mx, d_nx, d_ny, d_nxt, d_nrows, d_nrhs;
};

// Fill LDS from global memory: every global load of a thread is issued before
// any LDS write, so each thread keeps up to EPT loads in flight.
template <typename T, int EPT, typename F>
__device__ __forceinline__ void stage_in(cpx<T> *buf, int n, F &&load) {
  cpx<T> v[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) v[i] = load(e);
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) buf[e] = v[i];
  }
}

// Offsets in A of the rows (component c, row q) of an x-pass block, or -1 for
// rows past the end: rowoff[c * nrows + q] = ((c nz + z) nxt ny + y) W.
template <typename T, int LC>
__device__ __forceinline__ void x_row_offsets(int *rowoff, const PassDims &d, int nrows, int row0, int nrow) {
  constexpr int W = kW<T>;
  for (int pq = threadIdx.x; pq < 3 * nrows; pq += kNT) {
    const int c = LC > 0 ? pq / nrows : (int)d.d_nrows((uint32_t)pq);
    const int q = pq - c * nrows;
    int off = -1;
    if (q < nrow) {
      const int row = row0 + q;
      const int z = (int)d.d_ny((uint32_t)row), y = row - z * d.ny;
      off = ((c * d.nz + z) * d.nxt * d.ny + y) * W;
    }
    rowoff[pq] = off;
  }
}

// Rows of an x-pass block when the sites are numbered row after row
// (MatvecArgs::rowtab): the block's sites are then one contiguous range of P,
// read and written as one run of 3 * count complex values.
template <int NR>
struct RowRuns {
  // Per-row values are combined with arithmetic masks, not selected by row
  // index: a select between array elements becomes an indexed load, which
  // would put the arrays in scratch memory.
  int first, count;               // first site of the block, number of sites
  int s0[NR];                     // block-relative first site (INT_MAX past the block)
  int step[NR];                   // change of (LDS position - site) from row q-1 to q
  int lo[NR], len[NR];            // first x and count of row q
  // t: the block's row-table entries (4 ints per row, from global memory or LDS)
  __device__ __forceinline__ RowRuns(const int *t, int nrow, int L) {
    first = t[0];
    count = 0;
    int prev = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      int s = INT_MAX, x0 = 0, n = 0;
      if (q < nrow) {
        s = t[4 * q] - first;
        x0 = t[4 * q + 1];
        n = t[4 * q + 2];
      }
      const int base = q < nrow ? q * L + x0 - s : prev;   // LDS position of site s: base + s
      s0[q] = s;
      step[q] = base - prev;
      prev = base;
      lo[q] = x0;
      len[q] = n;
      count += n;
    }
  }
  // LDS position q * L + x of the block-relative site s (the first sites never
  // decrease, so the steps of rows q with s0[q] <= s add up to row q's offset)
  __device__ __forceinline__ int pos(int s) const {
    int b = step[0];
#pragma unroll
    for (int q = 1; q < NR; ++q) b += int(s0[q] <= s) * step[q];
    return b + s;
  }
  // whether position x of row q holds a site
  __device__ __forceinline__ bool holds(int q, int x) const {
    int l = 0, n = 0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int m = int(q == k);
      l += m * lo[k];
      n += m * len[k];
    }
    return unsigned(x - l) < unsigned(n);
  }
};

// Element-wise work on a run of n values, element e = threadIdx.x + i kNT:
// every load is issued before the first store.
template <int EPT, typename VT>
__device__ __forceinline__ void runs_load(c64 (&v)[EPT], int n, const VT *src) {
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) v[i] = vld(src + e);
  }
}

// v = d = a + c b (each vector c64 or c32)
template <int EPT, typename TA, typename TB, typename VT>
__device__ __forceinline__ void runs_axpy(c64 (&v)[EPT], int n, const TA *a, const TB *b, VT *d, c64 c) {
  c64 bv[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) {
      v[i] = vld(a + e);
      bv[i] = vld(b + e);
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) {
      v[i] = vround<VT>(v[i] + c * bv[i]);
      vst(d + e, v[i]);
    }
  }
}

// v = p = r + beta (p - omega w)
template <int EPT, typename VT, typename VW>
__device__ __forceinline__ void runs_p(c64 (&v)[EPT], int n, const c64 *r, VT *p, const VW *w, c64 beta,
                                       c64 omega) {
  c64 pv[EPT], wv[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) {
      v[i] = r[e];
      pv[i] = vld(p + e);
      wv[i] = vld(w + e);
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) {
      v[i] = vround<VT>(v[i] + beta * (pv[i] - omega * wv[i]));
      vst(p + e, v[i]);
    }
  }
}

// BiCGSTAB alpha = rho / <rh, v> from the records of the product that made v.
// Every block computes the same sum in the same order, so all agree; block 0
// stores alpha, or flags the breakdown.  Returns false on breakdown.
__device__ __forceinline__ bool block_alpha(const FuseArgs &f, int r, c64 &alpha) {
  __shared__ c64 s_alpha;
  __shared__ int s_ok;
  double s[2];
  sum_records<2, kNT>(f.partial, f.nrec, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = f.scal + (size_t)r * kScal;
    const c64 den = {s[0], s[1]};
    const bool ok = cabs2(den) > 1e-60 * sc[S_RH2].x * sc[S_RNORM2].x && cabs2(den) > 0.0;
    const c64 a = ok ? cdiv(sc[S_RHO], den) : c64{0, 0};
    s_alpha = a;
    s_ok = ok ? 1 : 0;
    if (blockIdx.x == 0) {
      if (ok) {
        sc[S_ALPHA] = a;
      } else {
        f.active[r] = 0;
        f.status[r] = ST_BREAK;
      }
    }
  }
  __syncthreads();
  alpha = s_alpha;
  return s_ok != 0;
}

// --------------------------------------------------------------- x-forward --
// f.in_mode (see FuseArgs): 0 transforms `in`; 1 and 2 first form the BiCGSTAB
// vector p or s from r, v (and the old p) and store it, so the vector update
// costs no pass of its own.  LC > 0: Mx = LC, known at compile time.
template <typename T, int EPT, int LC, int V, typename VT, typename VV>
__global__ __launch_bounds__(kNT) void k_xfwd(const VT *__restrict__ in, int64_t n3, const int *__restrict__ mask,
                                               const int *__restrict__ cell_site, const int4 *__restrict__ rowtab,
                                               Scaling sc, cpx<T> *__restrict__ A,
                                               size_t a_elems, const cpx<T> *__restrict__ twx, AxisPlan px,
                                               PassDims d, FuseArgs f) {
  constexpr int W = kW<T>, LOGW = kLogW<T>;
  constexpr int NE = (EPT + 2) / 3;      // nrows * Mx <= EPT * kNT / 3
  // VT: the type of in (and of w, the vector an update writes); VV: of v.
  // FP32 vectors (COCG's p; BiCGSTAB's p and v) are never part of an update
  // list longer than one (BiCGstab(2)); r is always FP64
  constexpr bool V64 = sizeof(VT) == sizeof(c64) && sizeof(VV) == sizeof(c64);
  VT *uw = reinterpret_cast<VT *>(f.w);
  const VV *uv = reinterpret_cast<const VV *>(f.v);
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = LC > 0 ? LC : px.L;
  const int nrows = LC > 0 ? xpass_rows(LC) : d.nrows;
  const int nxt = LC > 0 ? (LC + W - 1) / W : d.nxt;
  const c64 *ua = f.ax_a[0];
  const VT *ub = reinterpret_cast<const VT *>(f.ax_b[0]);
  VT *ud = reinterpret_cast<VT *>(f.ax_d[0]);
  const int ne = nrows * Mx;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * ne;
  int *rowoff = reinterpret_cast<int *>(tw + Mx);
  load_twiddles(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, d.ny * d.nz - row0);
  x_row_offsets<T, LC>(rowoff, d, nrows, row0, nrow);
  const size_t off = (size_t)r * n3;
  c64 beta = {0, 0}, omega = {0, 0}, alpha = {0, 0}, cf[3] = {{0, 0}, {0, 0}, {0, 0}};
  if (f.in_mode == 1 || f.in_mode == 2) {
    const c64 *sc = f.scal + (size_t)r * kScal;
    beta = sc[S_BETA];
    omega = sc[S_OMEGA];
    alpha = sc[S_ALPHA];
    if (f.in_mode == 2 && f.fold_alpha && !block_alpha(f, r, alpha)) return;   // uniform per block
  } else if (f.in_mode == 3) {
    const c64 *sc = f.scal + (size_t)r * kScal;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const c64 g = a < f.nax ? sc[f.ax_slot[a]] : c64{0, 0};
      cf[a] = f.ax_neg[a] ? c64{-g.x, -g.y} : g;
    }
  }
  bool staged = false;
  if constexpr (LC > 0) {
    // the block's sites as one run of P; with Mx >= 2 nx - 1 a block holds at
    // most NR (Mx + 1) / 2 sites, which sizes the registers of this path
    constexpr int NR = xpass_rows(LC > 0 ? LC : 1);
    constexpr int ER = (3 * NR * ((LC + 1) / 2) + kNT - 1) / kNT;
    if (rowtab && d.nx <= (LC + 1) / 2) {
      const RowRuns<NR> rr(reinterpret_cast<const int *>(rowtab + row0), nrow, LC);
      const int n = 3 * rr.count;
      const size_t j0 = off + (size_t)3 * rr.first;
      c64 v[ER];
      if (f.in_mode == 0) {
        runs_load(v, n, in + j0);
      } else if (f.in_mode == 3) {
        runs_axpy(v, n, ua + j0, ub + j0, ud + j0, cf[0]);
        if constexpr (V64) {
          c64 u[ER];
          if (f.nax > 1) runs_axpy(u, n, f.ax_a[1] + j0, f.ax_b[1] + j0, f.ax_d[1] + j0, cf[1]);
          if (f.nax > 2) runs_axpy(u, n, f.ax_a[2] + j0, f.ax_b[2] + j0, f.ax_d[2] + j0, cf[2]);
        }
      } else if (f.in_mode == 1) {
        runs_p(v, n, f.r + j0, uw + j0, uv + j0, beta, omega);
      } else {
        runs_axpy(v, n, f.r + j0, uv + j0, uw + j0, c64{-alpha.x, -alpha.y});
      }
      const c64 *sr = sc.s ? sc.rhs(r) : nullptr;
#pragma unroll
      for (int i = 0; i < ER; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) {
          const int st = e / 3;
          const c64 x = sr ? sc.at(sr, rr.first + st, e - 3 * st) * v[i] : v[i];
          buf[(e - 3 * st) * ne + rr.pos(st)] = to_t<T>(x);
        }
      }
      for (int e = threadIdx.x; e < ne; e += kNT) {
        const int q = e / LC;
        if (!rr.holds(q, e - q * LC)) {
#pragma unroll
          for (int c = 0; c < 3; ++c) buf[c * ne + e] = cpx<T>{0, 0};
        }
      }
      staged = true;
    }
  }
  if (!staged) {
    int site[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = threadIdx.x + i * kNT;
      site[i] = -1;
      if (e < ne) {
        const int q = LC > 0 ? e / LC : (int)d.d_mx((uint32_t)e);
        const int x = e - q * Mx;
        if (q < nrow && x < d.nx) site[i] = cell_site[(size_t)(row0 + q) * d.nx + x];
      }
    }
    c64 v[NE][3];
    if (f.in_mode == 0) {
#pragma unroll
      for (int i = 0; i < NE; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[i][c] = site[i] >= 0 ? vld(in + off + (size_t)3 * site[i] + c) : c64{0, 0};
    } else if (f.in_mode == 3) {
      // update list d_i = a_i + c_i b_i; d_0 is transformed
#pragma unroll
      for (int i = 0; i < NE; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          c64 val = {0, 0};
          if (site[i] >= 0) {
            const size_t j = off + (size_t)3 * site[i] + c;
            val = vround<VT>(vld(ua + j) + cf[0] * vld(ub + j));
            vst(ud + j, val);
            if constexpr (V64) {
              if (f.nax > 1) f.ax_d[1][j] = f.ax_a[1][j] + cf[1] * f.ax_b[1][j];
              if (f.nax > 2) f.ax_d[2][j] = f.ax_a[2][j] + cf[2] * f.ax_b[2][j];
            }
          }
          v[i][c] = val;
        }
    } else {
#pragma unroll
      for (int i = 0; i < NE; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          c64 val = {0, 0};
          if (site[i] >= 0) {
            const size_t j = off + (size_t)3 * site[i] + c;
            if (f.in_mode == 1) val = vround<VT>(f.r[j] + beta * (vld(uw + j) - omega * vld(uv + j)));
            else val = vround<VT>(f.r[j] - alpha * vld(uv + j));
            vst(uw + j, val);
          }
          v[i][c] = val;
        }
    }
    if (sc.s) {
      const c64 *sr = sc.rhs(r);
#pragma unroll
      for (int i = 0; i < NE; ++i)
        if (site[i] >= 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) v[i][c] = sc.at(sr, site[i], c) * v[i][c];
        }
    }
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = threadIdx.x + i * kNT;
      if (e < ne) {
#pragma unroll
        for (int c = 0; c < 3; ++c) buf[c * ne + e] = to_t<T>(v[i][c]);
      }
    }
  }
  __syncthreads();
  fft_rows<T, EPT, -1, LC, V>(buf, tw, px, 3 * nrows);
  cpx<T> *Ar = A + (size_t)r * a_elems;
  const int nyW = d.ny * W;
  const int nseg = 3 * nrows * nxt;
  for (int e = threadIdx.x; e < (nseg << LOGW); e += kNT) {
    const int sg = e >> LOGW, p = e & (W - 1);
    const int pq = LC > 0 ? sg / ((LC + W - 1) / W) : (int)d.d_nxt((uint32_t)sg);
    const int xt = sg - pq * nxt;
    const int ro = rowoff[pq];
    if (ro >= 0) {
      const int kx = (xt << LOGW) + p;
      Ar[ro + xt * nyW + p] = kx < Mx ? buf[pq * Mx + kx] : cpx<T>{0, 0};
    }
  }
}

// --------------------------------------------------------------- y-forward --
template <typename T, int EPT, int LC>
__global__ __launch_bounds__(kNT) void k_yfwd(const int *__restrict__ mask, const cpx<T> *__restrict__ A,
                                               size_t a_elems, cpx<T> *__restrict__ B, size_t b_elems,
                                               const cpx<T> *__restrict__ twy, AxisPlan py, PassDims d) {
  constexpr int W = kW<T>, LOGW = kLogW<T>;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = LC > 0 ? LC : py.L;
  const int n = My << LOGW;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + n;
  load_twiddles(tw, twy, My);
  const int nxt = d.nxt, nz = d.nz;
  const int b = blockIdx.x;
  const int cz = b / nxt, xt = b - cz * nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *src = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * d.ny * W;
  const int nyW = d.ny << LOGW;
  stage_in<T, EPT>(buf, n, [&](int e) { return e < nyW ? src[e] : cpx<T>{0, 0}; });
  __syncthreads();
  fft_pen<T, EPT, -1, LOGW, LC>(buf, tw, py);
  cpx<T> *dst = B + (size_t)r * b_elems + (((size_t)xt * 3 + c) * nz + z) * W;
  const int kstr = nxt * 3 * nz * W;
  for (int e = threadIdx.x; e < n; e += kNT) dst[(e >> LOGW) * kstr + (e & (W - 1))] = buf[e];
}

// ------------------------------------------------------------------ z-pass --
template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

template <typename T>
__device__ __forceinline__ cpx<T> neg(cpx<T> a) { return {-a.x, -a.y}; }

// g0 p0 + g1 p1 + g2 p2 as two chains of one multiply and five fused
// multiply-adds (one per real product), instead of three complex products
// and two complex sums.
template <typename T>
__device__ __forceinline__ cpx<T> dot3(cpx<T> g0, cpx<T> p0, cpx<T> g1, cpx<T> p1, cpx<T> g2, cpx<T> p2) {
  T re = -g2.y * p2.y, im = g2.y * p2.x;
  re = fmaT(g2.x, p2.x, re);
  im = fmaT(g2.x, p2.y, im);
  re = fmaT(-g1.y, p1.y, re);
  im = fmaT(g1.y, p1.x, im);
  re = fmaT(g1.x, p1.x, re);
  im = fmaT(g1.x, p1.y, im);
  re = fmaT(-g0.y, p0.y, re);
  im = fmaT(g0.y, p0.x, im);
  re = fmaT(g0.x, p0.x, re);
  im = fmaT(g0.x, p0.y, im);
  return {re, im};
}

// The six Green values of one octant cell (stored cell-major, xx yy zz xy xz
// yz): three 16-byte loads in FP32, six in FP64.  Eight lanes of a wave read
// 8 consecutive cells, one contiguous run of 384 (FP32) bytes.
template <typename T>
__device__ __forceinline__ void load_green(const cpx<T> *g, cpx<T> (&v)[6]) {
  if constexpr (sizeof(T) == 4) {
    const float4 *p = reinterpret_cast<const float4 *>(g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 a = p[k];
      v[2 * k] = cpx<T>{a.x, a.y};
      v[2 * k + 1] = cpx<T>{a.z, a.w};
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = g[c];
  }
}

// Fold a frequency index into the stored octant: k <= M/2 is kept (sign +1),
// k > M/2 maps to M - k (sign -1 for components odd along this axis).
__device__ __forceinline__ int fold(int k, int M, int &sgn) {
  if (2 * k <= M) { sgn = 1; return k; }
  sgn = -1;
  return M - k;
}

// One block per (ky, x tile), or per half of an x tile (HALF = 1: the block
// takes NP = W/2 of the tile's W pencils, which halves its registers for long
// Mz; the two halves run next to each other and share the tile's 128-byte
// lines in L2).  The three components are transformed one after the other in
// an Mz x NP LDS buffer (in-place stages); the nz data rows of the next
// component are loaded into registers while the current one is transformed.
// Each thread owns octant cells (oz, p), oz <= Mz/2, and with them the mirror
// frequency Mz - oz of the same pencil: one read of the six Green values
// serves both, with the z-odd components (xz, yz) negated for the mirror.
// Forward spectra of components 0 and 1 are parked in registers, component 2
// stays in LDS.  V selects one of the alternative radix plans of a
// compile-time length (plan_variant); the plan autotuner picks it per length.
template <typename T, int EPT, int LC, int HALF, int V>
__global__ __launch_bounds__(kNT) void k_zpass(const int *__restrict__ mask, cpx<T> *__restrict__ B, size_t b_elems,
                                                const cpx<T> *__restrict__ ghat, const cpx<T> *__restrict__ twz,
                                                AxisPlan pz, PassDims d) {
  constexpr int W = kW<T>, LOGW = kLogW<T>;
  constexpr int LOGP = LOGW - HALF, NP = 1 << LOGP;
  // octant cells per thread, (Mz/2 + 1) NP <= NQ kNT, and data rows per
  // thread, nz NP <= (Mz + 1) NP / 2 <= NL kNT (exact when Mz = LC is known)
  constexpr int NQ = LC > 0 ? cdiv_c((LC / 2 + 1) << LOGP, kNT) : EPT / 2 + 1;
  constexpr int NL = LC > 0 ? cdiv_c(((LC + 1) / 2) << LOGP, kNT) : EPT / 2 + 1;
  // XCD-aware order.  Workgroups are dispatched to the 8 XCDs round-robin
  // (XCD = b mod 8), and each XCD has its own L2.  Logical index li runs
  // through contiguous ranges per XCD; consecutive li take the right-hand
  // sides of one column (so a batch reads the column's Green values from HBM
  // once), then the halves of a tile, ky and My - ky, and the x tiles t and
  // nxt - 1 - t: the (up to) four columns that read the same octant Green
  // values, and the two halves of a tile, share one L2.
  const int b = blockIdx.x;
  const int nb = ((d.My * d.nxt) << HALF) * d.nrhs, per = nb >> 3;
  const int lr = b < (per << 3) ? (b & 7) * per + (b >> 3) : b;
  const int li = (int)d.d_nrhs((uint32_t)lr), r = lr - li * d.nrhs;
  if (mask && !mask[r]) return;
  const int Mz = LC > 0 ? LC : pz.L;
  const int n = Mz << LOGP;
  const int nq = ((Mz >> 1) + 1) << LOGP;
  const int nzP = d.nz << LOGP;
  const int nzW = d.nz << LOGW;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + n;
  TwiddleStage<T, LC> tws;
  tws.issue(tw, twz, Mz);
  const int h = li & HALF, lt = li >> HALF;
  const int iy = (int)d.d_nxt((uint32_t)lt), ix = lt - iy * d.nxt;
  const int ky = (iy & 1) ? d.My - ((iy + 1) >> 1) : (iy >> 1);
  const int xt = (ix & 1) ? d.nxt - 1 - (ix >> 1) : (ix >> 1);
  cpx<T> *tile = B + (size_t)r * b_elems + (((size_t)ky * d.nxt + xt) * 3) * d.nz * W + h * NP;
  // element e = m NP + p of the block is tile[m W + p] of its component
  auto toff = [&](int e) { return HALF ? ((e >> LOGP) << LOGW) + (e & (NP - 1)) : e; };
  cpx<T> a0[NQ], b0[NQ], a1[NQ], b1[NQ];
  // forward spectra of components 0 and 1 -> registers (after the transform)
  auto park = [&](int c) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int q = threadIdx.x + i * kNT;
      if (q < nq) {
        const int oz = q >> LOGP, p = q & (NP - 1);
        const bool mir = oz != 0 && 2 * oz != Mz;
        const cpx<T> va = buf[q];
        const cpx<T> vb = mir ? buf[((Mz - oz) << LOGP) + p] : cpx<T>{0, 0};
        if (c == 0) { a0[i] = va; b0[i] = vb; }
        else { a1[i] = va; b1[i] = vb; }
      }
    }
    __syncthreads();
  };
  if constexpr (LC > 0) {
    // Compile-time plan: the nz data rows are loaded straight into the
    // registers of the first stage (rows >= (Mz + 1) / 2 >= nz are known
    // zeros), in a two-slot ring so component c + 1 is in flight while c is
    // transformed.
    using PE = PenEnds<LC, LOGP, V>;
    constexpr int MB = (LC + 1) / 2;
    cpx<T> pre[2][PE::NB0][PE::R0];
    auto fetch = [&](int c, cpx<T>(&dst)[PE::NB0][PE::R0]) {
#pragma unroll
      for (int i = 0; i < PE::NB0; ++i) {
        const int b = threadIdx.x + i * kNT;
#pragma unroll
        for (int k = 0; k < PE::R0; ++k) {
          const int e = b + k * PE::NBF0;
          const bool live = k * (LC / PE::R0) < MB && b < PE::NBF0 && (e >> LOGP) < d.nz;
          dst[i][k] = live ? tile[c * nzW + toff(e)] : cpx<T>{0, 0};
        }
      }
    };
    fetch(0, pre[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < 2) fetch(c + 1, pre[(c + 1) & 1]);
      if (c == 0) tws.commit(tw);
      fft_pen_from_regs<T, -1, LOGP, LC, V>(buf, tw, pre[c & 1]);
      if (c < 2) park(c);
    }
  } else {
    // two-slot ring: the rows of component c + 1 are in flight while c is transformed
    cpx<T> pre[2][NL];
    auto fetch = [&](int c, cpx<T>(&dst)[NL]) {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int e = threadIdx.x + i * kNT;
        dst[i] = e < nzP ? tile[c * nzW + toff(e)] : cpx<T>{0, 0};
      }
    };
    fetch(0, pre[0]);
    tws.commit(tw);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) buf[e] = (i < NL && e < nzP) ? pre[c & 1][i < NL ? i : 0] : cpx<T>{0, 0};
      }
      if (c < 2) fetch(c + 1, pre[(c + 1) & 1]);
      __syncthreads();
      fft_pen<T, EPT, -1, LOGP, LC>(buf, tw, pz);
      if (c < 2) park(c);
    }
  }
  int sy;
  const int oy = fold(ky, d.My, sy);
  // Green values of the thread's i-th cell and the x sign of its fold.  Lanes
  // past Mx (the last x tile) hold zeros, which the x-forward pass wrote there;
  // any Green value keeps them zero, so their index is clamped.  Slots past
  // nq load cell 0 (in bounds, unused): the loads are unconditional, so in
  // FP32 the next cell's loads stay in flight while the current cell is
  // multiplied.  FP64 loads each cell's values where they are used: holding
  // the next cell's twelve doubles costs the FP64 kernel occupancy.
  constexpr bool kAhead = sizeof(T) == 4;
  auto green_at = [&](int i, cpx<T>(&gv)[6], int &sx) {
    const int q = threadIdx.x + i * kNT;
    const int qc = q < nq ? q : 0;
    const int kx = min((xt << LOGW) + h * NP + (qc & (NP - 1)), d.Mx - 1);
    const int ox = fold(kx, d.Mx, sx);
    load_green(ghat + 6 * (size_t)(mul24(mul24(qc >> LOGP, d.Myh) + oy, d.Mxh) + ox), gv);
  };
  cpx<T> gnext[6];
  int sxnext = 1;
  if constexpr (kAhead) green_at(0, gnext, sxnext);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + i * kNT;
    cpx<T> gv[6];
    int sx;
    if constexpr (kAhead) {
#pragma unroll
      for (int c = 0; c < 6; ++c) gv[c] = gnext[c];
      sx = sxnext;
      if (i + 1 < NQ) green_at(i + 1, gnext, sxnext);
    } else {
      green_at(i, gv, sx);
    }
    if (q < nq) {
      const int oz = q >> LOGP, p = q & (NP - 1);
      const bool mir = oz != 0 && 2 * oz != Mz;
      // without a mirror (oz = 0 or Mz/2) the mirror products are computed on
      // the cell itself and discarded
      const int zb = mir ? ((Mz - oz) << LOGP) + p : q;
      const cpx<T> gxx = gv[0], gyy = gv[1], gzz = gv[2];
      const cpx<T> gxy = T(sx * sy) * gv[3], gxz = T(sx) * gv[4], gyz = T(sy) * gv[5];
      const cpx<T> a2 = buf[q], b2 = buf[zb];
      const cpx<T> qa0 = dot3(gxx, a0[i], gxy, a1[i], gxz, a2);
      const cpx<T> qa1 = dot3(gxy, a0[i], gyy, a1[i], gyz, a2);
      const cpx<T> qa2 = dot3(gxz, a0[i], gyz, a1[i], gzz, a2);
      // the mirror frequency Mz - oz: the z-odd components change sign
      const cpx<T> qb0 = dot3(gxx, b0[i], gxy, b1[i], neg(gxz), b2);
      const cpx<T> qb1 = dot3(gxy, b0[i], gyy, b1[i], neg(gyz), b2);
      const cpx<T> qb2 = dot3(neg(gxz), b0[i], neg(gyz), b1[i], gzz, b2);
      a0[i] = qa0;
      a1[i] = qa1;
      b0[i] = qb0;
      b1[i] = qb1;
      buf[q] = qa2;
      if (mir) buf[zb] = qb2;
    }
  }
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const int c = (cc + 2) % 3;     // 2 (already in LDS), then 0, 1
    if (c != 2) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int q = threadIdx.x + i * kNT;
        if (q < nq) {
          const int oz = q >> LOGP, p = q & (NP - 1);
          buf[q] = c == 0 ? a0[i] : a1[i];
          if (oz != 0 && 2 * oz != Mz) buf[((Mz - oz) << LOGP) + p] = c == 0 ? b0[i] : b1[i];
        }
      }
      __syncthreads();
    }
    cpx<T> *dst = tile + c * nzW;
    if constexpr (LC > 0) {
      // the last stage writes the nz kept rows straight to global memory
      fft_pen_to_store<T, +1, LOGP, LC, V>(buf, tw, [&](int e, cpx<T> v) {
        if ((e >> LOGP) < d.nz) dst[toff(e)] = v;
      });
    } else {
      fft_pen<T, EPT, +1, LOGP, LC>(buf, tw, pz);
      for (int e = threadIdx.x; e < nzP; e += kNT) dst[toff(e)] = buf[e];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------- y-inverse --
template <typename T, int EPT, int LC>
__global__ __launch_bounds__(kNT) void k_yinv(const int *__restrict__ mask, const cpx<T> *__restrict__ B,
                                               size_t b_elems, cpx<T> *__restrict__ A, size_t a_elems,
                                               const cpx<T> *__restrict__ twy, AxisPlan py, PassDims d) {
  constexpr int W = kW<T>, LOGW = kLogW<T>;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = LC > 0 ? LC : py.L;
  const int n = My << LOGW;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + n;
  load_twiddles(tw, twy, My);
  const int nxt = d.nxt, nz = d.nz;
  const int b = blockIdx.x;
  const int cz = b / nxt, xt = b - cz * nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *src = B + (size_t)r * b_elems + (((size_t)xt * 3 + c) * nz + z) * W;
  const int kstr = nxt * 3 * nz * W;
  stage_in<T, EPT>(buf, n, [&](int e) { return src[(e >> LOGW) * kstr + (e & (W - 1))]; });
  __syncthreads();
  fft_pen<T, EPT, +1, LOGW, LC>(buf, tw, py);
  cpx<T> *dst = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * d.ny * W;
  const int nyW = d.ny << LOGW;
  for (int e = threadIdx.x; e < nyW; e += kNT) dst[e] = buf[e];
}

// --------------------------------------------------------------- x-inverse --
// f.out_mode (see FuseArgs): 0 only writes out = ainv * in - G*in; 1 and 2 also
// write per-block partial sums of the BiCGSTAB inner products of `out`.
// MODES, chosen when the kernel is launched, names the out_modes an
// instantiation handles, so that it holds only the registers those need:
// 1 = {0, 4} (the plain product; the bilinear in^T out of COCG and QMR: no
// FP64 operand, two sums; in FP32 68 instead of 92 VGPRs, 7 resident waves
// per SIMD instead of 5), 2 = {1, 2} (BiCGSTAB: three sums), 0 = all
// (BiCGstab(2)'s mode 3: eight sums).
template <typename T, int EPT, int LC, int V, typename VT, int MODES>
__global__ __launch_bounds__(kNT) void k_xinv(const VT *__restrict__ in, VT *__restrict__ out, int64_t n3,
                                               const int *__restrict__ mask, const c64 *__restrict__ ainv,
                                               int ncomp, const uint8_t *__restrict__ comp,
                                               const int *__restrict__ cell_site, const int4 *__restrict__ rowtab,
                                               Scaling sc, const cpx<T> *__restrict__ A, size_t a_elems,
                                               const cpx<T> *__restrict__ twx, AxisPlan px, PassDims d, FuseArgs f) {
  constexpr int W = kW<T>, LOGW = kLogW<T>;
  constexpr int NE = (EPT + 2) / 3;
  constexpr bool kSmall = MODES == 1, kBicg = MODES == 2;
  const int out_mode = kSmall ? (f.out_mode == 4 ? 4 : 0) : f.out_mode;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = LC > 0 ? LC : px.L;
  const int nrows = LC > 0 ? xpass_rows(LC) : d.nrows;
  const int ne = nrows * Mx;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * ne;
  int *rowoff = reinterpret_cast<int *>(tw + Mx);
  TwiddleStage<T, LC> tws;
  tws.issue(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, d.ny * d.nz - row0);
  x_row_offsets<T, LC>(rowoff, d, nrows, row0, nrow);
  // Read before the transform, so that these loads overlap those of A: the
  // block's row runs (sites numbered row after row) and, with one
  // composition, the three values of 1/alpha that every site of this
  // right-hand side takes.
  constexpr int NR = xpass_rows(LC > 0 ? LC : 1);
  const bool runs = LC > 0 && rowtab && d.nx <= (LC + 1) / 2;
  // The row-table entries go to LDS (a global read after the transform
  // would delay every load of P behind it); their load is in flight with
  // those of A.
  int *rtab = rowoff + 3 * nrows;
  const bool rt_lane = runs && threadIdx.x < 4 * nrow;
  const int rt_val = rt_lane ? reinterpret_cast<const int *>(rowtab + row0)[threadIdx.x] : 0;
  const c64 *ai = ainv + (size_t)r * ncomp * 3;      // [ncomp][3] of this RHS
  // (three values, not an array: a select between array elements would put
  // the array in scratch memory)
  c64 ax{0, 0}, ay{0, 0}, az{0, 0};
  if (!comp) {
    ax = ai[0];
    ay = ai[1];
    az = ai[2];
  }
  // 1/alpha of component c at a site
  auto alpha_inv = [&](int site, int c) -> c64 {
    if (comp) return ai[3 * comp[site] + c];
    c64 v = az;
    if (c == 0) v = ax;
    if (c == 1) v = ay;
    return v;
  };
  __syncthreads();
  const cpx<T> *Ar = A + (size_t)r * a_elems;
  const int nyW = d.ny * W;
  stage_in<T, EPT>(buf, 3 * ne, [&](int e) {
    const int pq = LC > 0 ? e / LC : (int)d.d_mx((uint32_t)e);
    const int kx = e - pq * Mx;
    const int ro = rowoff[pq];
    return ro >= 0 ? Ar[ro + (kx >> LOGW) * nyW + (kx & (W - 1))] : cpx<T>{0, 0};
  });
  if (rt_lane) rtab[threadIdx.x] = rt_val;
  tws.commit(tw);
  __syncthreads();
  const size_t off = (size_t)r * n3;
  // FP64 small mode with row runs: the loads of the block's run of P are
  // issued here, so that they are in flight during the transform (FP64
  // blocks are bound by LDS to 5 per CU, so the registers are free; in FP32
  // they cost a resident wave and the pass was measured slower).
  constexpr bool kPre = LC > 0 && kSmall && sizeof(T) == 8;
  constexpr int ERP = kPre ? (3 * NR * ((LC + 1) / 2) + kNT - 1) / kNT : 1;
  VT pin[ERP];
  if constexpr (kPre) {
    // Unconditional loads (no branch, so the compiler keeps them in flight
    // across the transform): indices past the run are clamped to its first
    // element, and a block without row runs or sites reads the first element
    // of P.  Without row runs the row-table words read here are unused.
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) cnt += q < nrow ? rtab[4 * q + 2] : 0;
    const int np = runs ? 3 * cnt : 0;
    const VT *src = np > 0 ? in + off + (size_t)3 * rtab[0] : in;
#pragma unroll
    for (int i = 0; i < ERP; ++i) {
      const int e = threadIdx.x + i * kNT;
      pin[i] = src[e < np ? e : 0];
    }
  }
  fft_rows<T, EPT, +1, LC, V>(buf, tw, px, 3 * nrows);
  if constexpr (kPre) {
    // keeps the compiler from converting (and so waiting for) the loaded
    // values before the transform
#pragma unroll
    for (int i = 0; i < ERP; ++i) asm volatile("" : "+v"(pin[i].x), "+v"(pin[i].y));
  }
  constexpr int NACC = kSmall ? 2 : kBicg ? 3 : 8;
  double acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
  const c64 *sr = sc.s ? sc.rhs(r) : nullptr;
  // with scaling the field term becomes s (G s P): each thread scales the
  // transformed values it is about to read
  auto scale_at = [&](int idx, int site, int c) {
    const cpx<T> g = buf[idx];
    buf[idx] = to_t<T>(sc.at(sr, site, c) * c64{double(g.x), double(g.y)});
  };
  // out = ainv P - (G P) at one element; x is rh (out_mode 1) or r0 (out_mode 3)
  auto finish = [&](size_t j, c64 a, c64 pv, cpx<T> fv, c64 x) {
    const c64 dd = a * pv;
    const c64 o = vround<VT>(c64{dd.x - double(fv.x), dd.y - double(fv.y)});
    vst(out + j, o);
    if (out_mode == 4) {
      const c64 g = pv * o;                          // bilinear in^T out
      acc[0] += g.x;
      acc[1] += g.y;
    }
    if constexpr (!kSmall) {
      if (out_mode == 1) {
        const c64 g = cmulc(x, o);
        acc[0] += g.x;
        acc[1] += g.y;
      } else if (out_mode == 2) {
        const c64 g = cmulc(o, pv);
        acc[0] += g.x;
        acc[1] += g.y;
        acc[2] += o.x * o.x + o.y * o.y;
      } else if constexpr (!kBicg) {
        if (out_mode == 3) {
          // in = r1, out = r2, f.r = r0
          const c64 g12 = cmulc(pv, o), g10 = cmulc(pv, x), g20 = cmulc(o, x);
          acc[0] += pv.x * pv.x + pv.y * pv.y;
          acc[1] += o.x * o.x + o.y * o.y;
          acc[2] += g12.x;
          acc[3] += g12.y;
          acc[4] += g10.x;
          acc[5] += g10.y;
          acc[6] += g20.x;
          acc[7] += g20.y;
        }
      }
    }
  };
  // BiCGSTAB's rh (out mode 1) and BiCGstab(2)'s r0 (out mode 3) are FP64 vectors
  const c64 *xsrc = kSmall ? nullptr : out_mode == 1 ? f.rh : (!kBicg && out_mode == 3) ? f.r : nullptr;
  bool done = false;
  if constexpr (LC > 0) {
    constexpr int ER = (3 * NR * ((LC + 1) / 2) + kNT - 1) / kNT;
    if (runs) {
      const RowRuns<NR> rr(rtab, nrow, LC);
      const int n = 3 * rr.count;
      const size_t j0 = off + (size_t)3 * rr.first;
      if (sr) {
#pragma unroll
        for (int i = 0; i < ER; ++i) {
          const int e = threadIdx.x + i * kNT;
          if (e < n) {
            const int st = e / 3;
            scale_at((e - 3 * st) * ne + rr.pos(st), rr.first + st, e - 3 * st);
          }
        }
      }
      c64 pv[ER], xv[ER], av[ER];
#pragma unroll
      for (int i = 0; i < ER; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) {
          if constexpr (kPre) pv[i] = vld(&pin[i]);
          else pv[i] = vld(in + j0 + e);
          xv[i] = xsrc ? xsrc[j0 + e] : c64{0, 0};
          const int st = e / 3;
          av[i] = alpha_inv(rr.first + st, e - 3 * st);
        }
      }
#pragma unroll
      for (int i = 0; i < ER; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) {
          const int st = e / 3;
          finish(j0 + e, av[i], pv[i], buf[(e - 3 * st) * ne + rr.pos(st)], xv[i]);
        }
      }
      done = true;
    }
  }
  if (!done) {
    const int nsite = nrow * d.nx;
    const int *cs = cell_site + (size_t)row0 * d.nx;
    int site[NE], bi[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = threadIdx.x + i * kNT;
      site[i] = -1;
      bi[i] = 0;
      if (e < nsite) {
        site[i] = cs[e];
        const int q = (int)d.d_nx((uint32_t)e);
        bi[i] = q * Mx + (e - q * d.nx);
      }
    }
    if (sr) {
#pragma unroll
      for (int i = 0; i < NE; ++i)
        if (site[i] >= 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) scale_at(c * ne + bi[i], site[i], c);
        }
    }
    c64 pv[NE][3];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) pv[i][c] = site[i] >= 0 ? vld(in + off + (size_t)3 * site[i] + c) : c64{0, 0};
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      if (site[i] >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const size_t j = off + (size_t)3 * site[i] + c;
          finish(j, alpha_inv(site[i], c), pv[i][c], buf[c * ne + bi[i]], xsrc ? xsrc[j] : c64{0, 0});
        }
      }
    }
  }
  // one partial record per block; a one-block kernel adds them in block order
  if constexpr (kSmall) {
    // COCG's and QMR's records hold the two parts of in^T out
    if (out_mode == 4) {
      double tot[2];
      block_sum<2, kNT>(acc, tot);
      if (threadIdx.x == 0) write_record<2>(f.partial, r, gridDim.x, blockIdx.x, tot);
    }
  } else if constexpr (kBicg) {
    double tot[3];
    block_sum<3, kNT>(acc, tot);
    if (threadIdx.x == 0) write_record<3>(f.partial, r, gridDim.x, blockIdx.x, tot);
  } else if (out_mode == 3) {
    double tot[8];
    block_sum<8, kNT>(acc, tot);
    if (threadIdx.x == 0) write_record<8>(f.partial, r, gridDim.x, blockIdx.x, tot);
  } else if (out_mode != 0) {
    double a3[3] = {acc[0], acc[1], acc[2]};
    double tot[3];
    block_sum<3, kNT>(a3, tot);
    if (threadIdx.x == 0) write_record<3>(f.partial, r, gridDim.x, blockIdx.x, tot);
  }
}

// --------------------------------------------------------------- launchers --
template <int V>
using IC = std::integral_constant<int, V>;

// Register arrays are sized by EPT = elements per thread (a compile-time
// bound, one kernel instantiation per size).
constexpr int pick_ept_c(size_t elems, bool xpass) {
  const int opts[7] = {4, 8, 12, 16, 20, 24, 32};
  for (int i = 0; i < (xpass ? 2 : 7); ++i)
    if ((size_t)opts[i] * kNT >= elems) return opts[i];
  return 0;
}

// f(IC<EPT>) for the smallest EPT in {4, 8, 12, 16, 20, 24, 32} with
// EPT * kNT >= elems; only the sizes up to MAXE are instantiated.
template <int MAXE, typename F>
static inline void with_ept(size_t elems, F &&f) {
  const int e = pick_ept_c(elems, false);
  if (e == 0 || e > MAXE) throw Error{DDA_ENOTSUP, "FFT tile too large for one block"};
  switch (e) {
    case 4: f(IC<4>{}); break;
    case 8: if constexpr (MAXE >= 8) f(IC<8>{}); break;
    case 12: if constexpr (MAXE >= 12) f(IC<12>{}); break;
    case 16: if constexpr (MAXE >= 16) f(IC<16>{}); break;
    case 20: if constexpr (MAXE >= 20) f(IC<20>{}); break;
    case 24: if constexpr (MAXE >= 24) f(IC<24>{}); break;
    default: if constexpr (MAXE >= 32) f(IC<32>{}); break;
  }
}

// Transform lengths with a compile-time plan: every 2/3/5-smooth length from
// 27 to 192 (the padded extents of targets up to 96 dipoles across) and the
// 256 and 270 of larger workloads; the others use the run-time plan.
template <int... Ls>
struct LenList {};
using StaticLens = LenList<27, 30, 32, 36, 40, 45, 48, 50, 54, 60, 64, 72, 75, 80, 81, 90, 96, 100, 108, 120, 125, 128,
                           135, 144, 150, 160, 162, 180, 192, 256, 270>;

template <typename F>
static inline void with_len_in(int, F &&f, LenList<>) {
  f(IC<0>{});
}
template <typename F, int L0, int... Ls>
static inline void with_len_in(int L, F &&f, LenList<L0, Ls...>) {
  if (L == L0) f(IC<L0>{});
  else with_len_in(L, f, LenList<Ls...>{});
}
template <typename F>
static inline void with_len(int L, F &&f) {
  with_len_in(L, f, StaticLens{});
}

// Calls f(IC<EPT>, IC<LC>) for a pass of `elems` elements per block along an
// axis of length L (with LC > 0 the caller derives EPT from LC).
template <int MAXE, typename F>
static inline void with_pass(int L, size_t elems, F &&f) {
  with_len(L, [&](auto lc) {
    constexpr int LC = decltype(lc)::value;
    if constexpr (LC > 0) f(IC<0>{}, lc);
    else with_ept<MAXE>(elems, [&](auto e) { f(e, lc); });
  });
}

template <typename K>
static inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) DDA_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// The x-forward (k = 0) or x-inverse (k = 4) pass with the product's input and
// output of type VT and the update's v of type VV (c64, or c32 for the search
// directions and their products in a DDA_MIXED_V32 solve).  The x-inverse does
// not depend on VV.
template <typename T, typename VT, typename VV>
void launch_x_pass(int k, const Geometry &g, const MatvecArgs &a, const PassDims &d, hipStream_t s) {
  if constexpr (!std::is_same_v<VT, VV>) {
    if (k != 0) {
      launch_x_pass<T, VT, VT>(k, g, a, d, s);
      return;
    }
  }
  const bool f32 = sizeof(T) == 4;
  const size_t ae = g.a_elems(f32);
  cpx<T> *A = static_cast<cpx<T> *>(a.bufA);
  const cpx<T> *twx = static_cast<const cpx<T> *>(a.twx);
  const int64_t n3 = 3 * g.n_sites;
  const int nrows = xpass_rows(g.Mx);
  const int nrowblk = (g.ny * g.nz + nrows - 1) / nrows;
  const size_t cs = sizeof(cpx<T>);
  const FuseArgs &f = a.fuse;
  const VT *in = reinterpret_cast<const VT *>(a.in);
  VT *out = reinterpret_cast<VT *>(a.out);
  // rows-plan variants of the x-forward and x-inverse passes (forced or tuned)
  const int xv[2] = {a.xvar[0] >= 0 ? a.xvar[0] : tuned_variant(kPassXfwd, g.Mx, f32),
                     a.xvar[1] >= 0 ? a.xvar[1] : tuned_variant(kPassXinv, g.Mx, f32)};
  // rows, twiddles, the row offsets and the block's row-table entries
  const size_t xlds = ((size_t)3 * nrows * g.Mx + g.Mx) * cs + (size_t)7 * nrows * sizeof(int);
  if (k == 0) {
    with_pass<8>(g.Mx, (size_t)3 * nrows * g.Mx, [&](auto e, auto lc) {
      constexpr int LC = decltype(lc)::value;
      constexpr int E = LC > 0 ? pick_ept_c((size_t)3 * xpass_rows(LC) * LC, true) : decltype(e)::value;
      auto go = [&](auto vv) {
        hipLaunchKernelGGL((k_xfwd<T, E, LC, decltype(vv)::value, VT, VV>), dim3(nrowblk, a.nrhs), dim3(kNT), xlds, s,
                           in, n3, a.mask, a.cell_site, a.rowtab, a.scl, A, ae, twx, a.px, d, f);
      };
      if constexpr (LC >= kTunedMinLen) {
        if (xv[0] == 1) go(IC<1>{});
        else go(IC<0>{});
      } else {
        go(IC<0>{});
      }
    });
  } else {
    with_pass<8>(g.Mx, (size_t)3 * nrows * g.Mx, [&](auto e, auto lc) {
      constexpr int LC = decltype(lc)::value;
      constexpr int E = LC > 0 ? pick_ept_c((size_t)3 * xpass_rows(LC) * LC, true) : decltype(e)::value;
      // the instantiation that holds only the registers of this out_mode
      const int modes = (f.out_mode == 0 || f.out_mode == 4) ? 1 : (f.out_mode == 1 || f.out_mode == 2) ? 2 : 0;
      auto go = [&](auto vv) {
        constexpr int PV = decltype(vv)::value;
        if (modes == 1)
          hipLaunchKernelGGL((k_xinv<T, E, LC, PV, VT, 1>), dim3(nrowblk, a.nrhs), dim3(kNT), xlds, s, in, out, n3,
                             a.mask, a.ainv, a.ncomp, a.comp, a.cell_site, a.rowtab, a.scl, A, ae, twx, a.px, d, f);
        else if (modes == 2)
          hipLaunchKernelGGL((k_xinv<T, E, LC, PV, VT, 2>), dim3(nrowblk, a.nrhs), dim3(kNT), xlds, s, in, out, n3,
                             a.mask, a.ainv, a.ncomp, a.comp, a.cell_site, a.rowtab, a.scl, A, ae, twx, a.px, d, f);
        else
          hipLaunchKernelGGL((k_xinv<T, E, LC, PV, VT, 0>), dim3(nrowblk, a.nrhs), dim3(kNT), xlds, s, in, out, n3,
                             a.mask, a.ainv, a.ncomp, a.comp, a.cell_site, a.rowtab, a.scl, A, ae, twx, a.px, d, f);
      };
      if constexpr (LC >= kTunedMinLen) {
        if (xv[1] == 1) go(IC<1>{});
        else go(IC<0>{});
      } else {
        go(IC<0>{});
      }
    });
  }
}

template <typename T>
void launch_matvec(const Geometry &g, const MatvecArgs &a, hipStream_t s, const hipEvent_t *ev, int only_pass,
                   int reps) {
  const bool f32 = sizeof(T) == 4;
  constexpr int W = kW<T>;
  const int nxt = g.nxt(f32);
  const size_t ae = g.a_elems(f32), be = g.b_elems(f32);
  DDA_REQUIRE(ae < (size_t(1) << 31) && be < (size_t(1) << 31), "grid too large for 32-bit tile offsets");
  cpx<T> *A = static_cast<cpx<T> *>(a.bufA);
  cpx<T> *B = static_cast<cpx<T> *>(a.bufB);
  const cpx<T> *twy = static_cast<const cpx<T> *>(a.twy);
  const cpx<T> *twz = static_cast<const cpx<T> *>(a.twz);
  const int nrows = xpass_rows(g.Mx);
  const int nrowblk = (g.ny * g.nz + nrows - 1) / nrows;
  const size_t cs = sizeof(cpx<T>);
  PassDims d{};
  d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
  d.Mx = g.Mx; d.My = g.My;
  d.nxt = nxt;
  d.nrows = nrows;
  d.Mxh = g.Mxh; d.Myh = g.Myh;
  d.d_mx = make_fastdiv(g.Mx);
  d.d_nx = make_fastdiv(g.nx);
  d.d_ny = make_fastdiv(g.ny);
  d.d_nxt = make_fastdiv(nxt);
  d.d_nrows = make_fastdiv(nrows);
  d.nrhs = a.nrhs;
  d.d_nrhs = make_fastdiv(a.nrhs);
  // the z-pass divides its block index (< blocks * nrhs) by nrhs with d_nrhs,
  // exact while that index times nrhs stays below 2^32
  DDA_REQUIRE((uint64_t)((g.My * nxt) << 1) * a.nrhs * a.nrhs < (uint64_t(1) << 32),
              "too many right-hand sides in one product for this grid");
  const FuseArgs &f = a.fuse;
  // the x-inverse writes one record per block; a folding x-forward reads nrec
  DDA_REQUIRE(f.out_mode == 0 || (f.partial && nrowblk <= f.rec_cap), "product records exceed their buffer");
  DDA_REQUIRE(!f.fold_alpha || (f.nrec >= 1 && f.nrec <= f.rec_cap), "folded records exceed their buffer");
  auto pass = [&](int k) {
    switch (k) {
      case 0:
      case 4:
        // FP32 Krylov vectors only with the FP32 product
        if constexpr (sizeof(T) == 4) {
          if (a.vec32) {
            launch_x_pass<T, c32, c32>(k, g, a, d, s);
            break;
          }
          if (a.vvec32) {
            launch_x_pass<T, c64, c32>(k, g, a, d, s);
            break;
          }
        }
        launch_x_pass<T, c64, c64>(k, g, a, d, s);
        break;
      case 1:
        with_pass<32>(g.My, (size_t)g.My * W, [&](auto e, auto lc) {
          constexpr int LC = decltype(lc)::value;
          constexpr int E = LC > 0 ? pick_ept_c((size_t)LC * W, false) : decltype(e)::value;
          const size_t lds = ((size_t)g.My * W + g.My) * cs;
          allow_lds(k_yfwd<T, E, LC>, lds);
          hipLaunchKernelGGL((k_yfwd<T, E, LC>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, A, ae, B,
                             be, twy, a.py, d);
        });
        break;
      case 2: {
        // half tiles for long columns (FP32: Mz > 128, FP64: Mz > 128): it halves
        // the registers a thread needs for the parked spectra
        constexpr int kHalfAbove = sizeof(T) == 4 ? 2048 : 1024;
        const int half = g.Mz * W > kHalfAbove ? 1 : 0;
        auto launch = [&](auto e, auto lc, auto hf, auto vv) {
          constexpr int LC = decltype(lc)::value, H = decltype(hf)::value, E = decltype(e)::value;
          constexpr int V = decltype(vv)::value;
          const size_t lds = (((size_t)g.Mz * W >> H) + g.Mz) * cs;
          allow_lds(k_zpass<T, E, LC, H, V>, lds);
          hipLaunchKernelGGL((k_zpass<T, E, LC, H, V>), dim3(((g.My * nxt) << H) * a.nrhs), dim3(kNT), lds, s,
                             a.mask, B, be, static_cast<const cpx<T> *>(a.ghat), twz, a.pz, d);
        };
        // plan variant: forced by the caller, else the autotuner's table, else the cost model's
        const int zv = a.zvar >= 0 ? a.zvar : tuned_variant(kPassZ, g.Mz, f32);
        with_len(g.Mz, [&](auto lc) {
          constexpr int LC = decltype(lc)::value;
          if constexpr (LC > 0) {
            constexpr int H = LC * W > kHalfAbove ? 1 : 0;
            constexpr int E = pick_ept_c((size_t)(LC * W) >> H, false);
            if constexpr (LC >= kTunedMinLen) {
              switch (zv) {
                case 1: launch(IC<E>{}, lc, IC<H>{}, IC<1>{}); break;
                case 2: launch(IC<E>{}, lc, IC<H>{}, IC<2>{}); break;
                case 3: launch(IC<E>{}, lc, IC<H>{}, IC<3>{}); break;
                default: launch(IC<E>{}, lc, IC<H>{}, IC<0>{}); break;
              }
            } else {
              launch(IC<E>{}, lc, IC<H>{}, IC<0>{});
            }
          } else if (half) {
            with_ept<16>((size_t)g.Mz * W / 2, [&](auto e) { launch(e, lc, IC<1>{}, IC<0>{}); });
          } else {
            with_ept<8>((size_t)g.Mz * W, [&](auto e) { launch(e, lc, IC<0>{}, IC<0>{}); });
          }
        });
      } break;
      case 3:
        with_pass<32>(g.My, (size_t)g.My * W, [&](auto e, auto lc) {
          constexpr int LC = decltype(lc)::value;
          constexpr int E = LC > 0 ? pick_ept_c((size_t)LC * W, false) : decltype(e)::value;
          const size_t lds = ((size_t)g.My * W + g.My) * cs;
          allow_lds(k_yinv<T, E, LC>, lds);
          hipLaunchKernelGGL((k_yinv<T, E, LC>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, B, be, A,
                             ae, twy, a.py, d);
        });
        break;
    }
  };
  if (only_pass >= 0) {
    // one pass, `reps` launches back to back between ev[0] and ev[1]
    if (ev) DDA_HIP(hipEventRecord(ev[0], s));
    for (int i = 0; i < reps; ++i) pass(only_pass);
    if (ev) DDA_HIP(hipEventRecord(ev[1], s));
  } else {
    for (int k = 0; k < 5; ++k) {
      if (ev) DDA_HIP(hipEventRecord(ev[k], s));
      pass(k);
    }
    if (ev) DDA_HIP(hipEventRecord(ev[5], s));
  }
  DDA_HIP(hipGetLastError());
}

}  // namespace dda
