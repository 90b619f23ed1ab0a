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

// --------------------------------------------------------------- x-forward --
// f.in_mode (see FuseArgs): 0 transforms `in`; 1 and 2 first form the BiCGSTAB
// vector p or s from r, v (and the old p) and store it, so the vector update
// costs no pass of its own.
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_xfwd(const c64 *__restrict__ in, int64_t n3, const int *__restrict__ mask,
                                               const int *__restrict__ cell_site, cpx<T> *__restrict__ A,
                                               size_t a_elems, const cpx<T> *__restrict__ twx, AxisPlan px,
                                               int nx, int ny, int nz, int nxt, int nrows, FuseArgs f) {
  constexpr int W = kW<T>;
  constexpr int NE = (EPT + 2) / 3;      // nrows * Mx <= EPT * kNT / 3
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = px.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * nrows * Mx;
  load_twiddles(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, ny * nz - row0);
  const size_t off = (size_t)r * n3;
  const int ne = nrows * Mx;
  int site[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = threadIdx.x + i * kNT;
    site[i] = -1;
    if (e < ne) {
      const int q = e / Mx, x = e - q * Mx;
      if (q < nrow && x < nx) site[i] = cell_site[(size_t)(row0 + q) * nx + x];
    }
  }
  c64 v[NE][3];
  if (f.in_mode == 0) {
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) v[i][c] = site[i] >= 0 ? in[off + (size_t)3 * site[i] + c] : c64{0, 0};
  } else {
    const c64 *sc = f.scal + (size_t)r * kScal;
    const c64 beta = sc[S_BETA], omega = sc[S_OMEGA], alpha = sc[S_ALPHA];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        c64 val = {0, 0};
        if (site[i] >= 0) {
          const size_t j = off + (size_t)3 * site[i] + c;
          if (f.in_mode == 1) val = f.r[j] + beta * (f.w[j] - omega * f.v[j]);
          else val = f.r[j] - alpha * f.v[j];
          f.w[j] = val;
        }
        v[i][c] = val;
      }
  }
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < ne) {
      const int q = e / Mx, x = e - q * Mx;
#pragma unroll
      for (int c = 0; c < 3; ++c) buf[(c * nrows + q) * Mx + x] = to_t<T>(v[i][c]);
    }
  }
  __syncthreads();
  fft_lds<T, EPT, -1>(buf, tw, px, 3 * nrows, Mx, 1, false);
  const int nxtW = nxt * W;
  cpx<T> *Ar = A + (size_t)r * a_elems;
  for (int e = threadIdx.x; e < 3 * nrows * nxtW; e += kNT) {
    const int pq = e / nxtW, kx = e - pq * nxtW;
    const int c = pq / nrows, q = pq - c * nrows;
    if (q < nrow) {
      const int row = row0 + q, z = row / ny, y = row - z * ny;
      const int xt = kx / W, p = kx % W;
      const cpx<T> val = kx < Mx ? buf[pq * Mx + kx] : cpx<T>{0, 0};
      Ar[((((size_t)c * nz + z) * nxt + xt) * ny + y) * W + p] = val;
    }
  }
}

// --------------------------------------------------------------- y-forward --
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_yfwd(const int *__restrict__ mask, const cpx<T> *__restrict__ A,
                                               size_t a_elems, cpx<T> *__restrict__ B, size_t b_elems,
                                               const cpx<T> *__restrict__ twy, AxisPlan py, int ny, int nz,
                                               int nxt) {
  constexpr int W = kW<T>;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = py.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + My * W;
  load_twiddles(tw, twy, My);
  const int b = blockIdx.x;
  const int xt = b % nxt, cz = b / nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *src = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * ny * W;
  stage_in<T, EPT>(buf, My * W, [&](int e) { return e < ny * W ? src[e] : cpx<T>{0, 0}; });
  __syncthreads();
  fft_lds<T, EPT, -1>(buf, tw, py, W, 1, W, true);
  cpx<T> *Br = B + (size_t)r * b_elems;
  for (int e = threadIdx.x; e < My * W; e += kNT) {
    const int ky = e / W, p = e % W;
    Br[((((size_t)ky * nxt + xt) * 3 + c) * nz + z) * W + p] = buf[e];
  }
}

// ------------------------------------------------------------------ z-pass --
// Fold a frequency index into the stored octant: k <= M/2 is kept (sign +1),
// k > M/2 maps to M - k (sign -1 for components odd along this axis).
__device__ __forceinline__ int fold(int k, int M, int &sgn) {
  if (2 * k <= M) { sgn = 1; return k; }
  sgn = -1;
  return M - k;
}

// One block per (ky, x tile); the three components are transformed one after
// the other in an Mz x W LDS buffer (staged loads, in-place stages).  Each
// thread owns octant cells (oz, p), oz <= Mz/2, and with them the mirror
// frequency Mz - oz of the same pencil: one read of the six Green values
// serves both, with the z-odd components (xz, yz) negated for the mirror.
// Forward spectra of components 0 and 1 are parked in registers, component 2
// stays in LDS.
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_zpass(const int *__restrict__ mask, cpx<T> *__restrict__ B, size_t b_elems,
                                                const cpx<T> *__restrict__ ghat, const cpx<T> *__restrict__ twz,
                                                AxisPlan pz, int Mx, int My, int nz, int nxt, int Mxh, int Myh,
                                                size_t moct) {
  constexpr int W = kW<T>;
  constexpr int NQ = EPT / 2 + 1;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mz = pz.L;
  const int n = Mz * W;
  const int nq = (Mz / 2 + 1) * W;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + n;
  load_twiddles(tw, twz, Mz);
  const int b = blockIdx.x;
  const int xt = b % nxt, ky = b / nxt;
  cpx<T> *tile = B + (size_t)r * b_elems + (((size_t)ky * nxt + xt) * 3) * nz * W;
  cpx<T> a0[NQ], b0[NQ], a1[NQ], b1[NQ];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cpx<T> *src = tile + (size_t)c * nz * W;
    stage_in<T, EPT>(buf, n, [&](int e) { return e < nz * W ? src[e] : cpx<T>{0, 0}; });
    __syncthreads();
    fft_lds<T, EPT, -1>(buf, tw, pz, W, 1, W, true);
    if (c < 2) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int q = threadIdx.x + i * kNT;
        if (q < nq) {
          const int oz = q / W, p = q % W;
          const bool mir = oz != 0 && 2 * oz != Mz;
          const cpx<T> va = buf[q];
          const cpx<T> vb = mir ? buf[(Mz - oz) * W + p] : cpx<T>{0, 0};
          if (c == 0) { a0[i] = va; b0[i] = vb; }
          else { a1[i] = va; b1[i] = vb; }
        }
      }
      __syncthreads();
    }
  }
  int sy;
  const int oy = fold(ky, My, sy);
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + i * kNT;
    if (q < nq) {
      const int oz = q / W, p = q % W, kx = xt * W + p;
      const bool mir = oz != 0 && 2 * oz != Mz;
      const int zb = (Mz - oz) * W + p;
      cpx<T> qa0 = {0, 0}, qa1 = {0, 0}, qa2 = {0, 0}, qb0 = {0, 0}, qb1 = {0, 0}, qb2 = {0, 0};
      if (kx < Mx) {
        int sx;
        const int ox = fold(kx, Mx, sx);
        const cpx<T> *g = ghat + ((size_t)oz * Myh + oy) * Mxh + ox;
        const cpx<T> gxx = g[0], gyy = g[moct], gzz = g[2 * moct];
        const cpx<T> gxy = T(sx * sy) * g[3 * moct], gxz = T(sx) * g[4 * moct], gyz = T(sy) * g[5 * moct];
        const cpx<T> a2 = buf[q];
        qa0 = gxx * a0[i] + gxy * a1[i] + gxz * a2;
        qa1 = gxy * a0[i] + gyy * a1[i] + gyz * a2;
        qa2 = gxz * a0[i] + gyz * a1[i] + gzz * a2;
        if (mir) {
          const cpx<T> b2 = buf[zb];
          qb0 = gxx * b0[i] + gxy * b1[i] - gxz * b2;
          qb1 = gxy * b0[i] + gyy * b1[i] - gyz * b2;
          qb2 = gzz * b2 - gxz * b0[i] - gyz * b1[i];
        }
      }
      a0[i] = qa0;
      a1[i] = qa1;
      buf[q] = qa2;
      if (mir) {
        b0[i] = qb0;
        b1[i] = qb1;
        buf[zb] = qb2;
      }
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
          const int oz = q / W, p = q % W;
          buf[q] = c == 0 ? a0[i] : a1[i];
          if (oz != 0 && 2 * oz != Mz) buf[(Mz - oz) * W + p] = c == 0 ? b0[i] : b1[i];
        }
      }
      __syncthreads();
    }
    fft_lds<T, EPT, +1>(buf, tw, pz, W, 1, W, true);
    cpx<T> *dst = tile + (size_t)c * nz * W;
    for (int e = threadIdx.x; e < nz * W; e += kNT) dst[e] = buf[e];
    __syncthreads();
  }
}

// --------------------------------------------------------------- y-inverse --
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_yinv(const int *__restrict__ mask, const cpx<T> *__restrict__ B,
                                               size_t b_elems, cpx<T> *__restrict__ A, size_t a_elems,
                                               const cpx<T> *__restrict__ twy, AxisPlan py, int ny, int nz,
                                               int nxt) {
  constexpr int W = kW<T>;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = py.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + My * W;
  load_twiddles(tw, twy, My);
  const int b = blockIdx.x;
  const int xt = b % nxt, cz = b / nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *Br = B + (size_t)r * b_elems;
  stage_in<T, EPT>(buf, My * W, [&](int e) {
    const int ky = e / W, p = e % W;
    return Br[((((size_t)ky * nxt + xt) * 3 + c) * nz + z) * W + p];
  });
  __syncthreads();
  fft_lds<T, EPT, +1>(buf, tw, py, W, 1, W, true);
  cpx<T> *dst = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * ny * W;
  for (int e = threadIdx.x; e < ny * W; e += kNT) dst[e] = buf[e];
}

// --------------------------------------------------------------- x-inverse --
// f.out_mode (see FuseArgs): 0 only writes out = ainv * in - G*in; 1 and 2 also
// write per-block partial sums of the BiCGSTAB inner products of `out`.
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_xinv(const c64 *__restrict__ in, c64 *__restrict__ out, int64_t n3,
                                               const int *__restrict__ mask, const c64 *__restrict__ ainv,
                                               int ncomp, const uint8_t *__restrict__ comp,
                                               const int *__restrict__ cell_site, const cpx<T> *__restrict__ A,
                                               size_t a_elems, const cpx<T> *__restrict__ twx, AxisPlan px,
                                               int nx, int ny, int nz, int nxt, int nrows, FuseArgs f) {
  constexpr int W = kW<T>;
  constexpr int NE = (EPT + 2) / 3;
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = px.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * nrows * Mx;
  load_twiddles(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, ny * nz - row0);
  const cpx<T> *Ar = A + (size_t)r * a_elems;
  stage_in<T, EPT>(buf, 3 * nrows * Mx, [&](int e) {
    const int pq = e / Mx, kx = e - pq * Mx;
    const int c = pq / nrows, q = pq - c * nrows;
    cpx<T> v = {0, 0};
    if (q < nrow) {
      const int row = row0 + q, z = row / ny, y = row - z * ny;
      const int xt = kx / W, p = kx % W;
      v = Ar[((((size_t)c * nz + z) * nxt + xt) * ny + y) * W + p];
    }
    return v;
  });
  __syncthreads();
  fft_lds<T, EPT, +1>(buf, tw, px, 3 * nrows, Mx, 1, false);
  const size_t off = (size_t)r * n3;
  const c64 *ai = ainv + (size_t)r * ncomp;
  const int ne = nrow * nx;
  int site[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = threadIdx.x + i * kNT;
    site[i] = -1;
    if (e < ne) {
      const int q = e / nx, x = e - q * nx;
      site[i] = cell_site[(size_t)(row0 + q) * nx + x];
    }
  }
  c64 pv[NE][3];
#pragma unroll
  for (int i = 0; i < NE; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[i][c] = site[i] >= 0 ? in[off + (size_t)3 * site[i] + c] : c64{0, 0};
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (site[i] >= 0) {
      const int q = e / nx, x = e - q * nx;
      const c64 a = ai[comp ? comp[site[i]] : 0];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t j = off + (size_t)3 * site[i] + c;
        const cpx<T> fv = buf[(c * nrows + q) * Mx + x];
        const c64 d = a * pv[i][c];
        const c64 o = c64{d.x - double(fv.x), d.y - double(fv.y)};
        out[j] = o;
        if (f.out_mode == 1) {
          const c64 g = cmulc(f.rh[j], o);
          acc[0] += g.x;
          acc[1] += g.y;
        } else if (f.out_mode == 2) {
          const c64 g = cmulc(o, pv[i][c]);
          acc[0] += g.x;
          acc[1] += g.y;
          acc[2] += o.x * o.x + o.y * o.y;
        }
      }
    }
  }
  if (f.out_mode != 0) {
    // one partial record per block; a one-block kernel adds them in block order
    double tot[3];
    block_sum<3, kNT>(acc, tot);
    if (threadIdx.x == 0) {
      double *o = f.partial + ((size_t)r * gridDim.x + blockIdx.x) * kPart;
      o[0] = tot[0];
      o[1] = tot[1];
      o[2] = tot[2];
    }
  }
}

// --------------------------------------------------------------- launchers --
// Register arrays are sized by EPT = elements per thread (a compile-time
// bound, one kernel instantiation per size).
static inline int pick_ept(size_t elems) {
  static const int opts[] = {4, 8, 12, 16, 20, 24, 32};
  for (int e : opts)
    if ((size_t)e * kNT >= elems) return e;
  throw Error{DDA_ENOTSUP, "FFT tile too large for one block"};
}

#define DDA_EPT_SWITCH(ept, BODY)                       \
  switch (ept) {                                        \
    case 4: { constexpr int E = 4; BODY; } break;       \
    case 8: { constexpr int E = 8; BODY; } break;       \
    case 12: { constexpr int E = 12; BODY; } break;     \
    case 16: { constexpr int E = 16; BODY; } break;     \
    case 20: { constexpr int E = 20; BODY; } break;     \
    case 24: { constexpr int E = 24; BODY; } break;     \
    default: { constexpr int E = 32; BODY; } break;     \
  }

#define DDA_EPT_SWITCH_X(ept, BODY)                     \
  switch (ept) {                                        \
    case 4: { constexpr int E = 4; BODY; } break;       \
    default: { constexpr int E = 8; BODY; } break;      \
  }

template <typename K>
static inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) DDA_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

static inline int rows_per_block(int Mx) { return xpass_rows(Mx); }

template <typename T>
void launch_matvec(const Geometry &g, const MatvecArgs &a, hipStream_t s, const hipEvent_t *ev, int only_pass,
                   int reps) {
  const bool f32 = sizeof(T) == 4;
  const int nxt = g.nxt(f32);
  const size_t ae = g.a_elems(f32), be = g.b_elems(f32);
  cpx<T> *A = static_cast<cpx<T> *>(a.bufA);
  cpx<T> *B = static_cast<cpx<T> *>(a.bufB);
  const cpx<T> *twx = static_cast<const cpx<T> *>(a.twx);
  const cpx<T> *twy = static_cast<const cpx<T> *>(a.twy);
  const cpx<T> *twz = static_cast<const cpx<T> *>(a.twz);
  const int64_t n3 = 3 * g.n_sites;
  const int nrows = rows_per_block(g.Mx);
  const int nrowblk = (g.ny * g.nz + nrows - 1) / nrows;
  const size_t cs = sizeof(cpx<T>);
  constexpr int W = kW<T>;
  const FuseArgs &f = a.fuse;
  auto pass = [&](int k) {
    switch (k) {
      case 0: {
        const size_t elems = (size_t)3 * nrows * g.Mx;
        const size_t lds = (elems + g.Mx) * cs;
        DDA_EPT_SWITCH_X(pick_ept(elems), {
          hipLaunchKernelGGL((k_xfwd<T, E>), dim3(nrowblk, a.nrhs), dim3(kNT), lds, s, a.in, n3, a.mask,
                             a.cell_site, A, ae, twx, a.px, g.nx, g.ny, g.nz, nxt, nrows, f);
        });
      } break;
      case 1: {
        const size_t elems = (size_t)g.My * W;
        const size_t lds = (elems + g.My) * cs;
        DDA_EPT_SWITCH(pick_ept(elems), {
          allow_lds(k_yfwd<T, E>, lds);
          hipLaunchKernelGGL((k_yfwd<T, E>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, A, ae, B, be,
                             twy, a.py, g.ny, g.nz, nxt);
        });
      } break;
      case 2: {
        const size_t elems = (size_t)g.Mz * W;
        const size_t lds = (elems + g.Mz) * cs;
        DDA_EPT_SWITCH(pick_ept(elems), {
          allow_lds(k_zpass<T, E>, lds);
          hipLaunchKernelGGL((k_zpass<T, E>), dim3(g.My * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, B, be,
                             static_cast<const cpx<T> *>(a.ghat), twz, a.pz, g.Mx, g.My, g.nz, nxt, g.Mxh, g.Myh,
                             g.oct_elems());
        });
      } break;
      case 3: {
        const size_t elems = (size_t)g.My * W;
        const size_t lds = (elems + g.My) * cs;
        DDA_EPT_SWITCH(pick_ept(elems), {
          allow_lds(k_yinv<T, E>, lds);
          hipLaunchKernelGGL((k_yinv<T, E>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, B, be, A, ae,
                             twy, a.py, g.ny, g.nz, nxt);
        });
      } break;
      default: {
        const size_t elems = (size_t)3 * nrows * g.Mx;
        const size_t lds = (elems + g.Mx) * cs;
        DDA_EPT_SWITCH_X(pick_ept(elems), {
          hipLaunchKernelGGL((k_xinv<T, E>), dim3(nrowblk, a.nrhs), dim3(kNT), lds, s, a.in, a.out, n3, a.mask,
                             a.ainv, a.ncomp, a.comp, a.cell_site, A, ae, twx, a.px, g.nx, g.ny, g.nz, nxt, nrows,
                             f);
        });
      } break;
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
