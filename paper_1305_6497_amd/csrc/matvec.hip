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

#include <algorithm>

#include "dda_internal.hpp"
#include "fft_lds.hpp"

namespace dda {

extern __shared__ __align__(16) unsigned char dda_smem[];

template <typename T>
__device__ __forceinline__ cpx<T> to_t(c64 v) { return {T(v.x), T(v.y)}; }

// --------------------------------------------------------------- x-forward --
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_xfwd(const c64 *__restrict__ in, int64_t n3, const int *__restrict__ mask,
                                               const int *__restrict__ cell_site, cpx<T> *__restrict__ A,
                                               size_t a_elems, const cpx<T> *__restrict__ twx, AxisPlan px,
                                               int nx, int ny, int nz, int nxt, int W, int nrows) {
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = px.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * nrows * Mx;
  load_twiddles(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, ny * nz - row0);
  const c64 *P = in + (size_t)r * n3;
  for (int e = threadIdx.x; e < nrows * Mx; e += kNT) {
    const int q = e / Mx, x = e - q * Mx;
    cpx<T> v0 = {0, 0}, v1 = {0, 0}, v2 = {0, 0};
    if (q < nrow && x < nx) {
      const int site = cell_site[(size_t)(row0 + q) * nx + x];
      if (site >= 0) {
        const c64 *ps = P + (size_t)3 * site;
        v0 = to_t<T>(ps[0]);
        v1 = to_t<T>(ps[1]);
        v2 = to_t<T>(ps[2]);
      }
    }
    buf[(0 * nrows + q) * Mx + x] = v0;
    buf[(1 * nrows + q) * Mx + x] = v1;
    buf[(2 * nrows + q) * Mx + x] = v2;
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
      const int xt = kx / W, p = kx - xt * W;
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
                                               int nxt, int W) {
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = py.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + My * W;
  load_twiddles(tw, twy, My);
  const int b = blockIdx.x;
  const int xt = b % nxt, cz = b / nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *src = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * ny * W;
  for (int e = threadIdx.x; e < My * W; e += kNT) {
    const int y = e / W;
    buf[e] = y < ny ? src[e] : cpx<T>{0, 0};
  }
  __syncthreads();
  fft_lds<T, EPT, -1>(buf, tw, py, W, 1, W, true);
  cpx<T> *Br = B + (size_t)r * b_elems;
  for (int e = threadIdx.x; e < My * W; e += kNT) {
    const int ky = e / W, p = e - ky * W;
    Br[((((size_t)ky * nxt + xt) * 3 + c) * nz + z) * W + p] = buf[e];
  }
}

// ------------------------------------------------------------------ z-pass --
template <typename T>
__device__ __forceinline__ int fold(int k, int M, int &sgn) {
  if (2 * k <= M) { sgn = 1; return k; }
  sgn = -1;
  return M - k;
}

template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_zpass(const int *__restrict__ mask, cpx<T> *__restrict__ B, size_t b_elems,
                                                const cpx<T> *__restrict__ ghat, const cpx<T> *__restrict__ twz,
                                                AxisPlan pz, int Mx, int My, int nz, int nxt, int W, int Mxh,
                                                int Myh, size_t moct) {
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mz = pz.L;
  const int n = Mz * W;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + n;
  load_twiddles(tw, twz, Mz);
  const int b = blockIdx.x;
  const int xt = b % nxt, ky = b / nxt;
  cpx<T> *tile = B + (size_t)r * b_elems + (((size_t)ky * nxt + xt) * 3) * nz * W;
  cpx<T> s0[EPT], s1[EPT];
  // forward transforms of components 0 and 1 are parked in registers,
  // component 2 stays in LDS.
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cpx<T> *src = tile + (size_t)c * nz * W;
    for (int e = threadIdx.x; e < n; e += kNT) {
      const int z = e / W;
      buf[e] = z < nz ? src[e] : cpx<T>{0, 0};
    }
    __syncthreads();
    fft_lds<T, EPT, -1>(buf, tw, pz, W, 1, W, true);
    if (c < 2) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) {
          if (c == 0) s0[i] = buf[e];
          else s1[i] = buf[e];
        }
      }
      __syncthreads();
    }
  }
  int sy;
  const int oy = fold<T>(ky, My, sy);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kNT;
    if (e < n) {
      const int kz = e / W, p = e - kz * W, kx = xt * W + p;
      cpx<T> q0 = {0, 0}, q1 = {0, 0}, q2 = {0, 0};
      if (kx < Mx) {
        int sx, sz;
        const int ox = fold<T>(kx, Mx, sx);
        const int oz = fold<T>(kz, Mz, sz);
        const cpx<T> *g = ghat + ((size_t)oz * Myh + oy) * Mxh + ox;
        const cpx<T> gxx = g[0], gyy = g[moct], gzz = g[2 * moct];
        cpx<T> gxy = g[3 * moct], gxz = g[4 * moct], gyz = g[5 * moct];
        const T fxy = T(sx * sy), fxz = T(sx * sz), fyz = T(sy * sz);
        gxy = fxy * gxy;
        gxz = fxz * gxz;
        gyz = fyz * gyz;
        const cpx<T> a0 = s0[i], a1 = s1[i], a2 = buf[e];
        q0 = gxx * a0 + gxy * a1 + gxz * a2;
        q1 = gxy * a0 + gyy * a1 + gyz * a2;
        q2 = gxz * a0 + gyz * a1 + gzz * a2;
      }
      s0[i] = q0;
      s1[i] = q1;
      buf[e] = q2;
    }
  }
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const int c = (cc + 2) % 3;     // 2, 0, 1
    if (c != 2) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * kNT;
        if (e < n) buf[e] = (c == 0) ? s0[i] : s1[i];
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
                                               int nxt, int W) {
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int My = py.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + My * W;
  load_twiddles(tw, twy, My);
  const int b = blockIdx.x;
  const int xt = b % nxt, cz = b / nxt, c = cz / nz, z = cz - c * nz;
  const cpx<T> *Br = B + (size_t)r * b_elems;
  for (int e = threadIdx.x; e < My * W; e += kNT) {
    const int ky = e / W, p = e - ky * W;
    buf[e] = Br[((((size_t)ky * nxt + xt) * 3 + c) * nz + z) * W + p];
  }
  __syncthreads();
  fft_lds<T, EPT, +1>(buf, tw, py, W, 1, W, true);
  cpx<T> *dst = A + (size_t)r * a_elems + (((size_t)c * nz + z) * nxt + xt) * ny * W;
  for (int e = threadIdx.x; e < ny * W; e += kNT) dst[e] = buf[e];
}

// --------------------------------------------------------------- x-inverse --
template <typename T, int EPT>
__global__ __launch_bounds__(kNT) void k_xinv(const c64 *__restrict__ in, c64 *__restrict__ out, int64_t n3,
                                               const int *__restrict__ mask, const c64 *__restrict__ ainv,
                                               int ncomp, const uint8_t *__restrict__ comp,
                                               const int *__restrict__ cell_site, const cpx<T> *__restrict__ A,
                                               size_t a_elems, const cpx<T> *__restrict__ twx, AxisPlan px,
                                               int nx, int ny, int nz, int nxt, int W, int nrows) {
  const int r = blockIdx.y;
  if (mask && !mask[r]) return;
  const int Mx = px.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + 3 * nrows * Mx;
  load_twiddles(tw, twx, Mx);
  const int row0 = blockIdx.x * nrows;
  const int nrow = min(nrows, ny * nz - row0);
  const cpx<T> *Ar = A + (size_t)r * a_elems;
  for (int e = threadIdx.x; e < 3 * nrows * Mx; e += kNT) {
    const int pq = e / Mx, kx = e - pq * Mx;
    const int c = pq / nrows, q = pq - c * nrows;
    cpx<T> v = {0, 0};
    if (q < nrow) {
      const int row = row0 + q, z = row / ny, y = row - z * ny;
      const int xt = kx / W, p = kx - xt * W;
      v = Ar[((((size_t)c * nz + z) * nxt + xt) * ny + y) * W + p];
    }
    buf[e] = v;
  }
  __syncthreads();
  fft_lds<T, EPT, +1>(buf, tw, px, 3 * nrows, Mx, 1, false);
  const c64 *P = in + (size_t)r * n3;
  c64 *Q = out + (size_t)r * n3;
  const c64 *ai = ainv + (size_t)r * ncomp;
  for (int e = threadIdx.x; e < nrow * nx; e += kNT) {
    const int q = e / nx, x = e - q * nx;
    const int site = cell_site[(size_t)(row0 + q) * nx + x];
    if (site >= 0) {
      const c64 a = ai[comp ? comp[site] : 0];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cpx<T> f = buf[(c * nrows + q) * Mx + x];
        const c64 pv = P[(size_t)3 * site + c];
        const c64 d = a * pv;
        Q[(size_t)3 * site + c] = c64{d.x - double(f.x), d.y - double(f.y)};
      }
    }
  }
}

// ------------------------------------------------- generic batched FFTs --
// Contiguous rows of length L (in may equal out).
template <typename T, int EPT, int DIR>
__global__ __launch_bounds__(kNT) void k_fft_rows(const cpx<T> *in, cpx<T> *out, int64_t batch, AxisPlan pl,
                                                   const cpx<T> *__restrict__ twg, int np, T scale) {
  const int L = pl.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + np * L;
  load_twiddles(tw, twg, L);
  const int64_t row0 = (int64_t)blockIdx.x * np;
  const int64_t rem = batch - row0;
  const int nvalid = rem < np ? (int)rem : np;
  for (int e = threadIdx.x; e < np * L; e += kNT) {
    const int q = e / L;
    buf[e] = q < nvalid ? in[row0 * L + e] : cpx<T>{0, 0};
  }
  __syncthreads();
  fft_lds<T, EPT, DIR>(buf, tw, pl, np, L, 1, false);
  for (int e = threadIdx.x; e < nvalid * L; e += kNT) out[row0 * L + e] = scale * buf[e];
}

// Pencils of stride `inner` in an array viewed as [outer][L][inner]; a block
// takes np consecutive inner indices of one outer index.  In place.
template <typename T, int EPT, int DIR>
__global__ __launch_bounds__(kNT) void k_fft_strided(cpx<T> *data, AxisPlan pl, const cpx<T> *__restrict__ twg,
                                                      int64_t inner, int np, int tiles) {
  const int L = pl.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + np * L;
  load_twiddles(tw, twg, L);
  const int64_t o = blockIdx.x / tiles;
  const int64_t i0 = (int64_t)(blockIdx.x % tiles) * np;
  const int64_t rem = inner - i0;
  const int nvalid = rem < np ? (int)rem : np;
  cpx<T> *base = data + o * L * inner + i0;
  for (int e = threadIdx.x; e < np * L; e += kNT) {
    const int m = e / np, p = e - m * np;
    buf[e] = p < nvalid ? base[(int64_t)m * inner + p] : cpx<T>{0, 0};
  }
  __syncthreads();
  fft_lds<T, EPT, DIR>(buf, tw, pl, np, 1, np, true);
  for (int e = threadIdx.x; e < np * L; e += kNT) {
    const int m = e / np, p = e - m * np;
    if (p < nvalid) base[(int64_t)m * inner + p] = buf[e];
  }
}

// ------------------------------------------------------------ Green build --
// The six components xx, yy, zz, xy, xz, yz of the dipole field tensor
//   G = (e^{ikR}/R) [ k^2 (I - n n) + ((ikR - 1)/R^2) (I - 3 n n) ]
// at lattice offset (dx, dy, dz) placed at index (d mod M) on each axis; zero
// at the origin and where |d_i| >= n_i (the indices never reached by a pair
// of sites in the box).
__global__ void k_green_fill(c64 *__restrict__ full, int nx, int ny, int nz, int Mx, int My, int Mz, double kd) {
  const int64_t M = (int64_t)Mx * My * Mz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int x = (int)(i % Mx);
  const int y = (int)((i / Mx) % My);
  const int z = (int)(i / ((int64_t)Mx * My));
  auto delta = [](int idx, int n, int m, bool &ok) {
    if (idx < n) return idx;
    if (idx > m - n) return idx - m;
    ok = false;
    return 0;
  };
  bool ok = true;
  const int dx = delta(x, nx, Mx, ok), dy = delta(y, ny, My, ok), dz = delta(z, nz, Mz, ok);
  c64 g[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (ok && (dx | dy | dz) != 0) {
    const double R2 = double(dx) * dx + double(dy) * dy + double(dz) * dz;
    const double R = sqrt(R2);
    const double n[3] = {dx / R, dy / R, dz / R};
    double sn, cs;
    sincos(kd * R, &sn, &cs);
    const c64 pref = {cs / R, sn / R};                         // e^{ikR}/R
    const c64 c1 = (kd * kd) * pref;
    const c64 c2 = (1.0 / R2) * (pref * c64{-1.0, kd * R});   // pref (ikR - 1)/R^2
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double nn = n[ia[c]] * n[ib[c]];
      const double del = (ia[c] == ib[c]) ? 1.0 : 0.0;
      g[c] = (del - nn) * c1 + (del - 3.0 * nn) * c2;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) full[c * M + i] = g[c];
}

__global__ void k_green_octant(const c64 *__restrict__ full, c64 *__restrict__ o64, c32 *__restrict__ o32, int Mx,
                               int My, int Mz, int Mxh, int Myh, int Mzh, double scale) {
  const int64_t moct = (int64_t)Mxh * Myh * Mzh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * moct) return;
  const int c = (int)(i / moct);
  const int64_t j = i - c * moct;
  const int ox = (int)(j % Mxh);
  const int oy = (int)((j / Mxh) % Myh);
  const int oz = (int)(j / ((int64_t)Mxh * Myh));
  const int64_t M = (int64_t)Mx * My * Mz;
  const c64 v = scale * full[c * M + ((int64_t)oz * My + oy) * Mx + ox];
  o64[i] = v;
  o32[i] = c32{float(v.x), float(v.y)};
}

// --------------------------------------------------------------- launchers --
static int pick_ept(size_t elems) {
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

template <typename K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) DDA_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// Element budget per block of the row (x) passes.
template <typename T>
static int row_budget() { return sizeof(T) == 4 ? 4096 : 3072; }

template <typename T>
static int rows_per_block(int Mx) { return std::max(1, row_budget<T>() / (3 * Mx)); }

template <typename T>
void launch_matvec(const Geometry &g, const MatvecArgs &a, hipStream_t s, const hipEvent_t *ev) {
  const bool f32 = sizeof(T) == 4;
  const int W = g.W(f32), nxt = g.nxt(f32);
  const size_t ae = g.a_elems(f32), be = g.b_elems(f32);
  cpx<T> *A = static_cast<cpx<T> *>(a.bufA);
  cpx<T> *B = static_cast<cpx<T> *>(a.bufB);
  const cpx<T> *twx = static_cast<const cpx<T> *>(a.twx);
  const cpx<T> *twy = static_cast<const cpx<T> *>(a.twy);
  const cpx<T> *twz = static_cast<const cpx<T> *>(a.twz);
  const int64_t n3 = 3 * g.n_sites;
  const int nrows = rows_per_block<T>(g.Mx);
  const int nrowblk = (g.ny * g.nz + nrows - 1) / nrows;
  const size_t cs = sizeof(cpx<T>);
  auto mark = [&](int i) {
    if (ev) DDA_HIP(hipEventRecord(ev[i], s));
  };
  mark(0);
  {
    const size_t elems = (size_t)3 * nrows * g.Mx;
    const size_t lds = (elems + g.Mx) * cs;
    DDA_EPT_SWITCH(pick_ept(elems), {
      allow_lds(k_xfwd<T, E>, lds);
      hipLaunchKernelGGL((k_xfwd<T, E>), dim3(nrowblk, a.nrhs), dim3(kNT), lds, s, a.in, n3, a.mask, a.cell_site, A,
                         ae, twx, a.px, g.nx, g.ny, g.nz, nxt, W, nrows);
    });
  }
  mark(1);
  {
    const size_t elems = (size_t)g.My * W;
    const size_t lds = (elems + g.My) * cs;
    DDA_EPT_SWITCH(pick_ept(elems), {
      allow_lds(k_yfwd<T, E>, lds);
      hipLaunchKernelGGL((k_yfwd<T, E>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, A, ae, B, be, twy,
                         a.py, g.ny, g.nz, nxt, W);
    });
  }
  mark(2);
  {
    const size_t elems = (size_t)g.Mz * W;
    const size_t lds = (elems + g.Mz) * cs;
    DDA_EPT_SWITCH(pick_ept(elems), {
      allow_lds(k_zpass<T, E>, lds);
      hipLaunchKernelGGL((k_zpass<T, E>), dim3(g.My * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, B, be,
                         static_cast<const cpx<T> *>(a.ghat), twz, a.pz, g.Mx, g.My, g.nz, nxt, W, g.Mxh, g.Myh,
                         g.oct_elems());
    });
  }
  mark(3);
  {
    const size_t elems = (size_t)g.My * W;
    const size_t lds = (elems + g.My) * cs;
    DDA_EPT_SWITCH(pick_ept(elems), {
      allow_lds(k_yinv<T, E>, lds);
      hipLaunchKernelGGL((k_yinv<T, E>), dim3(3 * g.nz * nxt, a.nrhs), dim3(kNT), lds, s, a.mask, B, be, A, ae, twy,
                         a.py, g.ny, g.nz, nxt, W);
    });
  }
  mark(4);
  {
    const size_t elems = (size_t)3 * nrows * g.Mx;
    const size_t lds = (elems + g.Mx) * cs;
    DDA_EPT_SWITCH(pick_ept(elems), {
      allow_lds(k_xinv<T, E>, lds);
      hipLaunchKernelGGL((k_xinv<T, E>), dim3(nrowblk, a.nrhs), dim3(kNT), lds, s, a.in, a.out, n3, a.mask, a.ainv,
                         a.ncomp, a.comp, a.cell_site, A, ae, twx, a.px, g.nx, g.ny, g.nz, nxt, W, nrows);
    });
  }
  mark(5);
  DDA_HIP(hipGetLastError());
}

template void launch_matvec<float>(const Geometry &, const MatvecArgs &, hipStream_t, const hipEvent_t *);
template void launch_matvec<double>(const Geometry &, const MatvecArgs &, hipStream_t, const hipEvent_t *);

template <typename T>
void launch_fft_rows(const cpx<T> *in, cpx<T> *out, int64_t batch, const AxisPlan &p, const cpx<T> *tw, int dir,
                     T scale, hipStream_t s) {
  if (batch <= 0) return;
  const int np = std::max(1, row_budget<T>() / p.L);
  const int64_t nblk = (batch + np - 1) / np;
  const size_t elems = (size_t)np * p.L;
  const size_t lds = (elems + p.L) * sizeof(cpx<T>);
  DDA_EPT_SWITCH(pick_ept(elems), {
    if (dir < 0) {
      allow_lds(k_fft_rows<T, E, -1>, lds);
      hipLaunchKernelGGL((k_fft_rows<T, E, -1>), dim3((unsigned)nblk), dim3(kNT), lds, s, in, out, batch, p, tw, np,
                         scale);
    } else {
      allow_lds(k_fft_rows<T, E, 1>, lds);
      hipLaunchKernelGGL((k_fft_rows<T, E, 1>), dim3((unsigned)nblk), dim3(kNT), lds, s, in, out, batch, p, tw, np,
                         scale);
    }
  });
  DDA_HIP(hipGetLastError());
}

template void launch_fft_rows<float>(const c32 *, c32 *, int64_t, const AxisPlan &, const c32 *, int, float,
                                     hipStream_t);
template void launch_fft_rows<double>(const c64 *, c64 *, int64_t, const AxisPlan &, const c64 *, int, double,
                                      hipStream_t);

static void fft_strided_fwd64(c64 *data, const AxisPlan &p, const c64 *tw, int64_t outer, int64_t inner,
                              hipStream_t s) {
  int np = (int)std::min<int64_t>(8, inner);
  while (np > 1 && (size_t)np * p.L > (size_t)row_budget<double>()) np /= 2;
  const int tiles = (int)((inner + np - 1) / np);
  const size_t elems = (size_t)np * p.L;
  const size_t lds = (elems + p.L) * sizeof(c64);
  DDA_EPT_SWITCH(pick_ept(elems), {
    allow_lds(k_fft_strided<double, E, -1>, lds);
    hipLaunchKernelGGL((k_fft_strided<double, E, -1>), dim3((unsigned)(outer * tiles)), dim3(kNT), lds, s, data, p,
                       tw, inner, np, tiles);
  });
  DDA_HIP(hipGetLastError());
}

void launch_green_build(const Geometry &g, double kd, c64 *full, c64 *oct64, c32 *oct32, const Twiddles &tx,
                        const Twiddles &ty, const Twiddles &tz, const AxisPlan &px, const AxisPlan &py,
                        const AxisPlan &pz, hipStream_t s) {
  const int64_t M = (int64_t)g.Mx * g.My * g.Mz;
  hipLaunchKernelGGL(k_green_fill, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, full, g.nx, g.ny, g.nz, g.Mx,
                     g.My, g.Mz, kd);
  DDA_HIP(hipGetLastError());
  // x: contiguous rows; y: stride Mx; z: stride Mx*My
  launch_fft_rows<double>(full, full, 6 * (int64_t)g.Mz * g.My, px, tx.d64, -1, 1.0, s);
  fft_strided_fwd64(full, py, ty.d64, 6 * (int64_t)g.Mz, g.Mx, s);
  fft_strided_fwd64(full, pz, tz.d64, 6, (int64_t)g.Mx * g.My, s);
  const int64_t n = 6 * (int64_t)g.oct_elems();
  hipLaunchKernelGGL(k_green_octant, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, full, oct64, oct32, g.Mx,
                     g.My, g.Mz, g.Mxh, g.Myh, g.Mzh, 1.0 / double(M));
  DDA_HIP(hipGetLastError());
}

}  // namespace dda
