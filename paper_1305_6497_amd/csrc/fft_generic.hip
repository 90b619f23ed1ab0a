// Generic batched FFTs (diagnostic entry point, Green-transform build) and
// the Green-tensor table itself.
#include <algorithm>

#include "dda_internal.hpp"
#include "fft_lds.hpp"
#include "nearfield.hpp"

namespace dda {

extern __shared__ __align__(16) unsigned char dda_smem[];

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
  fft_rows<T, EPT, DIR, 0>(buf, tw, pl, np);
  for (int e = threadIdx.x; e < nvalid * L; e += kNT) out[row0 * L + e] = scale * buf[e];
}

// Pencils of stride `inner` in an array viewed as [outer][L][inner]; a block
// takes NP = 2^LOGP consecutive inner indices of one outer index.  In place.
template <typename T, int EPT, int DIR, int LOGP>
__global__ __launch_bounds__(kNT) void k_fft_strided(cpx<T> *data, AxisPlan pl, const cpx<T> *__restrict__ twg,
                                                      int64_t inner, int tiles) {
  constexpr int NP = 1 << LOGP;
  const int L = pl.L;
  cpx<T> *buf = reinterpret_cast<cpx<T> *>(dda_smem);
  cpx<T> *tw = buf + NP * L;
  load_twiddles(tw, twg, L);
  const int64_t o = blockIdx.x / tiles;
  const int64_t i0 = (int64_t)(blockIdx.x % tiles) * NP;
  const int64_t rem = inner - i0;
  const int nvalid = rem < NP ? (int)rem : NP;
  cpx<T> *base = data + o * L * inner + i0;
  for (int e = threadIdx.x; e < NP * L; e += kNT) {
    const int m = e >> LOGP, p = e & (NP - 1);
    buf[e] = p < nvalid ? base[(int64_t)m * inner + p] : cpx<T>{0, 0};
  }
  __syncthreads();
  fft_pen<T, EPT, DIR, LOGP, 0>(buf, tw, pl);
  for (int e = threadIdx.x; e < NP * L; e += kNT) {
    const int m = e >> LOGP, p = e & (NP - 1);
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

// The magnetic field of a dipole p at offset R = R n (source to point),
//   B = k^2 (e^{ikR}/R) (1 - 1/(ikR)) n x p = h(R) x p,  h = k^2 (e^{ikR}/R) (1 + i/(kR)) n,
// as the three components of h on the same periodic grid (zero at the origin
// and outside the band), so that B_sca = h (*) P is a convolution with a cross
// product in place of the matrix product.
__global__ void k_magnetic_fill(c64 *__restrict__ full, int nx, int ny, int nz, int Mx, int My, int Mz, double kd) {
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
  c64 h[3] = {{0, 0}, {0, 0}, {0, 0}};
  if (ok && (dx | dy | dz) != 0) {
    const double R = sqrt(double(dx) * dx + double(dy) * dy + double(dz) * dz);
    double sn, cs;
    sincos(kd * R, &sn, &cs);
    const c64 pref = {cs / R, sn / R};                                   // e^{ikR}/R
    const c64 f = (kd * kd) * (pref * c64{1.0, 1.0 / (kd * R)});        // k^2 e^{ikR}/R (1 + i/(kR))
    const double n[3] = {dx / R, dy / R, dz / R};
#pragma unroll
    for (int c = 0; c < 3; ++c) h[c] = n[c] * f;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) full[c * M + i] = h[c];
}

// One octant of the transformed Green tensor, scaled by 1/M, stored cell-major
// (the six components of a cell side by side) in FP64 and FP32: the z-pass
// reads a cell's six values as one contiguous 48-byte (FP32) record.
__global__ void k_green_octant(const c64 *__restrict__ full, c64 *__restrict__ o64, c32 *__restrict__ o32, int Mx,
                               int My, int Mz, int Mxh, int Myh, int Mzh, double scale) {
  const int64_t moct = (int64_t)Mxh * Myh * Mzh;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * moct) return;
  const int64_t j = i / 6;               // cell-major: value c of cell j at 6 j + c
  const int c = (int)(i - 6 * j);
  const int ox = (int)(j % Mxh);
  const int oy = (int)((j / Mxh) % Myh);
  const int oz = (int)(j / ((int64_t)Mxh * Myh));
  const int64_t M = (int64_t)Mx * My * Mz;
  const c64 v = scale * full[c * M + ((int64_t)oz * My + oy) * Mx + ox];
  o64[i] = v;
  o32[i] = c32{float(v.x), float(v.y)};
}

// ------------------------------------------------------------- launchers --
static int pick_ept_gen(size_t elems) {
  static const int opts[] = {4, 8, 16, 32};
  for (int e : opts)
    if ((size_t)e * kNT >= elems) return e;
  throw Error{DDA_ENOTSUP, "FFT tile too large for one block"};
}

#define DDA_EPT_SWITCH(ept, BODY)                       \
  switch (ept) {                                        \
    case 4: { constexpr int E = 4; BODY; } break;       \
    case 8: { constexpr int E = 8; BODY; } break;       \
    case 16: { constexpr int E = 16; BODY; } break;     \
    default: { constexpr int E = 32; BODY; } break;     \
  }

template <typename K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) DDA_HIP(hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// Element budget per block of the generic row transforms.
template <typename T>
static int row_budget() { return sizeof(T) == 4 ? 4096 : 3072; }

int xpass_blocks(const Geometry &g, bool) {
  const int nrows = xpass_rows(g.Mx);
  return (g.ny * g.nz + nrows - 1) / nrows;
}

template <typename T>
void launch_fft_rows(const cpx<T> *in, cpx<T> *out, int64_t batch, const AxisPlan &p, const cpx<T> *tw, int dir,
                     T scale, hipStream_t s) {
  if (batch <= 0) return;
  const int np = std::max(1, row_budget<T>() / p.L);
  const int64_t nblk = (batch + np - 1) / np;
  const size_t elems = (size_t)np * p.L;
  const size_t lds = (elems + p.L) * sizeof(cpx<T>);
  DDA_EPT_SWITCH(pick_ept_gen(elems), {
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

template <int DIR>
static void fft_strided64(c64 *data, const AxisPlan &p, const c64 *tw, int64_t outer, int64_t inner,
                          hipStream_t s) {
  // 8 pencils per block, 4 for the longest axes (LDS budget of row_budget)
  const bool wide = (size_t)8 * p.L <= (size_t)row_budget<double>();
  const int np = wide ? 8 : 4;
  const int tiles = (int)((inner + np - 1) / np);
  const size_t elems = (size_t)np * p.L;
  const size_t lds = (elems + p.L) * sizeof(c64);
  DDA_EPT_SWITCH(pick_ept_gen(elems), {
    if (wide) {
      allow_lds(k_fft_strided<double, E, DIR, 3>, lds);
      hipLaunchKernelGGL((k_fft_strided<double, E, DIR, 3>), dim3((unsigned)(outer * tiles)), dim3(kNT), lds, s,
                         data, p, tw, inner, tiles);
    } else {
      allow_lds(k_fft_strided<double, E, DIR, 2>, lds);
      hipLaunchKernelGGL((k_fft_strided<double, E, DIR, 2>), dim3((unsigned)(outer * tiles)), dim3(kNT), lds, s,
                         data, p, tw, inner, tiles);
    }
  });
  DDA_HIP(hipGetLastError());
}
static void fft_strided_fwd64(c64 *data, const AxisPlan &p, const c64 *tw, int64_t outer, int64_t inner,
                              hipStream_t s) {
  fft_strided64<-1>(data, p, tw, outer, inner, s);
}

void launch_fft3_full64(c64 *data, int ncomp, const Geometry &g, const Twiddles &tx, const Twiddles &ty,
                        const Twiddles &tz, const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int dir,
                        hipStream_t s) {
  // x: contiguous rows; y: stride Mx; z: stride Mx*My (unnormalised)
  launch_fft_rows<double>(data, data, (int64_t)ncomp * g.Mz * g.My, px, tx.d64, dir, 1.0, s);
  if (dir < 0) {
    fft_strided64<-1>(data, py, ty.d64, (int64_t)ncomp * g.Mz, g.Mx, s);
    fft_strided64<-1>(data, pz, tz.d64, ncomp, (int64_t)g.Mx * g.My, s);
  } else {
    fft_strided64<1>(data, py, ty.d64, (int64_t)ncomp * g.Mz, g.Mx, s);
    fft_strided64<1>(data, pz, tz.d64, ncomp, (int64_t)g.Mx * g.My, s);
  }
}

void launch_magnetic_kernel(const Geometry &g, double kd, c64 *h, const Twiddles &tx, const Twiddles &ty,
                            const Twiddles &tz, const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz,
                            hipStream_t s) {
  const int64_t M = (int64_t)g.Mx * g.My * g.Mz;
  hipLaunchKernelGGL(k_magnetic_fill, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, h, g.nx, g.ny, g.nz,
                     g.Mx, g.My, g.Mz, kd);
  DDA_HIP(hipGetLastError());
  launch_fft3_full64(h, 3, g, tx, ty, tz, px, py, pz, -1, s);
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
