// Far-field averages of a solved polarization: C_sca by quadrature over
// scattering directions, <cos theta> and <cos^2 theta> (the §3.1 outputs of
// the DDSCAT 7.3 guide; the angular resolution is its ETASCA parameter, §9).
//
// The scattered far field in direction n (|E_0| = 1, d = 1) is, up to the
// outgoing spherical wave, k^2 (I - n n) F(n) with
//     F(n) = sum_j P_j exp(-i k n . r_j),
// so C_sca = k^4 * integral |F_perp(n)|^2 dOmega and the averages are weighted
// by |F_perp|^2 with cos theta = n . khat.  Directions: Gauss-Legendre nodes
// mu_i in cos theta about khat (n_theta of them) times 2 n_theta uniform phi.
//
// F is summed over the box cell by cell along x: the phase of the row start
// comes from one sincos, each step in x multiplies it by exp(-i k n_x).  One
// thread per direction; the cell index and P are the same for every thread of
// the block (uniform loads).  The rows are split into chunks over blocks;
// the partial sums are added per direction in chunk order, then the weighted
// intensities per block and the block records in block order, so the result
// is deterministic.

#include <algorithm>
#include <cmath>

#include "dda_internal.hpp"
#include "reduce.hpp"

namespace dda {

constexpr int kFT = 256;

__global__ __launch_bounds__(kFT) void kf_partial(const int *__restrict__ cell_site, int nx, int ny, int nrows,
                                                  int rows_per_chunk, const c64 *__restrict__ P, double kd,
                                                  const double *__restrict__ dirs, int ndir,
                                                  double *__restrict__ fpart) {
  const int d = blockIdx.x * kFT + threadIdx.x;
  const bool live = d < ndir;
  const double n0 = live ? dirs[3 * d] : 0.0, n1 = live ? dirs[3 * d + 1] : 0.0, n2 = live ? dirs[3 * d + 2] : 0.0;
  double sa, ca;
  sincos(kd * n0, &sa, &ca);
  const c64 step = {ca, -sa};                       // exp(-i k n_x)
  c64 f0 = {0, 0}, f1 = {0, 0}, f2 = {0, 0};
  const int row0 = blockIdx.y * rows_per_chunk;
  const int row1 = min(row0 + rows_per_chunk, nrows);
  for (int row = row0; row < row1; ++row) {
    const int z = row / ny, y = row - z * ny;
    double sp, cp;
    sincos(kd * (n1 * y + n2 * z), &sp, &cp);
    c64 ph = {cp, -sp};                             // exp(-i k (n_y y + n_z z))
    const int *cs = cell_site + (size_t)row * nx;
    for (int x = 0; x < nx; ++x) {
      const int s = cs[x];
      if (s >= 0) {
        const c64 *p = P + (size_t)3 * s;
        f0 = f0 + ph * p[0];
        f1 = f1 + ph * p[1];
        f2 = f2 + ph * p[2];
      }
      ph = ph * step;
    }
  }
  if (live) {
    double *o = fpart + ((size_t)blockIdx.y * ndir + d) * 6;
    o[0] = f0.x;
    o[1] = f0.y;
    o[2] = f1.x;
    o[3] = f1.y;
    o[4] = f2.x;
    o[5] = f2.y;
  }
}

// Per direction: F = sum of the chunk partials; I = w |F - n (n . F)|^2; block
// records of sum I, sum mu I, sum mu^2 I.
__global__ __launch_bounds__(kFT) void kf_intensity(const double *__restrict__ fpart, int nchunk,
                                                    const double *__restrict__ dirs, const double *__restrict__ mu,
                                                    const double *__restrict__ w, int ndir,
                                                    double *__restrict__ rec) {
  const int d = blockIdx.x * kFT + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  if (d < ndir) {
    double f[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < nchunk; ++c) {
      const double *q = fpart + ((size_t)c * ndir + d) * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) f[k] += q[k];
    }
    const double n[3] = {dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2]};
    const double dre = n[0] * f[0] + n[1] * f[2] + n[2] * f[4];
    const double dim = n[0] * f[1] + n[1] * f[3] + n[2] * f[5];
    double i2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double re = f[2 * a] - n[a] * dre, im = f[2 * a + 1] - n[a] * dim;
      i2 += re * re + im * im;
    }
    const double wi = w[d] * i2;
    acc[0] = wi;
    acc[1] = mu[d] * wi;
    acc[2] = mu[d] * mu[d] * wi;
  }
  double out[3];
  block_sum<3, kFT>(acc, out);
  if (threadIdx.x == 0) write_record<3>(rec, 0, gridDim.x, blockIdx.x, out);
}

__global__ __launch_bounds__(kFT) void kf_final(const double *__restrict__ rec, int nblk, double *__restrict__ sums) {
  double s[3];
  sum_records<3, kFT>(rec, nblk, 0, s);
  if (threadIdx.x == 0) {
    sums[0] = s[0];
    sums[1] = s[1];
    sums[2] = s[2];
  }
}

// F[d] = sum over chunks of the partial sums (chunk order): the phase sums
// F(n_d) = sum_j P_j exp(-i k n_d . r_j), 3 complex values per direction
__global__ __launch_bounds__(kFT) void kf_collect(const double *__restrict__ fpart, int nchunk, int ndir,
                                                  double *__restrict__ F) {
  const int d = blockIdx.x * kFT + threadIdx.x;
  if (d >= ndir) return;
  double f[6] = {0, 0, 0, 0, 0, 0};
  for (int c = 0; c < nchunk; ++c) {
    const double *q = fpart + ((size_t)c * ndir + d) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] += q[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) F[(size_t)d * 6 + k] = f[k];
}

size_t far_field_scratch_bytes(const Geometry &g, int ndir) {
  const int dblk = (ndir + kFT - 1) / kFT;
  const int nrows = g.ny * g.nz;
  const int nchunk = std::min(nrows, std::max(1, (2048 + dblk - 1) / dblk));
  return (size_t)nchunk * ndir * 6 * sizeof(double) + (size_t)dblk * kPart * sizeof(double) + 3 * sizeof(double);
}

void launch_far_field(const Geometry &g, const int *cell_site, const c64 *P, double kd, const double *dirs,
                      const double *mu, const double *w, int ndir, double *scratch, double *sums, hipStream_t s) {
  const int dblk = (ndir + kFT - 1) / kFT;
  const int nrows = g.ny * g.nz;
  int nchunk = std::min(nrows, std::max(1, (2048 + dblk - 1) / dblk));
  const int rpc = (nrows + nchunk - 1) / nchunk;
  nchunk = (nrows + rpc - 1) / rpc;
  double *fpart = scratch;
  double *rec = scratch + (size_t)nchunk * ndir * 6;
  hipLaunchKernelGGL(kf_partial, dim3(dblk, nchunk), dim3(kFT), 0, s, cell_site, g.nx, g.ny, nrows, rpc, P, kd, dirs,
                     ndir, fpart);
  hipLaunchKernelGGL(kf_intensity, dim3(dblk), dim3(kFT), 0, s, fpart, nchunk, dirs, mu, w, ndir, rec);
  hipLaunchKernelGGL(kf_final, dim3(1), dim3(kFT), 0, s, rec, dblk, sums);
  DDA_HIP(hipGetLastError());
}

void launch_far_amplitudes(const Geometry &g, const int *cell_site, const c64 *P, double kd, const double *dirs,
                           int ndir, double *scratch, double *F, hipStream_t s) {
  const int dblk = (ndir + kFT - 1) / kFT;
  const int nrows = g.ny * g.nz;
  int nchunk = std::min(nrows, std::max(1, (2048 + dblk - 1) / dblk));
  const int rpc = (nrows + nchunk - 1) / nchunk;
  nchunk = (nrows + rpc - 1) / rpc;
  hipLaunchKernelGGL(kf_partial, dim3(dblk, nchunk), dim3(kFT), 0, s, cell_site, g.nx, g.ny, nrows, rpc, P, kd, dirs,
                     ndir, scratch);
  hipLaunchKernelGGL(kf_collect, dim3(dblk), dim3(kFT), 0, s, scratch, nchunk, ndir, F);
  DDA_HIP(hipGetLastError());
}

}  // namespace dda
