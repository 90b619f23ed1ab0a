// Near field (§29 of the DDSCAT 7.3 guide): the field at every lattice point
// of an extended box, E(q) = E_inc(q) + sum_{l, r_l != q} G(r_q - r_l) P_l.
// The sum is the FFT product of a target that occupies the whole extended box
// with P embedded (zero at vacuum points) and a zero diagonal: there
// A P_ext = -G * P_ext, so E = E_inc - A P_ext.  These kernels embed P and
// form E (with the optional macroscopic factor 3 / (eps + 2) inside the
// target).

#include <algorithm>

#include "dda_internal.hpp"
#include "nearfield.hpp"

namespace dda {

// P_ext[r][map[i]] = P[r][i]  (P_ext zeroed beforehand)
__global__ void kn_embed(const c64 *__restrict__ P, int64_t n, const int *__restrict__ map, c64 *__restrict__ Pext,
                         int64_t ne) {
  const int r = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const c64 *src = P + ((size_t)r * n + i) * 3;
    c64 *dst = Pext + ((size_t)r * ne + map[i]) * 3;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
  }
}

// E = E_inc - AP at extended point j = (z Y + y) X + x, site coordinate
// (x, y, z) - margin; cellc[j] >= 0: composition of the occupied site there
__global__ void kn_field(const c64 *__restrict__ AP, int64_t ne, int X, int Y, int mx, int my, int mz,
                         const RhsDev *__restrict__ rhs, double kd, const int *__restrict__ cellc,
                         const c64 *__restrict__ fac, c64 *__restrict__ E) {
  const int r = blockIdx.y;
  const RhsDev R = rhs[r];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ne; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t xy = (int64_t)X * Y;
    const int z = (int)(j / xy);
    const int64_t rem = j - (int64_t)z * xy;
    const int y = (int)(rem / X), x = (int)(rem - (int64_t)y * X);
    const double ph = kd * (R.khat[0] * (x - mx) + R.khat[1] * (y - my) + R.khat[2] * (z - mz));
    double sn, cs;
    sincos(ph, &sn, &cs);
    const c64 w = {cs, sn};
    const c64 *ap = AP + ((size_t)r * ne + j) * 3;
    c64 *o = E + ((size_t)r * ne + j) * 3;
    const int c = cellc[j];
    const c64 f = (fac && c >= 0) ? fac[c] : c64{1.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const c64 v = w * R.e[a] - ap[a];
      o[a] = f * v;
    }
  }
}

void launch_near_field_embed(const c64 *P, int64_t n, const int *map, c64 *Pext, int64_t ne, int nrhs,
                             hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(kn_embed, dim3(nb, nrhs), dim3(256), 0, s, P, n, map, Pext, ne);
  DDA_HIP(hipGetLastError());
}

void launch_near_field_combine(const c64 *AP, int64_t ne, int X, int Y, const int margin[3], const RhsDev *rhs,
                               int nrhs, double kd, const int *cellc, const c64 *fac, c64 *E, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>((ne + 255) / 256, 4096);
  hipLaunchKernelGGL(kn_field, dim3(nb, nrhs), dim3(256), 0, s, AP, ne, X, Y, margin[0], margin[1], margin[2], rhs,
                     kd, cellc, fac, E);
  DDA_HIP(hipGetLastError());
}

// ------------------------------------------------------- magnetic field --
__global__ void kb_embed(const c64 *__restrict__ P, int64_t n, const int64_t *__restrict__ mapM,
                         c64 *__restrict__ full, int64_t M) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = mapM[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) full[c * M + j] = P[i * 3 + c];
  }
}

__global__ void kb_cross(const c64 *__restrict__ h, c64 *__restrict__ full, int64_t M, double scale) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    const c64 hx = h[j], hy = h[M + j], hz = h[2 * M + j];
    const c64 px = full[j], py = full[M + j], pz = full[2 * M + j];
    full[j] = scale * (hy * pz - hz * py);
    full[M + j] = scale * (hz * px - hx * pz);
    full[2 * M + j] = scale * (hx * py - hy * px);
  }
}

// B_inc = khat x e exp(ik khat . r) plus the convolution at cell (z, y, x)
__global__ void kb_field(const c64 *__restrict__ full, int64_t M, int Mx, int My, int X, int Y, int64_t ne, int mx,
                         int my, int mz, const RhsDev *__restrict__ rhs, double kd, c64 *__restrict__ B) {
  const RhsDev R = rhs[0];
  const c64 bi[3] = {R.khat[1] * R.e[2] - R.khat[2] * R.e[1], R.khat[2] * R.e[0] - R.khat[0] * R.e[2],
                     R.khat[0] * R.e[1] - R.khat[1] * R.e[0]};
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ne; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t xy = (int64_t)X * Y;
    const int z = (int)(j / xy);
    const int64_t rem = j - (int64_t)z * xy;
    const int y = (int)(rem / X), x = (int)(rem - (int64_t)y * X);
    const double ph = kd * (R.khat[0] * (x - mx) + R.khat[1] * (y - my) + R.khat[2] * (z - mz));
    double sn, cs;
    sincos(ph, &sn, &cs);
    const c64 w = {cs, sn};
    const int64_t cell = ((int64_t)z * My + y) * Mx + x;
#pragma unroll
    for (int a = 0; a < 3; ++a) B[j * 3 + a] = w * bi[a] + full[a * M + cell];
  }
}

void launch_magnetic_embed(const c64 *P, int64_t n, const int64_t *mapM, c64 *full, int64_t M, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
  hipLaunchKernelGGL(kb_embed, dim3(nb), dim3(256), 0, s, P, n, mapM, full, M);
  DDA_HIP(hipGetLastError());
}

void launch_magnetic_cross(const c64 *h, c64 *full, int64_t M, double scale, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<int64_t>((M + 255) / 256, 8192);
  hipLaunchKernelGGL(kb_cross, dim3(nb), dim3(256), 0, s, h, full, M, scale);
  DDA_HIP(hipGetLastError());
}

void launch_magnetic_field(const c64 *full, const Geometry &g, int X, int Y, int64_t ne, const int margin[3],
                           const RhsDev *rhs, double kd, c64 *B, hipStream_t s) {
  const int64_t M = (int64_t)g.Mx * g.My * g.Mz;
  const unsigned nb = (unsigned)std::min<int64_t>((ne + 255) / 256, 4096);
  hipLaunchKernelGGL(kb_field, dim3(nb), dim3(256), 0, s, full, M, g.Mx, g.My, X, Y, ne, margin[0], margin[1],
                     margin[2], rhs, kd, B);
  DDA_HIP(hipGetLastError());
}

}  // namespace dda
