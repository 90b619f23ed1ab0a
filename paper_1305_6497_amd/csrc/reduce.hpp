// Deterministic FP64 block reductions.
//
// A kernel that produces a reduction writes one partial record per block; a
// later one-block kernel adds the records in block order.  The sum order never
// depends on scheduling, so results are bit-reproducible.  (A "last block
// finishes" variant with a device-scope atomic counter was measured slower on
// this chip: the agent-scope release fence of every block writes back the
// XCD's L2.)
#pragma once

#include "dda_internal.hpp"

namespace dda {

constexpr int kPart = 8;          // doubles per partial-sum record

// Sum NV values over the block (wavefront shuffles, then across wavefronts).
// The result is valid in thread 0.  Contains a barrier.
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += __shfl_down(v[k], off, 64);
  __shared__ double sh[NV][NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += sh[k][w];
      out[k] = s;
    }
  __syncthreads();
}

// Partial-sum records: value k of block b (of nblk) for RHS r is stored at
// partial[(r * kPart + k) * nblk + b], so one kind of value is contiguous
// across blocks.
template <int NV>
__device__ __forceinline__ void write_record(double *partial, int r, int nblk, int b, const double (&v)[NV]) {
  static_assert(NV <= kPart, "record too long");
#pragma unroll
  for (int k = 0; k < NV; ++k) partial[((size_t)r * kPart + k) * nblk + b] = v[k];
}

// Sum the NV-value records [0, nblk) of RHS r in block order.  All threads of
// the block take part; the result is valid in thread 0.  Each thread adds the
// records tid, tid + NT, tid + 2 NT, ... in that order; the loads of U of them
// are issued before the first add, so the (cross-XCD) load latency is paid
// once per U records rather than once per record (U does not change the
// order of the additions).
template <int NV, int NT>
__device__ __forceinline__ void sum_records(const double *partial, int nblk, int r, double *out) {
  constexpr int U = NV <= 2 ? 8 : NV <= 4 ? 4 : 2;      // U * NV loads in flight, without spilling
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const double *base = partial + (size_t)r * kPart * nblk;
  for (int j0 = 0; j0 < nblk; j0 += U * NT) {
    double t[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + threadIdx.x + u * NT;
#pragma unroll
      for (int k = 0; k < NV; ++k) t[u][k] = j < nblk ? base[(size_t)k * nblk + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k] += t[u][k];
  }
  block_sum<NV, NT>(v, out);
}

__device__ __forceinline__ c64 cdiv(c64 a, c64 b) {
  const double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ __forceinline__ double cabs2(c64 a) { return a.x * a.x + a.y * a.y; }

}  // namespace dda
