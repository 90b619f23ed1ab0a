// BiCGSTAB vector updates, FP64 reductions and per-RHS scalar logic; the
// incident field and the cross-section sums.
//
// BiCGSTAB (van der Vorst 1992; the PBCGST option of §12 of the DDSCAT 7.3
// guide), unpreconditioned, Hermitian inner products <a,b> = sum conj(a) b:
//     rho' = <rh, r>;  beta = (rho'/rho)(alpha/omega);  p = r + beta (p - omega v)
//     v = A p;  alpha = rho' / <rh, v>;  s = r - alpha v
//     t = A s;  omega = <t, s> / <t, t>;  x += alpha p + omega s;  r = s - omega t
// BiCGstab(2) (Sleijpen & Fokkema 1993; the PBCGS2 option the guide
// recommends, §12) runs on the same product kernels: the u/r updates of its
// BiCG steps are fused into the x-forward pass (update lists), <rt, .> and
// the Gram sums of its minimal-residual step into the x-inverse pass; the
// kernels here do its scalar recurrences and the closing update
//     x += g1 r0 + g2 r1;  r0 -= g1 r1 + g2 r2;  u0 -= g1 u1 + g2 u2.
// COCG (van der Vorst & Melissen 1990) and QMR for complex symmetric systems
// (Freund 1992; the QMRCCG option of §12) use the bilinear form a^T b, valid
// because A^T = A:
//     q = A p;  alpha = rho / p^T q;  x += alpha p;  r -= alpha q
//     rho' = r^T r;  beta = rho'/rho;  p = r + beta p
// p is formed in the x-forward pass (update list) and p^T q summed in the
// x-inverse pass.  QMR's iterates are the quasi-minimal-residual smoothing of
// COCG's (Zhou & Walker 1994):
//     theta = |r| / tau;  eta = 1 / (1 + theta^2);  tau = tau theta sqrt(eta)
//     y += eta (x - y);   s += eta (r - s)
// with y the QMR iterate and s its residual, whose norm decides convergence.
// Every RHS of a block carries its own scalars on the device, so a block of
// iterations can be queued without host round trips: each kernel returns
// early for an RHS whose `active` flag is cleared, and the scalar kernels
// clear it when the recursive residual passes the threshold, the iteration
// cap is hit, or the recurrence breaks down.
//
// Reductions are deterministic: a fixed grid writes per-block partial sums
// (wavefront shuffles, then LDS across the block's wavefronts) and one block
// per RHS adds them in a fixed order.  Repeated solves are bit-identical.

#include <algorithm>

#include "dda_internal.hpp"
#include "reduce.hpp"

namespace dda {

constexpr int KNT = 256;

int krylov_blocks(int64_t n3) {
  int64_t b = (n3 + (int64_t)KNT * 8 - 1) / ((int64_t)KNT * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
  dda::block_sum<NV, KNT>(v, out);
}
template <int NV>
__device__ __forceinline__ void sum_partials(const double *partial, int nblk, int r, double *out) {
  sum_records<NV, KNT>(partial, nblk, r, out);
}

#define RHS_PREAMBLE                                       \
  const int r = blockIdx.y;                                \
  if (!active[r]) return;                                  \
  const size_t off = (size_t)r * n3;

// ------------------------------------------------------------- init/restart --
// xs, ss: QMR's raw iterate (set to 0) and smoothed residual (set to b), or
// null; p and v FP32 (VT = c32) for a DDA_MIXED_V32 COCG or BiCGSTAB solve
template <typename VT>
__global__ void kk_init(c64 *x, c64 *rr, c64 *rh, VT *p, VT *v, c64 *xs, c64 *ss, const c64 *b, int64_t n3,
                        double *partial, int nblk) {
  const int r = blockIdx.y;
  const size_t off = (size_t)r * n3;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const c64 bv = b[off + i];
    x[off + i] = {0, 0};
    rr[off + i] = bv;
    if (rh) rh[off + i] = bv;
    vst(p + off + i, c64{0, 0});
    vst(v + off + i, c64{0, 0});
    if (xs) {
      xs[off + i] = {0, 0};
      ss[off + i] = bv;
    }
    acc[0] += bv.x * bv.x + bv.y * bv.y;
    acc[1] += bv.x * bv.x - bv.y * bv.y;           // b^T b
    acc[2] += 2.0 * bv.x * bv.y;
  }
  double out[3];
  block_sum<3>(acc, out);
  if (threadIdx.x == 0) write_record<3>(partial, r, nblk, blockIdx.x, out);
}

// bilinear: rho = b^T b (COCG / QMR), else |b|^2 (rh = b)
__global__ void kk_init_scalars(const double *partial, int nblk, c64 *scal, int *active, int *status, double tol2,
                                int max_iter, int bilinear) {
  const int r = blockIdx.x;
  double s[3];
  sum_partials<3>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const double b2 = s[0];
    sc[S_RHO] = bilinear ? c64{s[1], s[2]} : c64{b2, 0.0};
    sc[S_TAU] = {sqrt(b2), 0.0};
    sc[S_ETA] = {0.0, 0.0};
    sc[S_FLAG] = {0.0, 0.0};
    sc[S_ALPHA] = {1.0, 0.0};
    sc[S_OMEGA] = {1.0, 0.0};
    sc[S_BETA] = {0.0, 0.0};
    sc[S_RNORM2] = {b2, 0.0};
    sc[S_BNORM2] = {b2, 0.0};
    sc[S_THR2] = {tol2 * b2, 0.0};
    sc[S_ITERS] = {0.0, 0.0};
    sc[S_MAXIT] = {double(max_iter), 0.0};
    sc[S_RH2] = {b2, 0.0};
    const bool go = b2 > 0.0;
    active[r] = go ? 1 : 0;
    status[r] = go ? ST_RUN : ST_CONV;
  }
}


__global__ void kk_scalar_alpha(const double *partial, int nblk, c64 *scal, int *active, int *status) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double s[2];
  sum_partials<2>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const c64 den = {s[0], s[1]};
    // <rh, v> ~ 0 relative to |rh| |r|: the recurrence cannot continue
    if (cabs2(den) <= 1e-60 * sc[S_RH2].x * sc[S_RNORM2].x || !(cabs2(den) > 0.0)) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else {
      sc[S_ALPHA] = cdiv(sc[S_RHO], den);
    }
  }
}

// omega = <t, s> / <t, t> from the records of the product that made t.
__device__ __forceinline__ c64 omega_from(const double (&q)[3]) {
  return q[2] > 0.0 ? c64{q[0] / q[2], q[1] / q[2]} : c64{0.0, 0.0};
}

// One block per RHS: omega into S_OMEGA, for kk_update_xr without records.
__global__ void kk_scalar_omega(const double *partial, int nblk, c64 *scal, const int *active) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double q[3];
  sum_partials<3>(partial, nblk, r, q);
  if (threadIdx.x == 0) scal[(size_t)r * kScal + S_OMEGA] = omega_from(q);
}

// x += alpha p + omega s;  r = s - omega t;  partial <rh, r>, |r|^2.
// With rec_in, omega is computed by every block from the records of the
// product that made t (same sum and order in every block, and as
// kk_scalar_omega computes it); block 0 stores it.  Without, it is read from
// S_OMEGA.  Every block reading all records costs O(blocks x records), so
// the host folds only products with few records.
template <typename VT>
__global__ void kk_update_xr(const int *active, c64 *x, c64 *rr, const c64 *rh, const VT *p, const c64 *s,
                             const c64 *t, c64 *scal, int64_t n3, const double *rec_in, int nrec_in,
                             double *partial, int nblk) {
  RHS_PREAMBLE
  __shared__ c64 s_omega;
  if (rec_in) {
    double q[3];
    sum_partials<3>(rec_in, nrec_in, r, q);
    if (threadIdx.x == 0) {
      const c64 om = omega_from(q);
      s_omega = om;
      if (blockIdx.x == 0) scal[(size_t)r * kScal + S_OMEGA] = om;
    }
    __syncthreads();
  } else {
    if (threadIdx.x == 0) s_omega = scal[(size_t)r * kScal + S_OMEGA];
    __syncthreads();
  }
  const c64 alpha = scal[(size_t)r * kScal + S_ALPHA];
  const c64 omega = s_omega;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const c64 sv = s[off + i];
    x[off + i] = x[off + i] + alpha * vld(p + off + i) + omega * sv;
    const c64 rv = sv - omega * t[off + i];
    rr[off + i] = rv;
    const c64 d = cmulc(rh[off + i], rv);
    acc[0] += d.x;
    acc[1] += d.y;
    acc[2] += rv.x * rv.x + rv.y * rv.y;
  }
  double out[3];
  block_sum<3>(acc, out);
  if (threadIdx.x == 0) write_record<3>(partial, r, nblk, blockIdx.x, out);
}

__global__ void kk_scalar_rho(const double *partial, int nblk, c64 *scal, int *active, int *status, int step,
                              double bsign) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double s[3];
  sum_partials<3>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const c64 rho_new = {s[0], s[1]};
    const double rn2 = s[2];
    sc[S_RNORM2] = {rn2, 0.0};
    sc[S_ITERS].x += double(step);
    const c64 omega = sc[S_OMEGA];
    if (!(rn2 == rn2)) {                                     // NaN
      active[r] = 0;
      status[r] = ST_BREAK;
    } else if (rn2 <= sc[S_THR2].x) {
      active[r] = 0;
      status[r] = ST_CONV;
    } else if (sc[S_ITERS].x >= sc[S_MAXIT].x) {
      active[r] = 0;
      status[r] = ST_MAXIT;
    } else if (cabs2(rho_new) <= 1e-60 * sc[S_RH2].x * rn2 || cabs2(omega) == 0.0) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else {
      sc[S_BETA] = bsign * (cdiv(rho_new, sc[S_RHO]) * cdiv(sc[S_ALPHA], omega));
      sc[S_RHO] = rho_new;
    }
  }
}

// r = b - ax for checked RHS; partial |r|^2
__global__ void kk_true_residual(const int *check, const c64 *b, const c64 *ax, c64 *rr, int64_t n3,
                                 double *partial, int nblk) {
  const int r = blockIdx.y;
  if (!check[r]) return;
  const size_t off = (size_t)r * n3;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const c64 rv = b[off + i] - ax[off + i];
    rr[off + i] = rv;
    acc[0] += rv.x * rv.x + rv.y * rv.y;
    acc[1] += rv.x * rv.x - rv.y * rv.y;           // r^T r
    acc[2] += 2.0 * rv.x * rv.y;
  }
  double out[3];
  block_sum<3>(acc, out);
  if (threadIdx.x == 0) write_record<3>(partial, r, nblk, blockIdx.x, out);
}

__global__ void kk_scalar_true(const double *partial, int nblk, c64 *scal, const int *check) {
  const int r = blockIdx.x;
  if (!check[r]) return;
  double s[3];
  sum_partials<3>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    scal[(size_t)r * kScal + S_TRUE2] = {s[0], 0.0};
    scal[(size_t)r * kScal + S_TRUEB] = {s[1], s[2]};
  }
}

// Restart from the current x for RHS with restart[r]: r already holds the true
// residual; rh = r, p = v = 0 and fresh scalars.
// xs, ss (QMR, else null): the raw COCG iterate restarts at x, the smoothed
// residual at r
template <typename VT>
__global__ void kk_restart(const int *restart, const c64 *rr, c64 *rh, VT *p, VT *v, const c64 *x, c64 *xs,
                           c64 *ss, int64_t n3, int nblk) {
  const int r = blockIdx.y;
  if (!restart[r]) return;
  const size_t off = (size_t)r * n3;
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const c64 rv = rr[off + i];
    if (rh) rh[off + i] = rv;
    vst(p + off + i, c64{0, 0});
    vst(v + off + i, c64{0, 0});
    if (xs) {
      xs[off + i] = x[off + i];
      ss[off + i] = rv;
    }
  }
}

__global__ void kk_restart_scalars(const int *restart, c64 *scal, int *active, int *status, int nrhs, double tol2,
                                   double inner2, int bilinear) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !restart[r]) return;
  c64 *sc = scal + (size_t)r * kScal;
  const double t2 = sc[S_TRUE2].x;
  sc[S_RHO] = bilinear ? sc[S_TRUEB] : c64{t2, 0.0};
  sc[S_TAU] = {sqrt(t2), 0.0};
  sc[S_ETA] = {0.0, 0.0};
  sc[S_FLAG] = {0.0, 0.0};
  sc[S_ALPHA] = {1.0, 0.0};
  sc[S_OMEGA] = {1.0, 0.0};
  sc[S_BETA] = {0.0, 0.0};
  sc[S_RNORM2] = {t2, 0.0};
  sc[S_RH2] = {t2, 0.0};
  const double thr = tol2 * sc[S_BNORM2].x;
  const double inner = inner2 * t2;
  sc[S_THR2] = {thr > inner ? thr : inner, 0.0};
  active[r] = 1;
  status[r] = ST_RUN;
}

// ------------------------------------------------------------- BiCGstab(2) --
// Second BiCG step of a cycle: rho1 = <rt, r1> (records of the product that
// made r1); beta = alpha rho1 / rho0; rho0 = rho1.
__global__ void kk2_scalar_rho1(const double *partial, int nblk, c64 *scal, int *active, int *status) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double s[2];
  sum_partials<2>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const c64 rho1 = {s[0], s[1]};
    if (!(cabs2(rho1) > 1e-60 * sc[S_RH2].x * sc[S_RNORM2].x) || !(cabs2(sc[S_RHO]) > 0.0)) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else {
      sc[S_BETA] = sc[S_ALPHA] * cdiv(rho1, sc[S_RHO]);
      sc[S_RHO] = rho1;
    }
  }
}

// Minimal-residual step: with the Gram sums <r1,r1>, <r2,r2>, <r1,r2>,
// <r1,r0>, <r2,r0> (Hermitian products), solve the 2x2 normal equations of
// min |r0 - g1 r1 - g2 r2|.  omega = g2.
__global__ void kk2_scalar_mr(const double *partial, int nblk, c64 *scal, int *active, int *status) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double s[8];
  sum_partials<8>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const double r11 = s[0], r22 = s[1];
    const c64 r12 = {s[2], s[3]}, c1 = {s[4], s[5]}, c2 = {s[6], s[7]};
    const double det = r11 * r22 - cabs2(r12);
    if (!(det > 1e-14 * r11 * r22) || !(r11 > 0.0)) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else {
      const double id = 1.0 / det;
      const c64 g1 = id * (r22 * c1 - r12 * c2);
      const c64 g2 = id * (r11 * c2 - conj(r12) * c1);
      sc[S_G1] = g1;
      sc[S_OMEGA] = g2;
    }
  }
}

// x += g1 r0 + g2 r1;  r0 -= g1 r1 + g2 r2;  u0 -= g1 u1 + g2 u2;
// partials <rt, r0>, |r0|^2 of the new r0.
__global__ void kk2_update_mr(const int *active, c64 *x, c64 *r0, const c64 *r1, const c64 *r2, c64 *u0,
                              const c64 *u1, const c64 *u2, const c64 *rt, const c64 *scal, int64_t n3,
                              double *partial, int nblk) {
  RHS_PREAMBLE
  const c64 g1 = scal[(size_t)r * kScal + S_G1];
  const c64 g2 = scal[(size_t)r * kScal + S_OMEGA];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const size_t j = off + i;
    const c64 a0 = r0[j], a1 = r1[j], a2 = r2[j];
    x[j] = x[j] + g1 * a0 + g2 * a1;
    const c64 rn = a0 - g1 * a1 - g2 * a2;
    r0[j] = rn;
    u0[j] = u0[j] - g1 * u1[j] - g2 * u2[j];
    const c64 d = cmulc(rt[j], rn);
    acc[0] += d.x;
    acc[1] += d.y;
    acc[2] += rn.x * rn.x + rn.y * rn.y;
  }
  double out[3];
  block_sum<3>(acc, out);
  if (threadIdx.x == 0) write_record<3>(partial, r, nblk, blockIdx.x, out);
}

// ------------------------------------------------------------- COCG / QMR --
// alpha = rho / p^T q and the breakdown flag (p^T q ~ 0).
__device__ __forceinline__ bool cocg_alpha(const double (&d)[2], const c64 *sc, c64 &a) {
  const c64 den = {d[0], d[1]}, rho = sc[S_RHO];
  const bool ok = cabs2(den) > 1e-60 * cabs2(rho) && cabs2(den) > 0.0 && cabs2(den) < 1e300;
  a = ok ? cdiv(rho, den) : c64{0.0, 0.0};
  return ok;
}

// One block per RHS: alpha into S_ALPHA and the flag into S_FLAG, for
// kk_cocg_update without records.
__global__ void kk_cocg_alpha(const double *partial, int nblk, c64 *scal, const int *active) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double d[2];
  sum_partials<2>(partial, nblk, r, d);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    c64 a;
    const bool ok = cocg_alpha(d, sc, a);
    sc[S_ALPHA] = a;
    sc[S_FLAG] = {ok ? 0.0 : 1.0, 0.0};
  }
}

// alpha = rho / p^T q: with rec_in every block sums the records of the
// product q = A p in the same order (as kk_cocg_alpha does), so all agree;
// without, alpha is read from S_ALPHA.  A breakdown leaves x and r as they
// are and is flagged in S_FLAG for kk_cocg_scalar (no block clears `active`
// here, so every block does the same work).
// QMR (xs, ss non-null): x holds the smoothed iterate y, xs the COCG iterate
// and ss the smoothed residual; the smoothing of the previous step comes first:
//     y += eta (xs - y);  ss += eta (r - ss);  then xs += alpha p;  r -= alpha q.
// Records: r^T r, |r|^2 and |ss|^2 (the smoothed residual just formed).
template <typename VT>
__global__ void kk_cocg_update(const int *active, c64 *x, c64 *rr, const VT *p, const VT *q, c64 *xs, c64 *ss,
                               c64 *scal, int64_t n3, const double *rec_in, int nrec_in, double *partial,
                               int nblk) {
  RHS_PREAMBLE
  __shared__ c64 s_alpha;
  if (rec_in) {
    double d[2];
    sum_partials<2>(rec_in, nrec_in, r, d);
    if (threadIdx.x == 0) {
      c64 *sc = scal + (size_t)r * kScal;
      c64 a;
      const bool ok = cocg_alpha(d, sc, a);
      s_alpha = a;
      if (blockIdx.x == 0) {
        sc[S_ALPHA] = a;
        sc[S_FLAG] = {ok ? 0.0 : 1.0, 0.0};
      }
    }
    __syncthreads();
  } else {
    if (threadIdx.x == 0) s_alpha = scal[(size_t)r * kScal + S_ALPHA];
    __syncthreads();
  }
  const c64 alpha = s_alpha;
  const c64 eta = xs ? scal[(size_t)r * kScal + S_ETA] : c64{0.0, 0.0};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)KNT + threadIdx.x; i < n3; i += (int64_t)nblk * KNT) {
    const size_t j = off + i;
    const c64 pv = vld(p + j), qv = vld(q + j);
    c64 rv = rr[j];
    if (xs) {
      const c64 xv = xs[j], yv = x[j], sv = ss[j];
      x[j] = yv + eta * (xv - yv);
      const c64 sn = sv + eta * (rv - sv);
      ss[j] = sn;
      acc[3] += sn.x * sn.x + sn.y * sn.y;
      xs[j] = xv + alpha * pv;
    } else {
      x[j] = x[j] + alpha * pv;
    }
    rv = rv - alpha * qv;
    rr[j] = rv;
    acc[0] += rv.x * rv.x - rv.y * rv.y;             // r^T r
    acc[1] += 2.0 * rv.x * rv.y;
    acc[2] += rv.x * rv.x + rv.y * rv.y;
  }
  double out[4];
  block_sum<4>(acc, out);
  if (threadIdx.x == 0) write_record<4>(partial, r, nblk, blockIdx.x, out);
}

// rho' = r^T r, beta = rho'/rho; convergence on |r| (COCG) or on the smoothed
// residual |s| (QMR); QMR's tau and eta for the next smoothing step.
__global__ void kk_cocg_scalar(const double *partial, int nblk, c64 *scal, int *active, int *status, int qmr) {
  const int r = blockIdx.x;
  if (!active[r]) return;
  double s[4];
  sum_partials<4>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    c64 *sc = scal + (size_t)r * kScal;
    const c64 rho_new = {s[0], s[1]};
    const double rn2 = s[2];
    const double crit = qmr ? s[3] : rn2;
    sc[S_RNORM2] = {rn2, 0.0};
    sc[S_ITERS].x += 1.0;
    if (!(rn2 == rn2) || !(crit == crit) || sc[S_FLAG].x != 0.0) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else if (crit <= sc[S_THR2].x) {
      active[r] = 0;
      status[r] = ST_CONV;
    } else if (sc[S_ITERS].x >= sc[S_MAXIT].x) {
      active[r] = 0;
      status[r] = ST_MAXIT;
    } else if (!(cabs2(rho_new) > 1e-60 * rn2 * rn2) || !(cabs2(sc[S_RHO]) > 0.0)) {
      active[r] = 0;
      status[r] = ST_BREAK;
    } else {
      sc[S_BETA] = cdiv(rho_new, sc[S_RHO]);
      sc[S_RHO] = rho_new;
      if (qmr) {
        const double tau = sc[S_TAU].x;
        const double th = sqrt(rn2) / tau;
        const double eta = 1.0 / (1.0 + th * th);
        sc[S_TAU] = {tau * th * sqrt(eta), 0.0};
        sc[S_ETA] = {eta, 0.0};
      }
    }
  }
}

// ------------------------------------------------------------- host wrappers --
static dim3 vgrid(const KrylovState &k) { return dim3(k.nblk, k.nrhs); }

static bool bilinear_solver(int solver) { return solver == DDA_SOLVER_COCG || solver == DDA_SOLVER_QMR; }

// the c32 view of a vector buffer (COCG's FP32 p and q)
static c32 *r32(c64 *p) { return reinterpret_cast<c32 *>(p); }

// Records stay inside their buffers: k.partial holds k.nrec records per value
// and RHS (the products' x-inverse blocks and the vector kernels' blocks),
// k.partial2 k.nblk; nrec is the count a product wrote.
static void check_records(const KrylovState &k, int nrec) {
  DDA_REQUIRE(k.nblk >= 1 && k.nblk <= k.nrec, "vector-kernel records exceed their buffer");
  DDA_REQUIRE(nrec >= 1 && nrec <= k.nrec, "product records exceed their buffer");
}

void k_init_state(const KrylovState &k, double tol, int max_iter, int solver, hipStream_t s) {
  check_records(k, k.nblk);
  const bool qmr = solver == DDA_SOLVER_QMR;
  if (k.vec32) {
    DDA_REQUIRE(solver == DDA_SOLVER_COCG || solver == DDA_SOLVER_BICGSTAB,
                "FP32 search directions are built for COCG and BiCGSTAB only");
    hipLaunchKernelGGL(kk_init<c32>, vgrid(k), dim3(KNT), 0, s, k.x, k.r, k.rh, r32(k.p), r32(k.v),
                       nullptr, nullptr, k.b, k.n3, k.partial, k.nblk);
  } else {
    hipLaunchKernelGGL(kk_init<c64>, vgrid(k), dim3(KNT), 0, s, k.x, k.r, k.rh, k.p, k.v, qmr ? k.s : nullptr,
                       qmr ? k.t : nullptr, k.b, k.n3, k.partial, k.nblk);
  }
  hipLaunchKernelGGL(kk_init_scalars, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, k.nblk, k.scal, k.active, k.status,
                     tol * tol, max_iter, bilinear_solver(solver) ? 1 : 0);
  DDA_HIP(hipGetLastError());
}
void k_cocg_update(const KrylovState &k, hipStream_t s, int nrec, bool fold, bool qmr) {
  check_records(k, nrec);
  if (!fold)
    hipLaunchKernelGGL(kk_cocg_alpha, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, nrec, k.scal, k.active);
  if (k.vec32)
    hipLaunchKernelGGL(kk_cocg_update<c32>, vgrid(k), dim3(KNT), 0, s, k.active, k.x, k.r, r32(k.p), r32(k.v),
                       nullptr, nullptr, k.scal, k.n3, fold ? k.partial : nullptr, nrec, k.partial2, k.nblk);
  else
    hipLaunchKernelGGL(kk_cocg_update<c64>, vgrid(k), dim3(KNT), 0, s, k.active, k.x, k.r, k.p, k.v,
                       qmr ? k.s : nullptr, qmr ? k.t : nullptr, k.scal, k.n3, fold ? k.partial : nullptr, nrec,
                       k.partial2, k.nblk);
}
void k_cocg_scalar(const KrylovState &k, hipStream_t s, bool qmr) {
  hipLaunchKernelGGL(kk_cocg_scalar, dim3(k.nrhs), dim3(KNT), 0, s, k.partial2, k.nblk, k.scal, k.active, k.status,
                     qmr ? 1 : 0);
}
void k_scalar_alpha(const KrylovState &k, hipStream_t s, int nrec) {
  check_records(k, nrec);
  hipLaunchKernelGGL(kk_scalar_alpha, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, nrec, k.scal, k.active, k.status);
}
void k_update_xr(const KrylovState &k, hipStream_t s, int nrec, bool fold) {
  check_records(k, nrec);
  if (!fold)
    hipLaunchKernelGGL(kk_scalar_omega, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, nrec, k.scal, k.active);
  if (k.vec32)
    hipLaunchKernelGGL(kk_update_xr<c32>, vgrid(k), dim3(KNT), 0, s, k.active, k.x, k.r, k.rh, r32(k.p), k.s, k.t,
                       k.scal, k.n3, fold ? k.partial : nullptr, nrec, k.partial2, k.nblk);
  else
    hipLaunchKernelGGL(kk_update_xr<c64>, vgrid(k), dim3(KNT), 0, s, k.active, k.x, k.r, k.rh, k.p, k.s, k.t,
                       k.scal, k.n3, fold ? k.partial : nullptr, nrec, k.partial2, k.nblk);
}
void k_scalar_rho(const KrylovState &k, hipStream_t s, int step, double bsign) {
  // BiCGSTAB: records of kk_update_xr (partial2); BiCGstab(2): of kk2_update_mr (partial)
  hipLaunchKernelGGL(kk_scalar_rho, dim3(k.nrhs), dim3(KNT), 0, s, step == 1 ? k.partial2 : k.partial, k.nblk,
                     k.scal, k.active, k.status, step, bsign);
}
void k2_scalar_rho1(const KrylovState &k, hipStream_t s, int nrec) {
  check_records(k, nrec);
  hipLaunchKernelGGL(kk2_scalar_rho1, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, nrec, k.scal, k.active, k.status);
}
void k2_scalar_mr(const KrylovState &k, hipStream_t s, int nrec) {
  check_records(k, nrec);
  hipLaunchKernelGGL(kk2_scalar_mr, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, nrec, k.scal, k.active, k.status);
}
void k2_update_mr(const KrylovState &k, hipStream_t s) {
  hipLaunchKernelGGL(kk2_update_mr, vgrid(k), dim3(KNT), 0, s, k.active, k.x, k.r, k.s, k.t, k.p, k.v, k.u2, k.rh,
                     k.scal, k.n3, k.partial, k.nblk);
}
void k_true_residual(const KrylovState &k, const c64 *ax, hipStream_t s) {
  hipLaunchKernelGGL(kk_true_residual, vgrid(k), dim3(KNT), 0, s, k.check, k.b, ax, k.r, k.n3, k.partial, k.nblk);
  hipLaunchKernelGGL(kk_scalar_true, dim3(k.nrhs), dim3(KNT), 0, s, k.partial, k.nblk, k.scal, k.check);
  DDA_HIP(hipGetLastError());
}
void k_restart(const KrylovState &k, const int *restart, double tol, double inner_tol, int solver,
               hipStream_t s) {
  const bool qmr = solver == DDA_SOLVER_QMR;
  if (k.vec32)
    hipLaunchKernelGGL(kk_restart<c32>, vgrid(k), dim3(KNT), 0, s, restart, k.r, k.rh, r32(k.p), r32(k.v),
                       k.x, nullptr, nullptr, k.n3, k.nblk);
  else
    hipLaunchKernelGGL(kk_restart<c64>, vgrid(k), dim3(KNT), 0, s, restart, k.r, k.rh, k.p, k.v, k.x,
                       qmr ? k.s : nullptr, qmr ? k.t : nullptr, k.n3, k.nblk);
  hipLaunchKernelGGL(kk_restart_scalars, dim3((k.nrhs + 63) / 64), dim3(64), 0, s, restart, k.scal, k.active,
                     k.status, k.nrhs, tol * tol, inner_tol * inner_tol, bilinear_solver(solver) ? 1 : 0);
  DDA_HIP(hipGetLastError());
}

// ------------------------------------------------------- incident field --
// E_j = e exp(i kd khat . r_j)  (eq. AP=E with |E0| = 1)
__global__ void kk_incident(const int32_t *ijk, int64_t n, const RhsDev *rhs, double kd, c64 *e) {
  const int r = blockIdx.y;
  const RhsDev R = rhs[r];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const double ph = kd * (R.khat[0] * ijk[3 * j] + R.khat[1] * ijk[3 * j + 1] + R.khat[2] * ijk[3 * j + 2]);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const c64 w = {cs, sn};
    c64 *o = e + ((size_t)r * n + j) * 3;
    o[0] = w * R.e[0];
    o[1] = w * R.e[1];
    o[2] = w * R.e[2];
  }
}

void launch_incident(const Geometry &g, const int32_t *ijk, const RhsDev *rhs, int nrhs, double kd, c64 *e,
                     hipStream_t s) {
  const int64_t n = g.n_sites;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(kk_incident, dim3(nb, nrhs), dim3(256), 0, s, ijk, n, rhs, kd, e);
  DDA_HIP(hipGetLastError());
}

// ------------------------------------------------------ Jacobi scaling --
// v <- s v (inverse: v <- v / s), s per RHS, composition and component
__global__ void kk_scale(c64 *v, int64_t n, const c64 *scl, int ncomp, const uint8_t *comp, int inverse) {
  const int r = blockIdx.y;
  const c64 *sr = scl + (size_t)r * ncomp * 3;
  for (int64_t j = blockIdx.x * (int64_t)KNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * KNT) {
    const c64 *sj = sr + (comp ? 3 * comp[j] : 0);
    c64 *vj = v + ((size_t)r * n + j) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) vj[c] = inverse ? cdiv(vj[c], sj[c]) : sj[c] * vj[c];
  }
}

void launch_scale(const Geometry &g, c64 *v, int nrhs, const c64 *scl, int ncomp, const uint8_t *comp, bool inverse,
                  hipStream_t s) {
  const int64_t n = g.n_sites;
  const unsigned nb = (unsigned)std::min<int64_t>((n + KNT - 1) / KNT, 2048);
  hipLaunchKernelGGL(kk_scale, dim3(nb, nrhs), dim3(KNT), 0, s, v, n, scl, ncomp, comp, inverse ? 1 : 0);
  DDA_HIP(hipGetLastError());
}

// --------------------------------------------------------- cross sections --
// per site: Im(conj(E_j) . P_j)  and  sum_c (-Im(ainv_jc) - (2/3) kd^3) |P_jc|^2
__global__ void kk_cross(const int32_t *ijk, int64_t n, const RhsDev *rhs, double kd, const c64 *P, const c64 *ainv,
                         int ncomp, const uint8_t *comp, double *partial, int nblk) {
  const int r = blockIdx.y;
  const RhsDev R = rhs[r];
  const double rr = (2.0 / 3.0) * kd * kd * kd;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t j = blockIdx.x * (int64_t)KNT + threadIdx.x; j < n; j += (int64_t)nblk * KNT) {
    const double ph = kd * (R.khat[0] * ijk[3 * j] + R.khat[1] * ijk[3 * j + 1] + R.khat[2] * ijk[3 * j + 2]);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const c64 w = {cs, sn};
    const c64 *pj = P + ((size_t)r * n + j) * 3;
    const c64 *ai = ainv + ((size_t)r * ncomp + (comp ? comp[j] : 0)) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const c64 ec = w * R.e[c];
      const c64 pc = pj[c];
      acc[0] += ec.x * pc.y - ec.y * pc.x;        // Im(conj(E) P)
      acc[2] += ec.x * pc.x + ec.y * pc.y;        // Re(conj(E) P)
      acc[1] += (-ai[c].y - rr) * (pc.x * pc.x + pc.y * pc.y);
    }
  }
  double out[3];
  block_sum<3>(acc, out);
  if (threadIdx.x == 0) write_record<3>(partial, r, nblk, blockIdx.x, out);
}

// sums[3 r + i]: sum Im(conj(E) P), the absorption sum, sum Re(conj(E) P)
__global__ void kk_cross_final(const double *partial, int nblk, double *sums) {
  const int r = blockIdx.x;
  double s[3];
  sum_partials<3>(partial, nblk, r, s);
  if (threadIdx.x == 0) {
    sums[3 * r] = s[0];
    sums[3 * r + 1] = s[1];
    sums[3 * r + 2] = s[2];
  }
}

void launch_cross_sums(const Geometry &g, const int32_t *ijk, const RhsDev *rhs, int nrhs, double kd, const c64 *P,
                       const c64 *ainv, int ncomp, const uint8_t *comp, double *partial, double *sums,
                       hipStream_t s) {
  const int nblk = krylov_blocks(3 * g.n_sites);
  hipLaunchKernelGGL(kk_cross, dim3(nblk, nrhs), dim3(KNT), 0, s, ijk, g.n_sites, rhs, kd, P, ainv, ncomp, comp,
                     partial, nblk);
  hipLaunchKernelGGL(kk_cross_final, dim3(nrhs), dim3(KNT), 0, s, partial, nblk, sums);
  DDA_HIP(hipGetLastError());
}

}  // namespace dda
