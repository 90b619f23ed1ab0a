// Internal declarations shared by the HIP sources of the DDA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dda.h"

namespace dda {

// ------------------------------------------------------------------ errors --
void set_error(const std::string &msg);

struct Error {
  int code;
  std::string msg;
};

#define DDA_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::dda::Error{(e_ == hipErrorOutOfMemory) ? DDA_ENOMEM : DDA_EDEVICE,       \
                         std::string(#call) + ": " + hipGetErrorString(e_)};           \
  } while (0)

#define DDA_REQUIRE(cond, msg)                                                         \
  do {                                                                                 \
    if (!(cond)) throw ::dda::Error{DDA_EINVAL, (msg)};                                \
  } while (0)

// ----------------------------------------------------------------- complex --
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

using c64 = cpx<double>;
using c32 = cpx<float>;

// Krylov vectors are complex FP64 (c64), or FP32 (c32) for the search
// direction and its product in a DDA_MIXED_V32 COCG solve; arithmetic on them
// is FP64.
__host__ __device__ __forceinline__ c64 vld(const c64 *p) { return *p; }
__host__ __device__ __forceinline__ c64 vld(const c32 *p) {
  const c32 v = *p;
  return {double(v.x), double(v.y)};
}
__host__ __device__ __forceinline__ void vst(c64 *p, c64 v) { *p = v; }
__host__ __device__ __forceinline__ void vst(c32 *p, c64 v) { *p = c32{float(v.x), float(v.y)}; }
// the value a vector of type VT holds after storing v (so that a product
// transforms exactly the vector it stores)
template <typename VT>
__host__ __device__ __forceinline__ c64 vround(c64 v) {
  if constexpr (sizeof(VT) == sizeof(c32)) return {double(float(v.x)), double(float(v.y))};
  else return v;
}

// ---------------------------------------------------------------- FFT plan --
constexpr int kMaxStages = 8;     // a 2/3/5-smooth L <= 512 needs at most 6 stages
constexpr int kMaxLen = 512;      // largest supported padded extent

// Unsigned division by a divisor d >= 1 fixed at launch time, without a
// divide instruction sequence.  For d = 2^sh it is a shift.  Otherwise, with
// m = floor(2^32 / d) + 1 = 2^32 / d + e (0 < e < 1),
//   umulhi(x, m) = floor(x / d + x e / 2^32),
// and x e / 2^32 < 1 / d whenever x d < 2^32: the extra term never reaches the
// next integer, so the quotient is exact for every x with x * d < 2^32.
struct FastDiv {
  uint32_t m = 0;
  int32_t sh = 0;                 // >= 0: d = 2^sh
  __host__ __device__ __forceinline__ uint32_t operator()(uint32_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    return sh >= 0 ? x >> sh : __umulhi(x, m);
#else
    return sh >= 0 ? x >> sh : (uint32_t)(((uint64_t)x * m) >> 32);
#endif
  }
};
FastDiv make_fastdiv(uint32_t d);

// Stockham plan of one axis.  Stage s has radix R = radix[s] and sub-transform
// length ns[s] = radix[0] * ... * radix[s-1]; it reads inputs lr[s] = L / R
// apart and uses twiddle exponents that are multiples of twstep[s] =
// L / (ns[s] R).
struct AxisPlan {
  int L;                          // transform length
  int nstages;
  int radix[kMaxStages];          // radices in execution order (each 2, 3, 4, 5 or 8)
  int ns[kMaxStages];
  int lr[kMaxStages];
  int twstep[kMaxStages];
  FastDiv ns_div[kMaxStages];     // division by ns[s]
  FastDiv lr_div[kMaxStages];     // division by lr[s]
};

AxisPlan make_axis_plan(int L);   // throws for non-smooth L or L > kMaxLen
int next_smooth(int n);

// Twiddle tables exp(-2 pi i n / L), n = 0..L-1, in both precisions.
struct Twiddles {
  c64 *d64 = nullptr;
  c32 *d32 = nullptr;
  int L = 0;
};

// Threads per block of every FFT kernel.
constexpr int kNT = 256;

// ----------------------------------------------------------- grid geometry --
// Layouts of the two intermediate buffers of the convolution (per RHS):
//   A: [3][nz][nxt][ny][W]   x-transformed rows, tiled in x by W
//   B: [My][nxt][3][nz][W]   x- and y-transformed, tiled in x by W
// W = 16 (FP32) or 8 (FP64) so that a tile row is 128 bytes; nxt = ceil(Mx/W).
struct Geometry {
  int nx, ny, nz;
  int Mx, My, Mz;
  int Mxh, Myh, Mzh;              // octant extents M/2 + 1
  int64_t n_sites;
  int W(bool fp32) const { return fp32 ? 16 : 8; }
  int nxt(bool fp32) const { return (Mx + W(fp32) - 1) / W(fp32); }
  size_t a_elems(bool fp32) const { return (size_t)3 * nz * nxt(fp32) * ny * W(fp32); }
  size_t b_elems(bool fp32) const { return (size_t)My * nxt(fp32) * 3 * nz * W(fp32); }
  size_t oct_elems() const { return (size_t)Mxh * Myh * Mzh; }
};

// Per-RHS device description used by the field and diagonal kernels.
struct RhsDev {
  double khat[3];
  c64 e[3];
};

// ------------------------------------------------------------ kernel API --
// Symmetric diagonal (Jacobi) scaling of the product: with s non-null the
// passes compute S A S y = S (1/alpha) S y - S G S y, S = diag(s) of one value
// per RHS, composition and component ([nrhs][ncomp][3]): the x-forward
// transforms s y and the x-inverse writes ainv y - s (G s y), ainv then
// holding s (1/alpha) s.
struct Scaling {
  const c64 *s = nullptr;
  const uint8_t *comp = nullptr;  // device [N] composition index, or nullptr (all 0)
  int ncomp = 1;
  __device__ __forceinline__ const c64 *rhs(int r) const { return s + (size_t)r * ncomp * 3; }
  __device__ __forceinline__ c64 at(const c64 *sr, int site, int c) const {
    return sr[(comp ? 3 * comp[site] : 0) + c];
  }
};

// BiCGSTAB work fused into the first and last pass of a product.
struct FuseArgs {
  int in_mode = 0;     // 0: transform `in` as given
                       // 1: form p = r + beta (p - omega v), store it in w (= p), transform it
                       // 2: form s = r - alpha v, store it in w (= s), transform it
                       // 3: nax element-wise updates d_i = a_i + c_i b_i, c_i = (-1)^neg_i scal[slot_i];
                       //    d_0 is transformed (it must be `in`)
  int out_mode = 0;    // 0: nothing
                       // 1: per-block partial sums of <rh, out>
                       // 2: per-block partial sums of <out, in> and <out, out>
                       // 3: per-block Gram sums of in = r1, out = r2 and r = r0:
                       //    <r1,r1>, <r2,r2>, <r1,r2>, <r1,r0>, <r2,r0>
                       // 4: per-block partial sums of the bilinear in^T out (COCG / QMR)
  const c64 *r = nullptr, *v = nullptr, *rh = nullptr;
  c64 *w = nullptr;
  c64 *scal = nullptr;
  int *active = nullptr, *status = nullptr;
  double *partial = nullptr;      // records [nrhs][kPart][x-pass blocks] (see reduce.hpp)
  int rec_cap = 0;                // records per value and RHS that `partial` holds
  // in_mode 2 with fold_alpha: every block computes alpha = rho / <rh, v> from
  // the nrec records in `partial` of the product that made v (no separate
  // scalar kernel); block 0 stores it
  int fold_alpha = 0;
  int nrec = 0;
  int nax = 0;
  c64 *ax_d[3] = {nullptr, nullptr, nullptr};
  const c64 *ax_a[3] = {nullptr, nullptr, nullptr}, *ax_b[3] = {nullptr, nullptr, nullptr};
  int ax_slot[3] = {0, 0, 0};
  int ax_neg[3] = {0, 0, 0};
};

// Convolution + diagonal:  out_r = ainv_r[comp] * in_r - (G * in_r)   (r < nrhs)
// in/out are FP64 [nrhs][N][3]; the FFT pipeline runs in T.
struct MatvecArgs {
  const c64 *in;
  c64 *out;
  int nrhs;
  const int *mask;                // device [nrhs] (nonzero = process) or nullptr
  const c64 *ainv;                // device [nrhs][ncomp][3]: diagonal of 1/alpha per composition
  int ncomp;
  const uint8_t *comp;            // device [N] or nullptr
  const int *cell_site;           // device [nz][ny][nx], -1 = empty
  // device [nz * ny] of {first site, first x, count} when every row's sites are
  // one run of consecutive x with consecutive site indices (count 0: empty
  // row), else nullptr; the x passes then move P as contiguous runs
  const int4 *rowtab;
  void *bufA, *bufB;              // workspaces (sized for nrhs in FP64)
  const void *ghat;               // octant Green transform [Mzh][Myh][Mxh][6] (scaled by 1/M)
  const void *twx, *twy, *twz;    // twiddles of the T precision
  AxisPlan px, py, pz;
  FuseArgs fuse;
  Scaling scl;                    // Jacobi scaling (s = nullptr: none)
  // DDA_MIXED_V32 (FP32 product only): vec32, the product's input and output
  // and the vector its fused update writes are c32 (COCG's p and q = A p,
  // BiCGSTAB's p and v = A p); vvec32, the update's v is c32 (BiCGSTAB's
  // s -> t product, whose s and t stay c64)
  bool vec32 = false;
  bool vvec32 = false;
  int zvar = -1;                  // z-pass plan variant (0..3), or -1: the tuned table's choice
  int xvar[2] = {-1, -1};         // x-forward / x-inverse rows-plan variant (0..1), or -1
};

// Plan variants exist for the compile-time lengths from kTunedMinLen up: four
// for the z-pass (plan_variant in fft_lds.hpp), two for the x passes
// (rows_plan).  tuned_variant returns the autotuner's measured choice per
// pass, length and precision (plan_tuned.inc), 0 for lengths it has not timed.
constexpr int kTunedMinLen = 96;
constexpr int kPlanVariantsHost = 4;     // = kPlanVariants of fft_lds.hpp
constexpr int kRowPlanVariantsHost = 2;  // = kRowPlanVariants of fft_lds.hpp
enum : int { kPassXfwd = 0, kPassZ = 2, kPassXinv = 4 };
int tuned_variant(int pass, int L, bool fp32);

// The x passes keep 3 * rows * Mx <= kXBudget elements per block (EPT <= 8):
// more, lighter blocks keep more loads in flight than few heavy ones.
constexpr int kXBudget = 1536;
constexpr int xpass_rows(int Mx) {
  return 3 * Mx >= kXBudget ? 1 : kXBudget / (3 * Mx) >= 2 ? kXBudget / (3 * Mx) : 6 * Mx <= 2048 ? 2 : 1;
}

// Blocks of the x passes (= partial records an out_mode reduction writes).
int xpass_blocks(const Geometry &g, bool fp32);

// ev: optional events recorded before each of the five passes and after the
// last (6 events).  only_pass >= 0 launches that pass alone `reps` times back to
// back, between ev[0] and ev[1] (timing of one kernel).
template <typename T>
void launch_matvec(const Geometry &g, const MatvecArgs &a, hipStream_t s, const hipEvent_t *ev = nullptr,
                   int only_pass = -1, int reps = 1);

// Green-tensor transform: fills `full` [6][Mz][My][Mx] (FP64), transforms it in
// place and writes the octant copies (scaled by 1/M) in FP64 and FP32.
void launch_green_build(const Geometry &g, double kd, c64 *full, c64 *oct64, c32 *oct32,
                        const Twiddles &tx, const Twiddles &ty, const Twiddles &tz,
                        const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, hipStream_t s);

// Batched 1-D FFT of contiguous pencils (diagnostic and setup helper).
template <typename T>
void launch_fft_rows(const cpx<T> *in, cpx<T> *out, int64_t batch, const AxisPlan &p,
                     const cpx<T> *tw, int dir, T scale, hipStream_t s);

// ------------------------------------------------------ Krylov kernels --
struct KrylovState {
  int nrhs = 0;
  int64_t n3 = 0;                 // 3N complex entries per RHS
  // BiCGSTAB: x, r, rh (shadow), p, v, s, t; b = E.  BiCGstab(2) uses
  // x, r = r_0, rh = shadow, p = u_0, v = u_1, u2 = u_2, s = r_1, t = r_2.
  c64 *x = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr, *s = nullptr,
      *t = nullptr, *b = nullptr, *u2 = nullptr;
  double *partial = nullptr;      // records [nrhs][kPart][nrec] of the products and of most Krylov kernels
  double *partial2 = nullptr;     // records of kk_update_xr (written while `partial` is read)
  c64 *scal = nullptr;            // [nrhs][kScal]
  int *active = nullptr;          // [nrhs]
  int *status = nullptr;          // [nrhs]
  int *check = nullptr;           // [nrhs]
  int nblk = 0;
  int nrec = 0;                   // records per RHS in `partial` (max of Krylov and x-pass blocks)
  // DDA_MIXED_V32 COCG: p and v hold c32 values (in the first half of their
  // buffers); x, r, b, t and every sum stay FP64
  bool vec32 = false;
};

// scalar slots per RHS
enum : int {
  S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_RNORM2, S_BNORM2, S_THR2, S_ITERS, S_MAXIT, S_RH2, S_TRUE2,
  S_G1,                           // BiCGstab(2): first minimal-residual coefficient (the second is omega)
  S_TRUEB,                        // bilinear r^T r of the last true residual (COCG / QMR restarts)
  S_TAU, S_ETA,                   // QMR smoothing: quasi-residual tau and the weight of the next step
  S_FLAG,                         // COCG / QMR: nonzero when p^T q broke down in the last update
  kScal
};

// status values kept on the device
enum : int { ST_RUN = 0, ST_CONV = 1, ST_BREAK = 2, ST_MAXIT = 3, ST_DONE = 4, ST_IDLE = 5 };

int krylov_blocks(int64_t n3);
// solver: DDA_SOLVER_*; COCG / QMR start from the bilinear rho = b^T b, QMR
// also sets its raw COCG iterate (k.s) to 0 and its smoothed residual (k.t) to b
void k_init_state(const KrylovState &k, double tol, int max_iter, int solver, hipStream_t s);
void k_scalar_alpha(const KrylovState &k, hipStream_t s, int nrec);
// x += alpha p + omega s, r = s - omega t; omega is computed by every block
// from the nrec records (<t, s>, <t, t>) in k.partial; records of <rh, r>,
// |r|^2 go to k.partial2 (read by k_scalar_rho)
// fold: the consuming kernel computes omega (alpha) from the nrec records in
// every block; otherwise a one-block kernel computes it first.
void k_update_xr(const KrylovState &k, hipStream_t s, int nrec, bool fold);
// step = 1, bsign = +1: BiCGSTAB; step = 2, bsign = -1: end of a BiCGstab(2) cycle
void k_scalar_rho(const KrylovState &k, hipStream_t s, int step = 1, double bsign = 1.0);
// BiCGstab(2): second BiCG step's beta, minimal-residual coefficients, closing update
void k2_scalar_rho1(const KrylovState &k, hipStream_t s, int nrec);
void k2_scalar_mr(const KrylovState &k, hipStream_t s, int nrec);
void k2_update_mr(const KrylovState &k, hipStream_t s);
// COCG / QMR: alpha = rho / p^T q from the nrec records in k.partial (every
// block), x += alpha p, r -= alpha q; QMR first applies the smoothing of the
// previous step to x (the smoothed iterate) and k.t (the smoothed residual)
// with the raw COCG iterate in k.s.  Records of r^T r, |r|^2, |t|^2 go to
// k.partial2; k_cocg_scalar turns them into beta, QMR's weights and the status.
void k_cocg_update(const KrylovState &k, hipStream_t s, int nrec, bool fold, bool qmr);
void k_cocg_scalar(const KrylovState &k, hipStream_t s, bool qmr);

// r_true = b - Ax (Ax given in `ax`) for RHS with check[r]; writes norms into partial/scal.
void k_true_residual(const KrylovState &k, const c64 *ax, hipStream_t s);
// Restart RHS with restart[r] from the current x: r holds the true residual;
// rh = r, p = v = 0, fresh scalars, inner threshold max(tol |b|, inner_tol |r|);
// QMR: raw iterate k.s = x, smoothed residual k.t = r.
void k_restart(const KrylovState &k, const int *restart, double tol, double inner_tol, int solver,
               hipStream_t s);

// v <- S v (inverse: S^-1 v) for the Jacobi-scaled solve (see Scaling)
void launch_scale(const Geometry &g, c64 *v, int nrhs, const c64 *scl, int ncomp, const uint8_t *comp, bool inverse,
                  hipStream_t s);
void launch_incident(const Geometry &g, const int32_t *ijk, const RhsDev *rhs, int nrhs, double kd,
                     c64 *e, hipStream_t s);
// Sums per RHS: [0] = sum Im(conj(E) . P), [1] = sum_c (-Im(ainv_c) - (2/3) kd^3) |P_c|^2
// (ainv [nrhs][ncomp][3])
void launch_cross_sums(const Geometry &g, const int32_t *ijk, const RhsDev *rhs, int nrhs, double kd,
                       const c64 *P, const c64 *ainv, int ncomp, const uint8_t *comp, double *partial,
                       double *sums, hipStream_t s);

// Device blocks from the library's per-device cache (see devmem.cpp): the
// granted size (>= bytes) must be passed back on release, and a block may be
// released only when no queued work uses it any more.
void *dev_alloc(int device, size_t bytes, size_t *granted);
void dev_release(int device, void *p, size_t granted);
// pinned host blocks from a process-wide pool (reused, never freed)
void *pinned_alloc(size_t bytes, size_t *granted);
void pinned_release(void *p, size_t granted);

// Gauss-Legendre nodes and weights on [-1, 1] (host, Newton iteration).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
// Far-field quadrature sums over ndir directions (one RHS): sums[0..2] =
// sum w |F_perp|^2, sum w mu |F_perp|^2, sum w mu^2 |F_perp|^2.
size_t far_field_scratch_bytes(const Geometry &g, int ndir);
void launch_far_field(const Geometry &g, const int *cell_site, const c64 *P, double kd, const double *dirs,
                      const double *mu, const double *w, int ndir, double *scratch, double *sums, hipStream_t s);

// Phase sums F(n_d) = sum_j P_j exp(-i kd n_d . r_j) for ndir directions (one
// RHS): F host-visible device [ndir][3] complex; scratch as for the far field.
void launch_far_amplitudes(const Geometry &g, const int *cell_site, const c64 *P, double kd, const double *dirs,
                           int ndir, double *scratch, double *F, hipStream_t s);

// Near field: embed P [nrhs][n][3] into the extended box (P_ext[r][map[i]] =
// P[r][i]; P_ext zeroed by the caller), and E = E_inc - AP_ext on the box
// (fac[c] = 3 / (eps_c + 2) at points with cellc >= 0, or fac = nullptr).
void launch_near_field_embed(const c64 *P, int64_t n, const int *map, c64 *Pext, int64_t ne, int nrhs,
                             hipStream_t s);
void launch_near_field_combine(const c64 *AP, int64_t ne, int X, int Y, const int margin[3], const RhsDev *rhs,
                               int nrhs, double kd, const int *cellc, const c64 *fac, c64 *E, hipStream_t s);

// --------------------------------------------------------------- host side --
std::vector<int32_t> make_sites(int shape, const double shpar[3], int32_t box[3]);
void orient_rhs(double beta, double theta, double phi, const c64 e01[3], int which, RhsDev &out);
// Orientation sampling of §20: n points min + j (max - min) / n with weights
// 1/n (beta, phi); theta uniform in cos(theta), Simpson weights for odd n
// (end points included), midpoints with equal weights for even n.
void periodic_rule(double lo, double hi, int n, std::vector<double> &x, std::vector<double> &w);
void cos_theta_rule(double lo, double hi, int n, std::vector<double> &theta, std::vector<double> &w);
// Diagonal of the inverse polarizability tensor (a multiple of I except for
// GKDLDR) of one composition for one RHS.
void alpha_inverse(int kind, c64 m, double kd, const double khat[3], const c64 e[3], c64 out[3]);

}  // namespace dda
