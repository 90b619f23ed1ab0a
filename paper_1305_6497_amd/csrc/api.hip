// The C ABI (include/dda.h): target handles, the BiCGSTAB driver with FP64
// true-residual refinement, cross sections and diagnostics.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dda_internal.hpp"
#include "fft_lds.hpp"
#include "nearfield.hpp"
#include "reduce.hpp"

using namespace dda;

namespace dda {
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
}  // namespace dda

// Default of dda_solve_opts.fold_records: folding costs every consuming block
// a read of all records, O(blocks x records), which is cheap up to about this.
constexpr int kFoldRecords = 1024;

struct dda_target {
  int device = 0;
  hipStream_t stream = nullptr;
  Geometry g{};
  double kd = 0, aeff = 0;
  int alpha_kind = 0;
  int ncomp = 1;
  std::vector<c64> m;
  AxisPlan px{}, py{}, pz{};
  Twiddles tx, ty, tz;
  int32_t *d_ijk = nullptr;
  uint8_t *d_comp = nullptr;
  int *d_cell_site = nullptr;
  int4 *d_rowtab = nullptr;       // see MatvecArgs::rowtab
  c64 *d_ghat64 = nullptr;
  c32 *d_ghat32 = nullptr;
  // workspace, grown on demand
  int ws_nrhs = 0;
  void *d_bufA = nullptr, *d_bufB = nullptr;
  // Krylov state, grown on demand
  int kr_nrhs = 0;
  KrylovState k;
  c64 *d_ainv = nullptr;
  c64 *d_scl = nullptr;            // Jacobi scaling s per RHS, composition, component
  bool jacobi_active = false;      // inside a dda_solve with opts->jacobi
  RhsDev *d_rhs = nullptr;
  double *d_sums = nullptr;
  int *d_restart = nullptr;
  // host staging of the per-RHS uploads; kept alive until the copy that
  // reads them has completed (upload_done)
  std::vector<RhsDev> h_rhs;
  std::vector<c64> h_ainv;
  std::vector<c64> h_scl;
  hipEvent_t upload_done = nullptr;
  // pinned host copies of the per-RHS status and scalars read at every host
  // check of a solve (a pinned copy returns sooner than a pageable one)
  int *h_status = nullptr;
  c64 *h_scal = nullptr;
  size_t h_status_granted = 0, h_scal_granted = 0;
  int h_nrhs = 0;
  // captured block of BiCGSTAB iterations (see run_iterations)
  hipGraphExec_t graph = nullptr;
  int graph_nrhs = 0, graph_prec = -1, graph_k = 0, graph_solver = -1, graph_fold = -1, graph_jacobi = -1,
      graph_vec32 = -1;
  // products with at most this many partial records per RHS hand their
  // scalar (alpha, omega) to the consuming kernel, which computes it in every
  // block; larger ones get a one-block kernel first (set by each solve)
  int fold_records = kFoldRecords;
  // plan variants forced by dda_set_plan_variant (-1: the tuned table's)
  int zvar = -1;
  int xvar[2] = {-1, -1};
  uint64_t graph_gen = 0;
  uint64_t buffer_gen = 0;        // bumped whenever workspaces are reallocated
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // per-pass event timing of the products inside dda_solve (dda_set_pass_timing):
  // every pt_every-th eager product records six events (before each pass and
  // after the last); the call reads them back at its host synchronisations
  static constexpr int kPassTimingSets = 512;
  int pt_every = 0, pt_used = 0;
  int64_t pt_seen = 0;
  bool pt_active = false;          // inside dda_solve, not under graph capture
  std::vector<hipEvent_t> pt_ev;   // kPassTimingSets * 6
  std::vector<int> pt_prec;
  double pt_ms[2][5] = {};
  int64_t pt_n[2] = {};
  uint64_t bytes = 0;
  struct Block {
    void *p;
    size_t bytes, granted;
  };
  std::vector<Block> allocs;
  // one event per stream this handle has queued work on, recorded after each
  // call, so its blocks go back to the device cache only once that work is done
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;

  template <typename P>
  P *alloc(size_t bytes_) {
    size_t granted = 0;
    void *p = dev_alloc(device, bytes_, &granted);
    allocs.push_back({p, bytes_, granted});
    bytes += bytes_;
    return static_cast<P *>(p);
  }
  void note_use(hipStream_t s) {
    for (auto &u : uses)
      if (u.first == s) {
        (void)hipEventRecord(u.second, s);
        return;
      }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);      // cannot track: wait now instead
      return;
    }
    (void)hipEventRecord(e, s);
    uses.push_back({s, e});
  }
  // event sets for this product, or nullptr (timing off, not sampled, all sets in use)
  const hipEvent_t *pt_next(int precision) {
    if (!pt_active || pt_every <= 0 || pt_used >= kPassTimingSets) return nullptr;
    if (pt_seen++ % pt_every != 0) return nullptr;
    pt_prec[pt_used] = precision;
    return &pt_ev[(size_t)6 * pt_used++];
  }
  // add the recorded sets to the sums; called once the stream they were
  // recorded on has been synchronised
  void pt_harvest() {
    for (int i = 0; i < pt_used; ++i) {
      float ms[5];
      bool ok = true;
      for (int k = 0; k < 5 && ok; ++k)
        ok = hipEventElapsedTime(&ms[k], pt_ev[(size_t)6 * i + k], pt_ev[(size_t)6 * i + k + 1]) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        continue;
      }
      const int p = pt_prec[i] == DDA_MIXED ? 1 : 0;
      for (int k = 0; k < 5; ++k) pt_ms[p][k] += ms[k];
      ++pt_n[p];
    }
    pt_used = 0;
  }
  // wait for every piece of work this handle has queued
  void quiesce() {
    for (auto &u : uses) (void)hipEventSynchronize(u.second);
    if (upload_done) (void)hipEventSynchronize(upload_done);
    if (stream) (void)hipStreamSynchronize(stream);
  }
  void release(void *p) {
    if (!p) return;
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i].p == p) {
        quiesce();
        bytes -= allocs[i].bytes;
        dev_release(device, p, allocs[i].granted);
        allocs.erase(allocs.begin() + i);
        return;
      }
  }
  ~dda_target() {
    (void)hipSetDevice(device);
    quiesce();
    if (graph) (void)hipGraphExecDestroy(graph);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    for (hipEvent_t e : pt_ev) (void)hipEventDestroy(e);
    for (auto &a : allocs) dev_release(device, a.p, a.granted);
    for (auto &u : uses) (void)hipEventDestroy(u.second);
    if (upload_done) (void)hipEventDestroy(upload_done);
    pinned_release(h_status, h_status_granted);
    pinned_release(h_scal, h_scal_granted);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// Pass timing is on inside dda_solve only; sets not read back when the call
// ends (an error path) are dropped.
struct PassTimingScope {
  dda_target *t;
  explicit PassTimingScope(dda_target *t_) : t(t_) { t->pt_active = true; }
  ~PassTimingScope() {
    t->pt_active = false;
    t->pt_used = 0;
  }
};

// The search direction p and its product in FP32 for the duration of a
// DDA_MIXED_V32 solve.
struct Vec32Scope {
  dda_target *t;
  Vec32Scope(dda_target *t_, bool on) : t(t_) { t->k.vec32 = on; }
  ~Vec32Scope() { t->k.vec32 = false; }
};

// The products of a dda_solve with opts->jacobi use the scaling; others never.
struct JacobiScope {
  dda_target *t;
  JacobiScope(dda_target *t_, bool on) : t(t_) { t->jacobi_active = on; }
  ~JacobiScope() { t->jacobi_active = false; }
};

// Records, when the call returns, that the handle queued work on stream s.
struct StreamUse {
  dda_target *t;
  hipStream_t s;
  ~StreamUse() { t->note_use(s); }
};

namespace {

template <typename F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return DDA_ENOMEM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return DDA_EDEVICE;
  } catch (...) {
    set_error("unknown error");
    return DDA_EDEVICE;
  }
}

int grid_extent(int n) { return std::max(2, next_smooth(2 * n - 1)); }

Geometry make_geometry(int nx, int ny, int nz, int64_t n) {
  Geometry g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.Mx = grid_extent(nx);
  g.My = grid_extent(ny);
  g.Mz = grid_extent(nz);
  if (g.Mx > kMaxLen || g.My > kMaxLen || g.Mz > kMaxLen)
    throw Error{DDA_ENOTSUP, "padded FFT extent exceeds 512 (box extent > 256)"};
  g.Mxh = g.Mx / 2 + 1;
  g.Myh = g.My / 2 + 1;
  g.Mzh = g.Mz / 2 + 1;
  g.n_sites = n;
  return g;
}

void validate_desc(const dda_target_desc *d, bool need_sites) {
  DDA_REQUIRE(d != nullptr, "desc is NULL");
  DDA_REQUIRE(d->nx >= 1 && d->ny >= 1 && d->nz >= 1, "box extents must be >= 1");
  DDA_REQUIRE(d->n_sites >= 1, "n_sites must be >= 1");
  DDA_REQUIRE(d->n_sites <= (int64_t)d->nx * d->ny * d->nz, "more sites than box cells");
  DDA_REQUIRE(d->n_sites < (int64_t)INT32_MAX / 3, "too many sites");
  DDA_REQUIRE(d->n_comp >= 1 && d->n_comp <= 255, "n_comp must be in 1..255");
  DDA_REQUIRE(d->m != nullptr, "m is NULL");
  DDA_REQUIRE(std::isfinite(d->kd) && d->kd > 0.0, "kd must be finite and > 0");
  DDA_REQUIRE(d->alpha_kind == DDA_ALPHA_LDR || d->alpha_kind == DDA_ALPHA_CMRR || d->alpha_kind == DDA_ALPHA_FCD ||
                  d->alpha_kind == DDA_ALPHA_GKDLDR,
              "unknown alpha_kind");
  if (d->alpha_kind == DDA_ALPHA_FCD) DDA_REQUIRE(d->kd < 3.14159265358979323846, "FCD requires kd < pi");
  for (int c = 0; c < d->n_comp; ++c) {
    const std::complex<double> m(d->m[c].re, d->m[c].im);
    DDA_REQUIRE(std::isfinite(m.real()) && std::isfinite(m.imag()), "refractive index must be finite");
    DDA_REQUIRE(std::abs(m * m + 2.0) > 1e-12, "m^2 = -2: Clausius-Mossotti polarizability is singular");
    DDA_REQUIRE(std::abs(m * m - 1.0) > 1e-300, "m = 1: target has no polarizability");
  }
  if (need_sites) DDA_REQUIRE(d->ijk != nullptr, "ijk is NULL");
}

bool validity_warning(const dda_target_desc *d) {
  bool w = false;
  for (int c = 0; c < d->n_comp; ++c) {
    const std::complex<double> m(d->m[c].re, d->m[c].im);
    if (std::abs(m) * d->kd >= 1.0 || std::abs(m - 1.0) > 2.0) w = true;     // §2
  }
  return w;
}

void make_twiddles(dda_target *t, Twiddles &tw, int L) {
  std::vector<c64> h64(L);
  std::vector<c32> h32(L);
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < L; ++n) {
    const double a = 2.0 * pi * double(n) / double(L);
    h64[n] = c64{std::cos(a), -std::sin(a)};
    h32[n] = c32{float(h64[n].x), float(h64[n].y)};
  }
  tw.L = L;
  tw.d64 = t->alloc<c64>(sizeof(c64) * L);
  tw.d32 = t->alloc<c32>(sizeof(c32) * L);
  // on the handle's own (non-blocking) stream: no ordering against other streams
  DDA_HIP(hipMemcpyAsync(tw.d64, h64.data(), sizeof(c64) * L, hipMemcpyHostToDevice, t->stream));
  DDA_HIP(hipMemcpyAsync(tw.d32, h32.data(), sizeof(c32) * L, hipMemcpyHostToDevice, t->stream));
  DDA_HIP(hipStreamSynchronize(t->stream));
}

size_t workspace_bytes(const Geometry &g, int nrhs) {
  const size_t a = std::max(g.a_elems(true) * sizeof(c32), g.a_elems(false) * sizeof(c64));
  const size_t b = std::max(g.b_elems(true) * sizeof(c32), g.b_elems(false) * sizeof(c64));
  return (a + b) * (size_t)nrhs;
}

size_t krylov_bytes(const Geometry &g, int nrhs) {
  const int64_t n3 = 3 * g.n_sites;
  const size_t vec = (size_t)n3 * sizeof(c64) * nrhs;
  const int nblk = std::max(krylov_blocks(n3), std::max(xpass_blocks(g, true), xpass_blocks(g, false)));
  return 9 * vec + 2 * (size_t)nrhs * nblk * kPart * sizeof(double) + (size_t)nrhs * kScal * sizeof(c64) +
         4 * (size_t)nrhs * sizeof(int) + (size_t)nrhs * (sizeof(RhsDev) + 2 * sizeof(double)) +
         2 * (size_t)nrhs * 255 * 3 * sizeof(c64);
}

// Workspaces grow on demand.  Work already queued on s may still use the old
// buffers, so s is drained before they are freed; the new buffers are zeroed
// on s itself, ordered before the kernels that follow (a memset on the null
// stream would not be ordered against a non-blocking caller stream).
void ensure_workspace(dda_target *t, int nrhs, hipStream_t s) {
  if (t->ws_nrhs >= nrhs) return;
  DDA_HIP(hipStreamSynchronize(s));
  t->release(t->d_bufA);
  t->release(t->d_bufB);
  t->d_bufA = t->d_bufB = nullptr;
  const Geometry &g = t->g;
  const size_t a = std::max(g.a_elems(true) * sizeof(c32), g.a_elems(false) * sizeof(c64)) * nrhs;
  const size_t b = std::max(g.b_elems(true) * sizeof(c32), g.b_elems(false) * sizeof(c64)) * nrhs;
  t->d_bufA = t->alloc<void>(a);
  t->d_bufB = t->alloc<void>(b);
  // zero once: tile columns beyond Mx are never written by the passes
  DDA_HIP(hipMemsetAsync(t->d_bufA, 0, a, s));
  DDA_HIP(hipMemsetAsync(t->d_bufB, 0, b, s));
  t->ws_nrhs = nrhs;
  ++t->buffer_gen;
}

void ensure_krylov(dda_target *t, int nrhs, hipStream_t s) {
  if (t->kr_nrhs >= nrhs) {
    t->k.nrhs = nrhs;
    return;
  }
  DDA_HIP(hipStreamSynchronize(s));
  if (t->upload_done) DDA_HIP(hipEventSynchronize(t->upload_done));
  KrylovState &k = t->k;
  for (c64 *p : {k.x, k.r, k.rh, k.p, k.v, k.s, k.t, k.b, k.u2}) t->release(p);
  t->release(k.partial);
  t->release(k.partial2);
  t->release(k.scal);
  t->release(k.active);
  t->release(k.status);
  t->release(k.check);
  t->release(t->d_ainv);
  t->release(t->d_scl);
  t->release(t->d_rhs);
  t->release(t->d_sums);
  t->release(t->d_restart);
  const int64_t n3 = 3 * t->g.n_sites;
  const size_t vec = (size_t)n3 * sizeof(c64) * nrhs;
  k.n3 = n3;
  k.nblk = krylov_blocks(n3);
  k.nrec = std::max(k.nblk, std::max(xpass_blocks(t->g, true), xpass_blocks(t->g, false)));
  k.x = t->alloc<c64>(vec);
  k.r = t->alloc<c64>(vec);
  k.rh = t->alloc<c64>(vec);
  k.p = t->alloc<c64>(vec);
  k.v = t->alloc<c64>(vec);
  k.s = t->alloc<c64>(vec);
  k.t = t->alloc<c64>(vec);
  k.b = t->alloc<c64>(vec);
  k.u2 = t->alloc<c64>(vec);
  k.partial = t->alloc<double>((size_t)nrhs * k.nrec * kPart * sizeof(double));
  k.partial2 = t->alloc<double>((size_t)nrhs * k.nblk * kPart * sizeof(double));
  k.scal = t->alloc<c64>((size_t)nrhs * kScal * sizeof(c64));
  k.active = t->alloc<int>(nrhs * sizeof(int));
  k.status = t->alloc<int>(nrhs * sizeof(int));
  k.check = t->alloc<int>(nrhs * sizeof(int));
  t->d_restart = t->alloc<int>(nrhs * sizeof(int));
  t->d_ainv = t->alloc<c64>((size_t)nrhs * t->ncomp * 3 * sizeof(c64));
  t->d_scl = t->alloc<c64>((size_t)nrhs * t->ncomp * 3 * sizeof(c64));
  t->d_rhs = t->alloc<RhsDev>(nrhs * sizeof(RhsDev));
  t->d_sums = t->alloc<double>(3 * nrhs * sizeof(double));
  t->kr_nrhs = nrhs;
  k.nrhs = nrhs;
  ++t->buffer_gen;
}

// Validate and normalise one RHS.
void check_rhs(const dda_rhs &q, RhsDev &rd) {
  const double kn = std::sqrt(q.khat[0] * q.khat[0] + q.khat[1] * q.khat[1] + q.khat[2] * q.khat[2]);
  DDA_REQUIRE(std::fabs(kn - 1.0) <= 1e-12, "khat must be a unit vector");
  double en = 0.0;
  for (int a = 0; a < 3; ++a) en += q.e[a].re * q.e[a].re + q.e[a].im * q.e[a].im;
  en = std::sqrt(en);
  DDA_REQUIRE(en > 0.0 && std::isfinite(en), "polarization must be non-zero and finite");
  std::complex<double> dot = 0.0;
  for (int a = 0; a < 3; ++a) {
    rd.khat[a] = q.khat[a];
    rd.e[a] = c64{q.e[a].re / en, q.e[a].im / en};
    dot += q.khat[a] * std::complex<double>(rd.e[a].x, rd.e[a].y);
  }
  DDA_REQUIRE(std::abs(dot) <= 1e-9, "polarization must be transverse (khat . e = 0)");
}

// Validate and normalise the RHS; fill per-RHS descriptions and 1/alpha.
void prepare_rhs(dda_target *t, const dda_rhs *rhs, int nrhs, std::vector<RhsDev> &rd, std::vector<c64> &ainv) {
  DDA_REQUIRE(rhs != nullptr, "rhs is NULL");
  rd.resize(nrhs);
  ainv.resize((size_t)nrhs * t->ncomp * 3);
  for (int r = 0; r < nrhs; ++r) {
    check_rhs(rhs[r], rd[r]);
    for (int c = 0; c < t->ncomp; ++c)
      alpha_inverse(t->alpha_kind, t->m[c], t->kd, rd[r].khat, rd[r].e, &ainv[((size_t)r * t->ncomp + c) * 3]);
  }
}

void upload_rhs(dda_target *t, const std::vector<RhsDev> &rd, const std::vector<c64> &ainv, hipStream_t s,
                const std::vector<c64> *scl = nullptr) {
  if (!t->upload_done) DDA_HIP(hipEventCreateWithFlags(&t->upload_done, hipEventDisableTiming));
  DDA_HIP(hipEventSynchronize(t->upload_done));      // previous upload has read the staging
  t->h_rhs = rd;
  t->h_ainv = ainv;
  DDA_HIP(hipMemcpyAsync(t->d_rhs, t->h_rhs.data(), rd.size() * sizeof(RhsDev), hipMemcpyHostToDevice, s));
  DDA_HIP(hipMemcpyAsync(t->d_ainv, t->h_ainv.data(), ainv.size() * sizeof(c64), hipMemcpyHostToDevice, s));
  if (scl) {
    t->h_scl = *scl;
    DDA_HIP(hipMemcpyAsync(t->d_scl, t->h_scl.data(), scl->size() * sizeof(c64), hipMemcpyHostToDevice, s));
  }
  DDA_HIP(hipEventRecord(t->upload_done, s));
}

// Symmetric diagonal (Jacobi) scaling of the system: s = (1/alpha)^(-1/2)
// (principal root) per RHS, composition and component; 1/alpha is replaced by
// the diagonal of S A S, s (1/alpha) s (= 1 up to rounding).
void jacobi_scaling(std::vector<c64> &ainv, std::vector<c64> &scl) {
  scl.resize(ainv.size());
  for (size_t i = 0; i < ainv.size(); ++i) {
    const std::complex<double> a(ainv[i].x, ainv[i].y);
    const std::complex<double> sv = 1.0 / std::sqrt(a);
    const std::complex<double> dg = sv * a * sv;
    scl[i] = c64{sv.real(), sv.imag()};
    ainv[i] = c64{dg.real(), dg.imag()};
  }
}

// The product on explicit 1/alpha and work buffers (see MatvecArgs).
void matvec_on(dda_target *t, int precision, const c64 *in, c64 *out, int nrhs, const int *mask, const c64 *ainv,
               void *bufA, void *bufB, hipStream_t s, const hipEvent_t *ev = nullptr, int only_pass = -1,
               int reps = 1, const FuseArgs *fuse = nullptr) {
  if (!ev && only_pass < 0) ev = t->pt_next(precision);
  MatvecArgs a{};
  // FP32 vectors only in the iterations' FP32 products: COCG's p -> q and
  // BiCGSTAB's p -> v (in mode 3 or 1); BiCGSTAB's s -> t product (in mode 2)
  // keeps s and t in FP64 but reads the FP32 v in its fused update
  const bool v32 = t->k.vec32 && precision == DDA_MIXED && fuse != nullptr;
  a.vec32 = v32 && fuse->in_mode != 2;
  a.vvec32 = v32;
  if (t->jacobi_active) {
    a.scl.s = t->d_scl;
    a.scl.comp = t->d_comp;
    a.scl.ncomp = t->ncomp;
  }
  if (fuse) a.fuse = *fuse;
  a.in = in;
  a.out = out;
  a.nrhs = nrhs;
  a.mask = mask;
  a.ainv = ainv;
  a.ncomp = t->ncomp;
  a.comp = t->d_comp;
  a.cell_site = t->d_cell_site;
  a.rowtab = t->d_rowtab;
  a.bufA = bufA;
  a.bufB = bufB;
  a.px = t->px;
  a.py = t->py;
  a.pz = t->pz;
  a.zvar = t->zvar;
  a.xvar[0] = t->xvar[0];
  a.xvar[1] = t->xvar[1];
  if (precision == DDA_MIXED) {
    a.ghat = t->d_ghat32;
    a.twx = t->tx.d32;
    a.twy = t->ty.d32;
    a.twz = t->tz.d32;
    launch_matvec<float>(t->g, a, s, ev, only_pass, reps);
  } else {
    a.ghat = t->d_ghat64;
    a.twx = t->tx.d64;
    a.twy = t->ty.d64;
    a.twz = t->tz.d64;
    launch_matvec<double>(t->g, a, s, ev, only_pass, reps);
  }
}

void matvec(dda_target *t, int precision, const c64 *in, c64 *out, int nrhs, const int *mask, hipStream_t s,
            const hipEvent_t *ev = nullptr, int only_pass = -1, int reps = 1, const FuseArgs *fuse = nullptr) {
  matvec_on(t, precision, in, out, nrhs, mask, t->d_ainv, t->d_bufA, t->d_bufB, s, ev, only_pass, reps, fuse);
}

// One BiCGSTAB iteration for every active RHS of the block: 12 kernels
// (14 when the products have more than fold_records records).
//   product 1: x-forward forms p = r + beta (p - omega v); x-inverse writes
//              v = A p and partial sums of <rh, v>
//   product 2: x-forward computes alpha = rho / <rh, v> (every block, from
//              the records, or one block before it) and forms s = r - alpha v;
//              x-inverse writes t = A s and partial sums of <t, s>, <t, t>
//   update:    omega = <t, s> / <t, t> (likewise),
//              x += alpha p + omega s, r = s - omega t with <rh, r>, |r|^2;
//              rho, beta and the convergence status.
void iteration(dda_target *t, int precision, hipStream_t s) {
  KrylovState &k = t->k;
  const int nrec = xpass_blocks(t->g, precision == DDA_MIXED);
  const bool fold = nrec <= t->fold_records;
  FuseArgs f;
  f.r = k.r;
  f.v = k.v;
  f.rh = k.rh;
  f.scal = k.scal;
  f.active = k.active;
  f.status = k.status;
  f.partial = k.partial;
  f.rec_cap = k.nrec;
  f.in_mode = 1;
  f.out_mode = 1;
  f.w = k.p;
  matvec(t, precision, k.p, k.v, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  f.in_mode = 2;
  if (fold) {
    f.fold_alpha = 1;
    f.nrec = nrec;
  } else {
    k_scalar_alpha(k, s, nrec);
  }
  f.out_mode = 2;
  f.w = k.s;
  matvec(t, precision, k.s, k.t, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k_update_xr(k, s, nrec, fold);
  k_scalar_rho(k, s);
}

// One BiCGstab(2) cycle (two BiCG steps and the minimal-residual step, four
// products) for every active RHS: 25 kernels.  Vectors: r = r_0, s = r_1,
// t = r_2, p = u_0, v = u_1, u2 = u_2, rh = the shadow residual rt.
//   product 1: u0 = r0 - beta u0 (fused), u1 = A u0, <rt, u1>; alpha
//   product 2: r0 -= alpha u1, x += alpha u0 (fused), r1 = A r0, <rt, r1>; beta
//   product 3: u1 = r1 - beta u1, u0 = r0 - beta u0 (fused), u2 = A u1, <rt, u2>; alpha
//   product 4: r1 -= alpha u2, r0 -= alpha u1, x += alpha u0 (fused), r2 = A r1,
//              Gram sums of r0, r1, r2; g1, g2 = omega
//   update:    x += g1 r0 + g2 r1, r0 -= g1 r1 + g2 r2, u0 -= g1 u1 + g2 u2 with
//              <rt, r0>, |r0|^2; next beta and the convergence status.
void cycle2(dda_target *t, int precision, hipStream_t s) {
  KrylovState &k = t->k;
  const int nrec = xpass_blocks(t->g, precision == DDA_MIXED);
  FuseArgs f;
  f.rh = k.rh;
  f.scal = k.scal;
  f.active = k.active;
  f.status = k.status;
  f.partial = k.partial;
  f.rec_cap = k.nrec;
  f.in_mode = 3;
  auto ax = [&](int i, c64 *d, const c64 *a, const c64 *b, int slot, int neg) {
    f.ax_d[i] = d;
    f.ax_a[i] = a;
    f.ax_b[i] = b;
    f.ax_slot[i] = slot;
    f.ax_neg[i] = neg;
  };
  f.out_mode = 1;
  f.nax = 1;
  ax(0, k.p, k.r, k.p, S_BETA, 1);
  matvec(t, precision, k.p, k.v, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k_scalar_alpha(k, s, nrec);
  f.nax = 2;
  ax(0, k.r, k.r, k.v, S_ALPHA, 1);
  ax(1, k.x, k.x, k.p, S_ALPHA, 0);
  matvec(t, precision, k.r, k.s, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k2_scalar_rho1(k, s, nrec);
  f.nax = 2;
  ax(0, k.v, k.s, k.v, S_BETA, 1);
  ax(1, k.p, k.r, k.p, S_BETA, 1);
  matvec(t, precision, k.v, k.u2, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k_scalar_alpha(k, s, nrec);
  f.nax = 3;
  ax(0, k.s, k.s, k.u2, S_ALPHA, 1);
  ax(1, k.r, k.r, k.v, S_ALPHA, 1);
  ax(2, k.x, k.x, k.p, S_ALPHA, 0);
  f.out_mode = 3;
  f.r = k.r;
  matvec(t, precision, k.s, k.t, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k2_scalar_mr(k, s, nrec);
  k2_update_mr(k, s);
  k_scalar_rho(k, s, 2, -1.0);
}

// One COCG / QMR iteration (one product) for every active RHS: 7 kernels
// (8 when the product has more than fold_records records).
//   p = r + beta p (fused into the x-forward pass), q = A p -> v with p^T q
//   (x-inverse records); alpha, x and r (QMR: the smoothing first); next
//   beta, QMR's weight and the convergence status.
void cocg_iteration(dda_target *t, int precision, bool qmr, hipStream_t s) {
  KrylovState &k = t->k;
  const int nrec = xpass_blocks(t->g, precision == DDA_MIXED);
  FuseArgs f;
  f.scal = k.scal;
  f.active = k.active;
  f.status = k.status;
  f.partial = k.partial;
  f.rec_cap = k.nrec;
  f.in_mode = 3;
  f.nax = 1;
  f.ax_d[0] = k.p;
  f.ax_a[0] = k.r;
  f.ax_b[0] = k.p;
  f.ax_slot[0] = S_BETA;
  f.ax_neg[0] = 0;
  f.out_mode = 4;
  matvec(t, precision, k.p, k.v, k.nrhs, k.active, s, nullptr, -1, 1, &f);
  k_cocg_update(k, s, nrec, nrec <= t->fold_records, qmr);
  k_cocg_scalar(k, s, qmr);
}

void step(dda_target *t, int precision, int solver, hipStream_t s) {
  if (solver == DDA_SOLVER_BICGSTAB2) cycle2(t, precision, s);
  else if (solver == DDA_SOLVER_COCG || solver == DDA_SOLVER_QMR)
    cocg_iteration(t, precision, solver == DDA_SOLVER_QMR, s);
  else iteration(t, precision, s);
}

// K BiCGSTAB iterations (or K BiCGstab(2) cycles) on stream s.  With use_graph the block is captured
// once into a HIP graph on the handle's own stream (capture needs a non-null
// stream) and replayed; events order it after the work already queued on s
// and make s wait for it.  Every kernel reads its scalars and flags from
// device memory, so one captured block serves every replay; the graph is
// captured again when the block shape or the buffers change.  The captured
// kernels contain no memset nodes.
void run_iterations(dda_target *t, int precision, int solver, int K, bool use_graph, hipStream_t s) {
  if (!use_graph) {
    for (int it = 0; it < K; ++it) step(t, precision, solver, s);
    return;
  }
  if (!t->ev_in) {
    DDA_HIP(hipEventCreateWithFlags(&t->ev_in, hipEventDisableTiming));
    DDA_HIP(hipEventCreateWithFlags(&t->ev_out, hipEventDisableTiming));
  }
  if (!t->graph || t->graph_nrhs != t->k.nrhs || t->graph_prec != precision || t->graph_k != K ||
      t->graph_solver != solver || t->graph_fold != t->fold_records || t->graph_gen != t->buffer_gen ||
      t->graph_jacobi != (int)t->jacobi_active || t->graph_vec32 != (int)t->k.vec32) {
    if (t->graph) {
      DDA_HIP(hipGraphExecDestroy(t->graph));
      t->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    DDA_HIP(hipStreamBeginCapture(t->stream, hipStreamCaptureModeThreadLocal));
    const bool timing = t->pt_active;
    t->pt_active = false;        // no timing events inside the captured block
    try {
      for (int it = 0; it < K; ++it) step(t, precision, solver, t->stream);
    } catch (...) {
      t->pt_active = timing;
      (void)hipStreamEndCapture(t->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    t->pt_active = timing;
    DDA_HIP(hipStreamEndCapture(t->stream, &g));
    hipError_t e = hipGraphInstantiate(&t->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DDA_HIP(e);
    t->graph_nrhs = t->k.nrhs;
    t->graph_prec = precision;
    t->graph_solver = solver;
    t->graph_fold = t->fold_records;
    t->graph_jacobi = (int)t->jacobi_active;
    t->graph_vec32 = (int)t->k.vec32;
    t->graph_k = K;
    t->graph_gen = t->buffer_gen;
  }
  DDA_HIP(hipEventRecord(t->ev_in, s));
  DDA_HIP(hipStreamWaitEvent(t->stream, t->ev_in, 0));
  DDA_HIP(hipGraphLaunch(t->graph, t->stream));
  DDA_HIP(hipEventRecord(t->ev_out, t->stream));
  DDA_HIP(hipStreamWaitEvent(s, t->ev_out, 0));
}

// ------------------------------------------------- allocation-free product --
// dda_apply_noalloc keeps its work buffers in one static device array per GPU
// (the loader places it with the code object; it lives until the process
// ends): the per-RHS 1/alpha values first, then the two FFT work buffers.
constexpr int kNoAllocMaxRhsComp = 32;              // nrhs * n_comp per call
constexpr int kNoAllocMaxAinv = 3 * kNoAllocMaxRhsComp;   // tensor diagonals
constexpr size_t kNoAllocAinvBytes = 4096;          // >= kNoAllocMaxAinv * 16, keeps A 256-byte aligned
constexpr int kMaxDevices = 64;

// 1/alpha values travel as a kernel argument, so the call needs no host
// staging buffer and no copy node.
struct AinvArg {
  c64 v[kNoAllocMaxAinv];
  int n;
};

__global__ void k_fill_ainv(c64 *dst, AinvArg a) {
  if ((int)threadIdx.x < a.n) dst[threadIdx.x] = a.v[threadIdx.x];
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[DDA_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (which must be `device`).
// The host-side name of a __device__ array is only a stand-in; each GPU holds
// its own copy, looked up once per device and kept.
unsigned char *scratch_address(int device) {
  DDA_REQUIRE(device >= 0 && device < kMaxDevices, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *p = nullptr;
    DDA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DDA_REQUIRE(p != nullptr, "scratch array has no device address");
    g_scratch_dev[device] = p;
  }
  return static_cast<unsigned char *>(g_scratch_dev[device]);
}

}  // namespace

// ========================================================================= ABI

extern "C" {

const char *dda_last_error(void) { return g_last_error.c_str(); }

int32_t dda_next_smooth(int32_t n) { return next_smooth(n); }

double dda_aeff(int64_t n) { return std::cbrt(3.0 * double(n) / (4.0 * 3.14159265358979323846)); }

double dda_kd_from_x(double x, int64_t n) { return x / dda_aeff(n); }

int dda_make_sites(int32_t shape, const double shpar[3], int64_t *n_sites, int32_t box[3], int32_t *ijk,
                   int64_t capacity) {
  return guarded([&]() -> int {
    DDA_REQUIRE(shpar && n_sites && box, "NULL argument");
    for (int a = 0; a < 3; ++a) DDA_REQUIRE(std::isfinite(shpar[a]), "shape parameters must be finite");
    DDA_REQUIRE(shpar[0] <= 4096 && shpar[1] <= 4096 && shpar[2] <= 4096, "shape parameter too large");
    std::vector<int32_t> s = make_sites(shape, shpar, box);
    *n_sites = (int64_t)(s.size() / 3);
    if (ijk) {
      DDA_REQUIRE(capacity >= *n_sites, "ijk capacity too small");
      std::memcpy(ijk, s.data(), s.size() * sizeof(int32_t));
    }
    return DDA_OK;
  });
}

int dda_orientation_grid(double beta_min, double beta_max, int32_t nbeta, double theta_min, double theta_max,
                         int32_t ntheta, double phi_min, double phi_max, int32_t nphi, double *beta,
                         double *theta, double *phi, double *weight) {
  return guarded([&]() -> int {
    DDA_REQUIRE(beta && theta && phi && weight, "NULL argument");
    DDA_REQUIRE(nbeta >= 1 && ntheta >= 1 && nphi >= 1, "orientation counts must be >= 1");
    for (double v : {beta_min, beta_max, theta_min, theta_max, phi_min, phi_max})
      DDA_REQUIRE(std::isfinite(v), "angles must be finite");
    std::vector<double> b, wb, t, wt, p, wp;
    periodic_rule(beta_min, beta_max, nbeta, b, wb);
    cos_theta_rule(theta_min, theta_max, ntheta, t, wt);
    periodic_rule(phi_min, phi_max, nphi, p, wp);
    for (int it = 0; it < ntheta; ++it)
      for (int ip = 0; ip < nphi; ++ip)
        for (int ib = 0; ib < nbeta; ++ib) {
          const size_t i = ((size_t)it * nphi + ip) * nbeta + ib;
          beta[i] = b[ib];
          theta[i] = t[it];
          phi[i] = p[ip];
          weight[i] = wt[it] * wp[ip] * wb[ib];
        }
    return DDA_OK;
  });
}

int dda_orient_rhs(double beta, double theta, double phi, const dda_c64 e01_lf[3], int32_t which, dda_rhs *out) {
  return guarded([&]() -> int {
    DDA_REQUIRE(e01_lf && out, "NULL argument");
    c64 e[3];
    for (int a = 0; a < 3; ++a) e[a] = c64{e01_lf[a].re, e01_lf[a].im};
    RhsDev rd;
    orient_rhs(beta, theta, phi, e, which, rd);
    for (int a = 0; a < 3; ++a) {
      out->khat[a] = rd.khat[a];
      out->e[a].re = rd.e[a].x;
      out->e[a].im = rd.e[a].y;
    }
    return DDA_OK;
  });
}

int dda_footprint_bytes(const dda_target_desc *desc, int32_t nrhs, const dda_solve_opts *opts, uint64_t *bytes) {
  return guarded([&]() -> int {
    validate_desc(desc, false);
    DDA_REQUIRE(bytes != nullptr, "bytes is NULL");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    (void)opts;
    const Geometry g = make_geometry(desc->nx, desc->ny, desc->nz, desc->n_sites);
    const size_t M = (size_t)g.Mx * g.My * g.Mz;
    const size_t fixed = (size_t)desc->n_sites * (3 * sizeof(int32_t) + 1) + (size_t)g.nx * g.ny * g.nz * sizeof(int) +
                         6 * g.oct_elems() * (sizeof(c64) + sizeof(c32)) +
                         (size_t)(g.Mx + g.My + g.Mz) * (sizeof(c64) + sizeof(c32));
    const size_t setup_transient = 6 * M * sizeof(c64);
    const size_t solve = workspace_bytes(g, nrhs) + krylov_bytes(g, nrhs);
    *bytes = fixed + std::max(setup_transient, solve);
    return DDA_OK;
  });
}

int dda_setup_target(const dda_target_desc *desc, dda_target **out) {
  return guarded([&]() -> int {
    DDA_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    validate_desc(desc, true);
    const int nx = desc->nx, ny = desc->ny, nz = desc->nz;
    const int64_t n = desc->n_sites;
    // cell -> site map; rejects sites outside the box and duplicates
    std::vector<int> cell((size_t)nx * ny * nz, -1);
    for (int64_t j = 0; j < n; ++j) {
      const int32_t x = desc->ijk[3 * j], y = desc->ijk[3 * j + 1], z = desc->ijk[3 * j + 2];
      DDA_REQUIRE(x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz, "site outside the box");
      int &c = cell[((size_t)z * ny + y) * nx + x];
      DDA_REQUIRE(c < 0, "duplicate site");
      c = (int)j;
    }
    if (desc->comp)
      for (int64_t j = 0; j < n; ++j) DDA_REQUIRE(desc->comp[j] < desc->n_comp, "composition index >= n_comp");
    std::unique_ptr<dda_target> t(new dda_target());
    t->device = desc->device;
    DDA_HIP(hipSetDevice(t->device));
    DDA_HIP(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
    t->g = make_geometry(nx, ny, nz, n);
    t->kd = desc->kd;
    t->aeff = dda_aeff(n);
    t->alpha_kind = desc->alpha_kind;
    t->ncomp = desc->n_comp;
    t->m.resize(t->ncomp);
    for (int c = 0; c < t->ncomp; ++c) t->m[c] = c64{desc->m[c].re, desc->m[c].im};
    t->px = make_axis_plan(t->g.Mx);
    t->py = make_axis_plan(t->g.My);
    t->pz = make_axis_plan(t->g.Mz);
    make_twiddles(t.get(), t->tx, t->g.Mx);
    make_twiddles(t.get(), t->ty, t->g.My);
    make_twiddles(t.get(), t->tz, t->g.Mz);
    t->d_ijk = t->alloc<int32_t>((size_t)n * 3 * sizeof(int32_t));
    DDA_HIP(hipMemcpyAsync(t->d_ijk, desc->ijk, (size_t)n * 3 * sizeof(int32_t), hipMemcpyHostToDevice,
                           t->stream));
    if (desc->comp && t->ncomp > 1) {
      t->d_comp = t->alloc<uint8_t>((size_t)n);
      DDA_HIP(hipMemcpyAsync(t->d_comp, desc->comp, (size_t)n, hipMemcpyHostToDevice, t->stream));
    }
    t->d_cell_site = t->alloc<int>(cell.size() * sizeof(int));
    DDA_HIP(hipMemcpyAsync(t->d_cell_site, cell.data(), cell.size() * sizeof(int), hipMemcpyHostToDevice,
                           t->stream));
    // rows as runs: {first site, first x, count}, the sites numbered row after
    // row; any other numbering disables the table.  An empty row takes the
    // first site of the next occupied one, so the first sites never decrease.
    std::vector<int4> rows((size_t)ny * nz);
    bool runs = true;
    int next = 0;
    for (size_t row = 0; row < rows.size() && runs; ++row) {
      const int *c = &cell[row * nx];
      int x0 = 0;
      while (x0 < nx && c[x0] < 0) ++x0;
      int len = 0;
      while (x0 + len < nx && c[x0 + len] == next + len) ++len;
      for (int x = x0 + len; x < nx; ++x)
        if (c[x] >= 0) runs = false;
      if (x0 < nx && len == 0) runs = false;
      rows[row] = int4{next, x0 < nx ? x0 : 0, len, 0};
      next += len;
    }
    if (runs) {
      t->d_rowtab = t->alloc<int4>(rows.size() * sizeof(int4));
      DDA_HIP(hipMemcpyAsync(t->d_rowtab, rows.data(), rows.size() * sizeof(int4), hipMemcpyHostToDevice,
                             t->stream));
    }
    const Geometry &g = t->g;
    const size_t M = (size_t)g.Mx * g.My * g.Mz;
    t->d_ghat64 = t->alloc<c64>(6 * g.oct_elems() * sizeof(c64));
    t->d_ghat32 = t->alloc<c32>(6 * g.oct_elems() * sizeof(c32));
    c64 *full = t->alloc<c64>(6 * M * sizeof(c64));
    launch_green_build(g, t->kd, full, t->d_ghat64, t->d_ghat32, t->tx, t->ty, t->tz, t->px, t->py, t->pz,
                       t->stream);
    DDA_HIP(hipStreamSynchronize(t->stream));
    t->release(full);
    const bool warn = validity_warning(desc);
    *out = t.release();
    if (warn) {
      set_error("validity warning: |m|kd >= 1 or |m-1| > 2 for some composition");
      return DDA_WVALIDITY;
    }
    return DDA_OK;
  });
}

int dda_target_get_info(const dda_target *t, dda_target_info *info) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && info, "NULL argument");
    info->box[0] = t->g.nx;
    info->box[1] = t->g.ny;
    info->box[2] = t->g.nz;
    info->grid[0] = t->g.Mx;
    info->grid[1] = t->g.My;
    info->grid[2] = t->g.Mz;
    info->n_sites = t->g.n_sites;
    info->kd = t->kd;
    info->aeff = t->aeff;
    info->device_bytes = t->bytes;
    for (int p = 0; p < 2; ++p) {
      info->zpass_variant[p] = t->zvar >= 0 ? t->zvar : tuned_variant(kPassZ, t->g.Mz, p == 0);
      info->xfwd_variant[p] = t->xvar[0] >= 0 ? t->xvar[0] : tuned_variant(kPassXfwd, t->g.Mx, p == 0);
      info->xinv_variant[p] = t->xvar[1] >= 0 ? t->xvar[1] : tuned_variant(kPassXinv, t->g.Mx, p == 0);
    }
    return DDA_OK;
  });
}

void dda_free_target(dda_target *t) { delete t; }

int dda_pass_plan(int32_t pass, int32_t L, int32_t precision, int32_t variant, int32_t radices[8]) {
  return guarded([&]() -> int {
    DDA_REQUIRE(radices != nullptr, "NULL argument");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    DDA_REQUIRE(pass == kPassXfwd || pass == kPassZ || pass == kPassXinv, "pass must be 0, 2 or 4");
    const int nvar = pass == kPassZ ? kPlanVariants : kRowPlanVariants;
    DDA_REQUIRE(variant >= 0 && variant < nvar, "variant out of range for this pass");
    DDA_REQUIRE(L >= 2 && L <= kMaxLen && next_smooth(L) == L, "L must be 2/3/5-smooth and <= 512");
    const int v = L >= kTunedMinLen ? variant : 0;
    StaticPlan p{};
    if (pass == kPassZ) {
      // pencils per z-pass block: a 128-byte tile row, halved for long columns
      const bool f32 = precision == DDA_MIXED;
      const int logw = f32 ? 4 : 3, half = L * (1 << logw) > (f32 ? 2048 : 1024) ? 1 : 0;
      p = plan_variant(L, pen_rmax(L, logw - half), v);
    } else {
      p = rows_plan(L, v);
    }
    for (int i = 0; i < 8; ++i) radices[i] = i < p.n ? p.radix[i] : 0;
    return p.n;
  });
}

int dda_zpass_plan(int32_t L, int32_t precision, int32_t variant, int32_t radices[8]) {
  return dda_pass_plan(kPassZ, L, precision, variant, radices);
}

int dda_set_plan_variant(dda_target *t, int32_t pass, int32_t variant) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t != nullptr, "NULL argument");
    DDA_REQUIRE(pass == kPassXfwd || pass == kPassZ || pass == kPassXinv, "pass must be 0, 2 or 4");
    const int nvar = pass == kPassZ ? kPlanVariantsHost : kRowPlanVariantsHost;
    DDA_REQUIRE(variant >= -1 && variant < nvar, "variant out of range for this pass");
    if (pass == kPassZ) t->zvar = variant;
    else t->xvar[pass == kPassXfwd ? 0 : 1] = variant;
    ++t->buffer_gen;                  // a captured iteration graph holds the old kernels
    return DDA_OK;
  });
}

int dda_set_zpass_variant(dda_target *t, int32_t variant) { return dda_set_plan_variant(t, kPassZ, variant); }

int dda_set_pass_timing(dda_target *t, int32_t every) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t != nullptr, "NULL argument");
    DDA_REQUIRE(every >= 0, "every must be >= 0");
    DDA_HIP(hipSetDevice(t->device));
    if (every > 0 && t->pt_ev.empty()) {
      std::vector<hipEvent_t> ev((size_t)6 * dda_target::kPassTimingSets, nullptr);
      for (auto &e : ev) {
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) {
          for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
          DDA_HIP(err);
        }
      }
      t->pt_ev.swap(ev);
      t->pt_prec.assign(dda_target::kPassTimingSets, 0);
    }
    t->pt_every = every;
    t->pt_used = 0;
    t->pt_seen = 0;
    for (int p = 0; p < 2; ++p) {
      t->pt_n[p] = 0;
      for (int k = 0; k < 5; ++k) t->pt_ms[p][k] = 0.0;
    }
    return DDA_OK;
  });
}

int dda_get_pass_timing(const dda_target *t, int32_t precision, double ms[5], int64_t *products) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && ms && products, "NULL argument");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    const int p = precision == DDA_MIXED ? 1 : 0;
    for (int k = 0; k < 5; ++k) ms[k] = t->pt_ms[p][k];
    *products = t->pt_n[p];
    return DDA_OK;
  });
}

int dda_incident_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, void *e_dev, void *stream) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && e_dev, "NULL argument");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    std::vector<RhsDev> rd;
    std::vector<c64> ai;
    prepare_rhs(t, rhs, nrhs, rd, ai);
    ensure_krylov(t, nrhs, s);
    upload_rhs(t, rd, ai, s);
    launch_incident(t->g, t->d_ijk, t->d_rhs, nrhs, t->kd, static_cast<c64 *>(e_dev), s);
    return DDA_OK;
  });
}

int dda_apply(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision, const void *p_dev, void *ap_dev,
              void *stream) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && p_dev && ap_dev, "NULL argument");
    DDA_REQUIRE(p_dev != ap_dev, "p_dev and ap_dev must not alias");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    std::vector<RhsDev> rd;
    std::vector<c64> ai;
    prepare_rhs(t, rhs, nrhs, rd, ai);
    ensure_krylov(t, nrhs, s);
    ensure_workspace(t, nrhs, s);
    upload_rhs(t, rd, ai, s);
    matvec(t, precision, static_cast<const c64 *>(p_dev), static_cast<c64 *>(ap_dev), nrhs, nullptr, s);
    return DDA_OK;
  });
}

int dda_apply_noalloc(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision, const void *p_dev,
                      void *ap_dev, void *stream) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && rhs && p_dev && ap_dev, "NULL argument");
    DDA_REQUIRE(p_dev != ap_dev, "p_dev and ap_dev must not alias");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    DDA_REQUIRE((int64_t)nrhs * t->ncomp <= kNoAllocMaxRhsComp, "nrhs * n_comp exceeds 32 (allocation-free product)");
    const bool f32 = precision == DDA_MIXED;
    const size_t cs = f32 ? sizeof(c32) : sizeof(c64);
    const size_t a = t->g.a_elems(f32) * cs * nrhs;
    const size_t b = t->g.b_elems(f32) * cs * nrhs;
    const size_t a_pad = (a + 255) / 256 * 256;
    const size_t need = kNoAllocAinvBytes + a_pad + b;
    if (need > (size_t)DDA_NOALLOC_SCRATCH_BYTES)
      throw Error{DDA_ENOTSUP, "allocation-free product needs " + std::to_string(need) + " bytes of scratch, " +
                                   "more than the " + std::to_string((size_t)DDA_NOALLOC_SCRATCH_BYTES) +
                                   " available (fewer RHS, or dda_apply)"};
    AinvArg av{};
    av.n = 3 * nrhs * t->ncomp;
    for (int r = 0; r < nrhs; ++r) {
      RhsDev rd;
      check_rhs(rhs[r], rd);
      for (int c = 0; c < t->ncomp; ++c)
        alpha_inverse(t->alpha_kind, t->m[c], t->kd, rd.khat, rd.e, &av.v[3 * (r * t->ncomp + c)]);
    }
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *base = scratch_address(t->device);
    c64 *d_ainv = reinterpret_cast<c64 *>(base);
    void *bufA = base + kNoAllocAinvBytes;
    void *bufB = base + kNoAllocAinvBytes + a_pad;
    hipLaunchKernelGGL(k_fill_ainv, dim3(1), dim3(128), 0, s, d_ainv, av);
    DDA_HIP(hipGetLastError());
    matvec_on(t, precision, static_cast<const c64 *>(p_dev), static_cast<c64 *>(ap_dev), nrhs, nullptr, d_ainv, bufA,
              bufB, s);
    // the handle's release waits for this stream if it already tracks it
    // (creating a tracking event here would allocate)
    for (auto &u : t->uses)
      if (u.first == s) (void)hipEventRecord(u.second, s);
    return DDA_OK;
  });
}

int dda_profile_matvec(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision, int32_t reps,
                       const void *p_dev, void *ap_dev, void *stream, double ms_per_pass[6]) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && p_dev && ap_dev && ms_per_pass, "NULL argument");
    DDA_REQUIRE(p_dev != ap_dev, "p_dev and ap_dev must not alias");
    DDA_REQUIRE(nrhs >= 1 && reps >= 1, "nrhs and reps must be >= 1");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    std::vector<RhsDev> rd;
    std::vector<c64> ai;
    prepare_rhs(t, rhs, nrhs, rd, ai);
    ensure_krylov(t, nrhs, s);
    ensure_workspace(t, nrhs, s);
    upload_rhs(t, rd, ai, s);
    hipEvent_t ev[6];
    for (auto &e : ev) DDA_HIP(hipEventCreate(&e));
    const c64 *in = static_cast<const c64 *>(p_dev);
    c64 *out = static_cast<c64 *>(ap_dev);
    // whole products, events between the passes
    matvec(t, precision, in, out, nrhs, nullptr, s);        // warm-up
    double whole = 0.0;
    for (int i = 0; i < reps; ++i) {
      matvec(t, precision, in, out, nrhs, nullptr, s, ev);
      DDA_HIP(hipStreamSynchronize(s));
      float ms = 0.f;
      DDA_HIP(hipEventElapsedTime(&ms, ev[0], ev[5]));
      whole += ms;
    }
    ms_per_pass[5] = whole / reps;
    // each pass alone, launched `reps` times back to back on buffers that a
    // full product has just filled
    for (int k = 0; k < 5; ++k) {
      matvec(t, precision, in, out, nrhs, nullptr, s);
      matvec(t, precision, in, out, nrhs, nullptr, s, ev, k, reps);
      DDA_HIP(hipStreamSynchronize(s));
      float ms = 0.f;
      DDA_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
      ms_per_pass[k] = ms / reps;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return DDA_OK;
  });
}

int dda_solve(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const dda_solve_opts *opts, void *p_dev,
              dda_c64 *p_host, void *stream, dda_solve_stats *stats) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && opts, "NULL argument");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_REQUIRE(std::isfinite(opts->tol) && opts->tol > 0.0, "tol must be > 0");
    DDA_REQUIRE(opts->max_iter >= 1, "max_iter must be >= 1");
    DDA_REQUIRE(opts->precision == DDA_FP64 || opts->precision == DDA_MIXED || opts->precision == DDA_MIXED_V32,
                "unknown precision");
    DDA_REQUIRE(opts->precision != DDA_MIXED_V32 || opts->solver == DDA_SOLVER_COCG ||
                    opts->solver == DDA_SOLVER_BICGSTAB,
                "DDA_MIXED_V32 is built for DDA_SOLVER_COCG and DDA_SOLVER_BICGSTAB only");
    // the products run in FP32 for both mixed modes; V32 also keeps the search
    // direction p and its product in FP32
    const int prec = opts->precision == DDA_MIXED_V32 ? DDA_MIXED : opts->precision;
    DDA_REQUIRE(opts->inner_tol >= 0.0 && opts->inner_tol < 1.0, "inner_tol must be in [0, 1)");
    DDA_REQUIRE(opts->solver >= DDA_SOLVER_BICGSTAB && opts->solver <= DDA_SOLVER_QMR, "unknown solver");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    PassTimingScope timing_{t};
    // iterations between host checks: fixed, or (check_every <= 0, eager
    // launches) a first block of 8 (or -check_every) iterations, then blocks
    // predicted from the recursive residual's decay since the last check, so
    // that the next check falls where the slowest RHS should have converged
    // (each check costs a host round trip with the GPU idle)
    t->fold_records = opts->fold_records > 0 ? opts->fold_records : opts->fold_records < 0 ? 0 : kFoldRecords;
    // first block: 8 iterations, or 4 on grids of at most 64^3 points, whose
    // iterations cost less than the host round trip of a check (iterations
    // launched after convergence still cost a launch each)
    const int k0 = (size_t)t->g.Mx * t->g.My * t->g.Mz <= ((size_t)1 << 18) ? 4 : 8;
    int K = opts->check_every > 0 ? opts->check_every : opts->check_every < 0 ? std::min(-opts->check_every, 64) : k0;
    const bool adaptive = opts->check_every <= 0 && opts->use_graph == 0;
    const int max_outer = opts->max_outer > 0 ? opts->max_outer : 20;
    std::vector<RhsDev> rd;
    std::vector<c64> ai, scl;
    prepare_rhs(t, rhs, nrhs, rd, ai);
    const bool jacobi = opts->jacobi != 0;
    if (jacobi) jacobi_scaling(ai, scl);
    ensure_krylov(t, nrhs, s);
    ensure_workspace(t, nrhs, s);
    KrylovState &k = t->k;
    upload_rhs(t, rd, ai, s, jacobi ? &scl : nullptr);
    launch_incident(t->g, t->d_ijk, t->d_rhs, nrhs, t->kd, k.b, s);
    // with Jacobi scaling the iterations solve (S A S) y = S E, and P = S y
    JacobiScope jacobi_{t, jacobi};
    Vec32Scope vec32_{t, opts->precision == DDA_MIXED_V32};
    if (jacobi) launch_scale(t->g, k.b, nrhs, t->d_scl, t->ncomp, t->d_comp, false, s);
    k_init_state(k, opts->tol, opts->max_iter, opts->solver, s);

    if (t->h_nrhs < nrhs) {
      DDA_HIP(hipStreamSynchronize(s));               // no copy into the old blocks is pending
      pinned_release(t->h_status, t->h_status_granted);
      pinned_release(t->h_scal, t->h_scal_granted);
      t->h_status = nullptr;
      t->h_scal = nullptr;
      t->h_nrhs = 0;
      t->h_status = static_cast<int *>(pinned_alloc(3 * nrhs * sizeof(int), &t->h_status_granted));
      t->h_scal = static_cast<c64 *>(pinned_alloc((size_t)nrhs * kScal * sizeof(c64), &t->h_scal_granted));
      t->h_nrhs = nrhs;
    }
    std::vector<int> status(nrhs), check(nrhs), restart(nrhs), outer(nrhs, 0), final_status(nrhs, -1);
    std::vector<c64> scal((size_t)nrhs * kScal);
    std::vector<double> rel(nrhs, 0.0);
    // per RHS: residual^2 and iteration count of the last reference point
    // (the start, |b|^2 at 0 iterations; a restart, its true residual^2)
    std::vector<double> ref_r2(nrhs, -1.0), ref_it(nrhs, 0.0);
    const double steps_per_k = opts->solver == DDA_SOLVER_BICGSTAB2 ? 2.0 : 1.0;
    const double tol = opts->tol;
    const double inner = prec == DDA_MIXED ? opts->inner_tol : 0.0;
    // P = 0 start: an RHS with E = 0 is already solved (its status says so
    // after the first block; the first block is queued without a read).
    // With an initial guess every RHS starts stopped: the check below takes
    // the true residual of x0 and restarts the recurrence from it, or keeps
    // x0 when it is already within tol.
    const bool warm = opts->x0 != nullptr;
    if (warm) {
      DDA_HIP(hipMemcpyAsync(k.x, opts->x0, (size_t)k.n3 * nrhs * sizeof(c64), hipMemcpyDeviceToDevice, s));
      if (jacobi) launch_scale(t->g, k.x, nrhs, t->d_scl, t->ncomp, t->d_comp, true, s);
      DDA_HIP(hipMemsetAsync(k.active, 0, nrhs * sizeof(int), s));
    }
    bool first = true;
    while (true) {
      if (first) {
        std::fill(status.begin(), status.end(), warm ? (int)ST_CONV : (int)ST_RUN);
      } else {
        DDA_HIP(hipMemcpyAsync(t->h_status, k.status, nrhs * sizeof(int), hipMemcpyDeviceToHost, s));
        if (adaptive)
          DDA_HIP(hipMemcpyAsync(t->h_scal, k.scal, scal.size() * sizeof(c64), hipMemcpyDeviceToHost, s));
        DDA_HIP(hipStreamSynchronize(s));
        t->pt_harvest();
        std::copy(t->h_status, t->h_status + nrhs, status.begin());
        if (adaptive) std::copy(t->h_scal, t->h_scal + scal.size(), scal.begin());
      }
      if (adaptive && !first) {
        int kmax = 0;
        for (int r = 0; r < nrhs; ++r) {
          if (final_status[r] >= 0 || status[r] != ST_RUN) continue;
          const c64 *sc = &scal[(size_t)r * kScal];
          const double r2 = sc[S_RNORM2].x, thr = sc[S_THR2].x, it = sc[S_ITERS].x;
          if (ref_r2[r] < 0.0) ref_r2[r] = sc[S_BNORM2].x;
          int kr = 8;
          if (it > ref_it[r] && ref_r2[r] > 0.0 && r2 < ref_r2[r] && r2 > thr && thr > 0.0) {
            const double need = (it - ref_it[r]) * std::log(thr / r2) / std::log(r2 / ref_r2[r]) / steps_per_k;
            kr = need < 63.0 ? (int)std::ceil(need) + 1 : 64;
          }
          kmax = std::max(kmax, kr);
          ref_r2[r] = r2;
          ref_it[r] = it;
        }
        K = std::min(64, std::max(4, kmax > 0 ? kmax : 8));
      }
      first = false;
      bool any_run = false, any_check = false;
      for (int r = 0; r < nrhs; ++r) {
        check[r] = 0;
        if (final_status[r] >= 0) continue;
        if (status[r] == ST_RUN) any_run = true;
        else {
          check[r] = 1;
          any_check = true;
        }
      }
      if (any_check) {
        // FP64 true residual r = E - A x for the stopped RHS
        int *h_check = t->h_status + nrhs;           // pinned; not rewritten before the sync below
        std::copy(check.begin(), check.end(), h_check);
        DDA_HIP(hipMemcpyAsync(k.check, h_check, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        matvec(t, DDA_FP64, k.x, k.t, nrhs, k.check, s);
        k_true_residual(k, k.t, s);
        DDA_HIP(hipMemcpyAsync(t->h_scal, k.scal, scal.size() * sizeof(c64), hipMemcpyDeviceToHost, s));
        DDA_HIP(hipStreamSynchronize(s));
        t->pt_harvest();
        std::copy(t->h_scal, t->h_scal + scal.size(), scal.begin());
        bool any_restart = false;
        for (int r = 0; r < nrhs; ++r) {
          restart[r] = 0;
          if (!check[r]) continue;
          const double b2 = scal[(size_t)r * kScal + S_BNORM2].x;
          const double t2 = scal[(size_t)r * kScal + S_TRUE2].x;
          rel[r] = b2 > 0.0 ? std::sqrt(t2 / b2) : 0.0;
          ++outer[r];
          if (b2 == 0.0 || rel[r] <= tol) final_status[r] = 0;
          else if (status[r] == ST_MAXIT) final_status[r] = 1;
          else if (outer[r] >= max_outer || !(rel[r] == rel[r])) final_status[r] = status[r] == ST_BREAK ? 2 : 1;
          else {
            restart[r] = 1;
            any_restart = true;
          }
        }
        if (any_restart) {
          int *h_restart = t->h_status + 2 * nrhs;   // pinned; read by the copy before the next sync
          std::copy(restart.begin(), restart.end(), h_restart);
          DDA_HIP(hipMemcpyAsync(t->d_restart, h_restart, nrhs * sizeof(int), hipMemcpyHostToDevice, s));
          k_restart(k, t->d_restart, tol, inner, opts->solver, s);
          any_run = true;
          if (adaptive) {
            // a restarted RHS starts a new residual history
            for (int r = 0; r < nrhs; ++r)
              if (restart[r]) {
                ref_r2[r] = scal[(size_t)r * kScal + S_TRUE2].x;
                ref_it[r] = scal[(size_t)r * kScal + S_ITERS].x;
              }
            K = std::max(K, 8);
          }
        }
      }
      if (!any_run) break;
      run_iterations(t, prec, opts->solver, K, opts->use_graph != 0, s);
    }
    DDA_HIP(hipMemcpyAsync(t->h_scal, k.scal, scal.size() * sizeof(c64), hipMemcpyDeviceToHost, s));
    const size_t vec = (size_t)k.n3 * nrhs * sizeof(c64);
    if (jacobi) launch_scale(t->g, k.x, nrhs, t->d_scl, t->ncomp, t->d_comp, false, s);
    if (p_dev) DDA_HIP(hipMemcpyAsync(p_dev, k.x, vec, hipMemcpyDeviceToDevice, s));
    if (p_host) DDA_HIP(hipMemcpyAsync(p_host, k.x, vec, hipMemcpyDeviceToHost, s));
    DDA_HIP(hipStreamSynchronize(s));
    t->pt_harvest();
    std::copy(t->h_scal, t->h_scal + scal.size(), scal.begin());
    bool all_ok = true;
    for (int r = 0; r < nrhs; ++r) {
      if (final_status[r] != 0) all_ok = false;
      if (stats) {
        stats[r].status = final_status[r];
        stats[r].iters = (int)scal[(size_t)r * kScal + S_ITERS].x;
        stats[r].matvecs = (opts->solver == DDA_SOLVER_COCG || opts->solver == DDA_SOLVER_QMR ? 1 : 2) *
                           stats[r].iters;
        stats[r].outer = outer[r];
        stats[r].rel_resid = rel[r];
      }
    }
    return all_ok ? DDA_OK : DDA_NOT_CONVERGED;
  });
}

int dda_scattering_matrix(dda_target *t, const dda_rhs rhs[2], const void *p_dev, const double lab[9],
                          int32_t ndir, const double *theta_phi, void *stream, dda_scat *out) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && rhs && p_dev && lab && theta_phi && out, "NULL argument");
    DDA_REQUIRE(ndir >= 1, "ndir must be >= 1");
    std::vector<RhsDev> rd;
    std::vector<c64> ai;
    prepare_rhs(t, rhs, 2, rd, ai);
    const double *X = lab, *Y = lab + 3, *Z = lab + 6;
    auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    DDA_REQUIRE(std::fabs(dot(X, X) - 1) < 1e-9 && std::fabs(dot(Y, Y) - 1) < 1e-9 && std::fabs(dot(Z, Z) - 1) < 1e-9 &&
                    std::fabs(dot(X, Y)) < 1e-9 && std::fabs(dot(X, Z)) < 1e-9 && std::fabs(dot(Y, Z)) < 1e-9,
                "lab frame must be orthonormal");
    for (int r = 0; r < 2; ++r)
      DDA_REQUIRE(std::fabs(dot(X, rd[r].khat) - 1.0) < 1e-9, "x_LF must be khat of both rhs");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    // directions and the scattered basis (theta_hat, phi_hat) in the target frame
    std::vector<double> dirs((size_t)ndir * 3), eth((size_t)ndir * 3), eph((size_t)ndir * 3);
    for (int d = 0; d < ndir; ++d) {
      const double th = theta_phi[2 * d], ph = theta_phi[2 * d + 1];
      DDA_REQUIRE(std::isfinite(th) && std::isfinite(ph), "directions must be finite");
      const double ct = std::cos(th), st = std::sin(th), cp = std::cos(ph), sp = std::sin(ph);
      for (int a = 0; a < 3; ++a) {
        dirs[3 * d + a] = ct * X[a] + st * (cp * Y[a] + sp * Z[a]);
        eth[3 * d + a] = -st * X[a] + ct * (cp * Y[a] + sp * Z[a]);
        eph[3 * d + a] = -sp * Y[a] + cp * Z[a];
      }
    }
    const size_t scratch = far_field_scratch_bytes(t->g, ndir);
    const size_t bytes = (size_t)ndir * 3 * sizeof(double) + scratch + (size_t)2 * ndir * 6 * sizeof(double);
    double *buf = t->alloc<double>(bytes);
    double *d_dirs = buf, *d_scr = buf + (size_t)ndir * 3, *d_F = d_scr + scratch / sizeof(double);
    std::vector<double> F((size_t)2 * ndir * 6);
    try {
      DDA_HIP(hipMemcpyAsync(d_dirs, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, s));
      for (int l = 0; l < 2; ++l) {
        const c64 *P = static_cast<const c64 *>(p_dev) + (size_t)l * 3 * t->g.n_sites;
        launch_far_amplitudes(t->g, t->d_cell_site, P, t->kd, d_dirs, ndir, d_scr, d_F + (size_t)l * ndir * 6, s);
      }
      DDA_HIP(hipMemcpyAsync(F.data(), d_F, F.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      DDA_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      t->release(buf);
      throw;
    }
    t->release(buf);
    // f_ml, S_1..S_4 and the Mueller matrix (host arithmetic, §26)
    using cd = std::complex<double>;
    cd ab[2][2];                                 // [l][0] = e0l* . y_LF, [l][1] = e0l* . z_LF
    for (int l = 0; l < 2; ++l) {
      cd py = 0.0, pz = 0.0;
      for (int a = 0; a < 3; ++a) {
        const cd ec = std::conj(cd(rd[l].e[a].x, rd[l].e[a].y));
        py += ec * Y[a];
        pz += ec * Z[a];
      }
      ab[l][0] = py;
      ab[l][1] = pz;
    }
    const cd a = ab[0][0], b = ab[0][1], c = ab[1][0], d4 = ab[1][1], I(0.0, 1.0);
    const double k3 = t->kd * t->kd * t->kd;
    for (int d = 0; d < ndir; ++d) {
      cd f[2][2];
      for (int l = 0; l < 2; ++l) {
        const double *q = &F[((size_t)l * ndir + d) * 6];
        cd ft = 0.0, fp = 0.0;
        for (int a3 = 0; a3 < 3; ++a3) {
          const cd Fa(q[2 * a3], q[2 * a3 + 1]);
          ft += eth[3 * d + a3] * Fa;
          fp += eph[3 * d + a3] * Fa;
        }
        f[0][l] = k3 * ft;
        f[1][l] = k3 * fp;
      }
      const double cp = std::cos(theta_phi[2 * d + 1]), sp = std::sin(theta_phi[2 * d + 1]);
      const cd S1 = -I * (f[1][0] * (b * cp - a * sp) + f[1][1] * (d4 * cp - c * sp));
      const cd S2 = -I * (f[0][0] * (a * cp + b * sp) + f[0][1] * (c * cp + d4 * sp));
      const cd S3 = I * (f[0][0] * (b * cp - a * sp) + f[0][1] * (d4 * cp - c * sp));
      const cd S4 = I * (f[1][0] * (a * cp + b * sp) + f[1][1] * (c * cp + d4 * sp));
      dda_scat &o = out[d];
      for (int m = 0; m < 2; ++m)
        for (int l = 0; l < 2; ++l) o.f[m][l] = dda_c64{f[m][l].real(), f[m][l].imag()};
      const cd Sv[4] = {S1, S2, S3, S4};
      for (int j = 0; j < 4; ++j) o.s[j] = dda_c64{Sv[j].real(), Sv[j].imag()};
      const double a1 = std::norm(S1), a2 = std::norm(S2), a3 = std::norm(S3), a4 = std::norm(S4);
      double(*M)[4] = o.mueller;
      M[0][0] = (a1 + a2 + a3 + a4) / 2;
      M[0][1] = (a2 - a1 + a4 - a3) / 2;
      M[0][2] = std::real(S2 * std::conj(S3) + S1 * std::conj(S4));
      M[0][3] = std::imag(S2 * std::conj(S3) - S1 * std::conj(S4));
      M[1][0] = (a2 - a1 + a3 - a4) / 2;
      M[1][1] = (a1 + a2 - a3 - a4) / 2;
      M[1][2] = std::real(S2 * std::conj(S3) - S1 * std::conj(S4));
      M[1][3] = std::imag(S2 * std::conj(S3) + S1 * std::conj(S4));
      M[2][0] = std::real(S2 * std::conj(S4) + S1 * std::conj(S3));
      M[2][1] = std::real(S2 * std::conj(S4) - S1 * std::conj(S3));
      M[2][2] = std::real(S1 * std::conj(S2) + S3 * std::conj(S4));
      M[2][3] = std::imag(S2 * std::conj(S1) + S4 * std::conj(S3));
      M[3][0] = std::imag(S4 * std::conj(S2) + S1 * std::conj(S3));
      M[3][1] = std::imag(S4 * std::conj(S2) - S1 * std::conj(S3));
      M[3][2] = std::imag(S1 * std::conj(S2) - S3 * std::conj(S4));
      M[3][3] = std::real(S1 * std::conj(S2) - S3 * std::conj(S4));
    }
    return DDA_OK;
  });
}

int dda_near_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev, const int32_t margin[3],
                   int32_t macroscopic, void *e_dev, void *stream) {
  if (!e_dev) return guarded([&]() -> int { throw Error{DDA_EINVAL, "NULL argument"}; });
  return dda_near_field_eb(t, rhs, nrhs, p_dev, margin, macroscopic, e_dev, nullptr, stream);
}

int dda_near_field_eb(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev, const int32_t margin[3],
                      int32_t macroscopic, void *e_dev, void *b_dev, void *stream) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && rhs && p_dev && margin && (e_dev || b_dev), "NULL argument");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_REQUIRE(margin[0] >= 0 && margin[1] >= 0 && margin[2] >= 0, "margins must be >= 0");
    const int mg[3] = {margin[0], margin[1], margin[2]};
    const int64_t Xl = t->g.nx + 2 * (int64_t)mg[0], Yl = t->g.ny + 2 * (int64_t)mg[1], Zl = t->g.nz + 2 * (int64_t)mg[2];
    if (Xl > 256 || Yl > 256 || Zl > 256)
      throw Error{DDA_ENOTSUP, "extended box extent exceeds 256 (padded FFT extent 512)"};
    const int X = (int)Xl, Y = (int)Yl, Z = (int)Zl;
    const int64_t ne = Xl * Yl * Zl, n = t->g.n_sites;
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    // a target occupying the whole extended box, numbered row after row
    std::vector<int32_t> ijk((size_t)ne * 3);
    for (int z = 0, j = 0; z < Z; ++z)
      for (int y = 0; y < Y; ++y)
        for (int x = 0; x < X; ++x, ++j) {
          ijk[3 * (size_t)j] = x;
          ijk[3 * (size_t)j + 1] = y;
          ijk[3 * (size_t)j + 2] = z;
        }
    const dda_c64 any_m = {1.5, 0.0};           // unused: the diagonal is set to zero below
    dda_target_desc d{};
    d.nx = X;
    d.ny = Y;
    d.nz = Z;
    d.n_sites = ne;
    d.ijk = ijk.data();
    d.comp = nullptr;
    d.n_comp = 1;
    d.m = &any_m;
    d.kd = t->kd;
    d.alpha_kind = DDA_ALPHA_LDR;
    d.device = t->device;
    dda_target *ext = nullptr;
    const int rc = dda_setup_target(&d, &ext);
    if (rc < 0) throw Error{rc, std::string("near field: ") + dda_last_error()};
    std::unique_ptr<dda_target, void (*)(dda_target *)> hold(ext, dda_free_target);
    {
      StreamUse use_ext{ext, s};
      std::vector<RhsDev> rd;
      std::vector<c64> ai;
      prepare_rhs(ext, rhs, nrhs, rd, ai);
      std::fill(ai.begin(), ai.end(), c64{0.0, 0.0});     // zero diagonal: A P_ext = -G * P_ext
      ensure_krylov(ext, nrhs, s);
      ensure_workspace(ext, nrhs, s);
      upload_rhs(ext, rd, ai, s);
      // site i -> extended point; composition at each extended point (-1: vacuum)
      std::vector<int32_t> sites((size_t)n * 3);
      DDA_HIP(hipMemcpy(sites.data(), t->d_ijk, sites.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
      std::vector<uint8_t> comp;
      if (t->d_comp) {
        comp.resize((size_t)n);
        DDA_HIP(hipMemcpy(comp.data(), t->d_comp, comp.size(), hipMemcpyDeviceToHost));
      }
      std::vector<int> map((size_t)n), cellc((size_t)ne, -1);
      for (int64_t i = 0; i < n; ++i) {
        const int64_t j = ((int64_t)(sites[3 * i + 2] + mg[2]) * Y + (sites[3 * i + 1] + mg[1])) * X +
                          (sites[3 * i] + mg[0]);
        map[i] = (int)j;
        cellc[j] = comp.empty() ? 0 : comp[i];
      }
      std::vector<c64> fac((size_t)t->ncomp);
      for (int c = 0; c < t->ncomp; ++c) {
        const c64 m = t->m[c];
        const c64 eps2 = {m.x * m.x - m.y * m.y + 2.0, 2.0 * m.x * m.y};
        const double den = eps2.x * eps2.x + eps2.y * eps2.y;
        fac[c] = {3.0 * eps2.x / den, -3.0 * eps2.y / den};
      }
      int *d_map = ext->alloc<int>(map.size() * sizeof(int));
      int *d_cellc = ext->alloc<int>(cellc.size() * sizeof(int));
      c64 *d_fac = ext->alloc<c64>(fac.size() * sizeof(c64));
      DDA_HIP(hipMemcpy(d_map, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice));
      DDA_HIP(hipMemcpy(d_cellc, cellc.data(), cellc.size() * sizeof(int), hipMemcpyHostToDevice));
      DDA_HIP(hipMemcpy(d_fac, fac.data(), fac.size() * sizeof(c64), hipMemcpyHostToDevice));
      KrylovState &k = ext->k;
      if (e_dev) {
        DDA_HIP(hipMemsetAsync(k.x, 0, (size_t)nrhs * ne * 3 * sizeof(c64), s));
        launch_near_field_embed(static_cast<const c64 *>(p_dev), n, d_map, k.x, ne, nrhs, s);
        matvec(ext, DDA_FP64, k.x, k.v, nrhs, nullptr, s);
        launch_near_field_combine(k.v, ne, X, Y, mg, ext->d_rhs, nrhs, t->kd, d_cellc,
                                  macroscopic ? d_fac : nullptr, static_cast<c64 *>(e_dev), s);
      }
      if (b_dev) {
        // B = B_inc + h (*) P on the full padded grid of the extended box, one
        // RHS at a time: h transformed once, P embedded and transformed, the
        // cross product, the inverse transform (scaled by 1/M)
        const Geometry &ge = ext->g;
        const int64_t M = (int64_t)ge.Mx * ge.My * ge.Mz;
        std::vector<int64_t> mapM((size_t)n);
        for (int64_t i = 0; i < n; ++i)
          mapM[i] = ((int64_t)(sites[3 * i + 2] + mg[2]) * ge.My + (sites[3 * i + 1] + mg[1])) * ge.Mx +
                    (sites[3 * i] + mg[0]);
        int64_t *d_mapM = ext->alloc<int64_t>(mapM.size() * sizeof(int64_t));
        DDA_HIP(hipMemcpy(d_mapM, mapM.data(), mapM.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        c64 *h = ext->alloc<c64>((size_t)3 * M * sizeof(c64));
        c64 *full = ext->alloc<c64>((size_t)3 * M * sizeof(c64));
        launch_magnetic_kernel(ge, t->kd, h, ext->tx, ext->ty, ext->tz, ext->px, ext->py, ext->pz, s);
        for (int r = 0; r < nrhs; ++r) {
          DDA_HIP(hipMemsetAsync(full, 0, (size_t)3 * M * sizeof(c64), s));
          launch_magnetic_embed(static_cast<const c64 *>(p_dev) + (size_t)r * n * 3, n, d_mapM, full, M, s);
          launch_fft3_full64(full, 3, ge, ext->tx, ext->ty, ext->tz, ext->px, ext->py, ext->pz, -1, s);
          launch_magnetic_cross(h, full, M, 1.0 / double(M), s);
          launch_fft3_full64(full, 3, ge, ext->tx, ext->ty, ext->tz, ext->px, ext->py, ext->pz, 1, s);
          launch_magnetic_field(full, ge, X, Y, ne, mg, ext->d_rhs + r, t->kd,
                                static_cast<c64 *>(b_dev) + (size_t)r * ne * 3, s);
        }
      }
    }
    return DDA_OK;
  });
}

int dda_far_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev, double etasca, void *stream,
                  dda_far *out) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && rhs && p_dev && out, "NULL argument");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_REQUIRE(std::isfinite(etasca) && etasca > 0.0, "etasca must be > 0");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    const double x = t->kd * t->aeff;
    const double ntd = std::ceil((3.0 + x) / etasca) + 1.0;
    DDA_REQUIRE(ntd <= 2048.0, "etasca too small: more than 2048 polar angles");
    const int nt = (int)ntd, nf = 2 * nt, ndir = nt * nf;
    std::vector<double> gx, gw;
    gauss_legendre(nt, gx, gw);
    std::vector<double> mu((size_t)ndir), w((size_t)ndir), dirs((size_t)ndir * 3);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nf; ++j) {
        mu[(size_t)i * nf + j] = gx[i];
        w[(size_t)i * nf + j] = gw[i] * 2.0 * pi / nf;
      }
    // scratch for the quadrature and for the single backscattering direction
    const size_t scratch = std::max(far_field_scratch_bytes(t->g, ndir), far_field_scratch_bytes(t->g, 1));
    const size_t bytes = (size_t)ndir * 5 * sizeof(double) + scratch + 8 * sizeof(double);
    double *buf = t->alloc<double>(bytes);
    double *d_dirs = buf, *d_mu = buf + (size_t)ndir * 3, *d_w = d_mu + ndir, *d_scr = d_w + ndir;
    double *d_sums = d_scr + scratch / sizeof(double), *d_bk = d_sums + 3;
    std::vector<double> sums(3);
    try {
      DDA_HIP(hipMemcpyAsync(d_mu, mu.data(), (size_t)ndir * sizeof(double), hipMemcpyHostToDevice, s));
      DDA_HIP(hipMemcpyAsync(d_w, w.data(), (size_t)ndir * sizeof(double), hipMemcpyHostToDevice, s));
      for (int r = 0; r < nrhs; ++r) {
        const double *kh = rhs[r].khat;
        const double kn = std::sqrt(kh[0] * kh[0] + kh[1] * kh[1] + kh[2] * kh[2]);
        DDA_REQUIRE(std::fabs(kn - 1.0) <= 1e-12, "|khat| must be 1");
        // frame (e1, e2, khat): e1 from x (or y when khat is near x)
        const double k[3] = {kh[0] / kn, kh[1] / kn, kh[2] / kn};
        double tt[3] = {1.0, 0.0, 0.0};
        if (std::fabs(k[0]) >= 0.9) tt[0] = 0.0, tt[1] = 1.0;
        const double tk = tt[0] * k[0] + tt[1] * k[1] + tt[2] * k[2];
        double e1[3] = {tt[0] - tk * k[0], tt[1] - tk * k[1], tt[2] - tk * k[2]};
        const double e1n = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (double &v : e1) v /= e1n;
        const double e2[3] = {k[1] * e1[2] - k[2] * e1[1], k[2] * e1[0] - k[0] * e1[2], k[0] * e1[1] - k[1] * e1[0]};
        for (int i = 0; i < nt; ++i) {
          const double st = std::sqrt(std::max(0.0, 1.0 - gx[i] * gx[i]));
          for (int j = 0; j < nf; ++j) {
            const double ph = 2.0 * pi * j / nf, cp = std::cos(ph), sp = std::sin(ph);
            double *n = &dirs[((size_t)i * nf + j) * 3];
            for (int a = 0; a < 3; ++a) n[a] = gx[i] * k[a] + st * (cp * e1[a] + sp * e2[a]);
          }
        }
        DDA_HIP(hipMemcpyAsync(d_dirs, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, s));
        const c64 *P = static_cast<const c64 *>(p_dev) + (size_t)r * 3 * t->g.n_sites;
        launch_far_field(t->g, t->d_cell_site, P, t->kd, d_dirs, d_mu, d_w, ndir, d_scr, d_sums, s);
        DDA_HIP(hipMemcpyAsync(sums.data(), d_sums, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        DDA_HIP(hipStreamSynchronize(s));
        const double k4 = t->kd * t->kd * t->kd * t->kd;
        out[r].qsca = k4 * sums[0] / (pi * t->aeff * t->aeff);
        out[r].g = sums[0] > 0.0 ? sums[1] / sums[0] : 0.0;
        out[r].cos2 = sums[0] > 0.0 ? sums[2] / sums[0] : 0.0;
        out[r].n_theta = nt;
        out[r].n_phi = nf;
        // backscattering: the same phase sum in the one direction -khat (weight 1)
        const double bk[5] = {-k[0], -k[1], -k[2], -1.0, 1.0};
        double bsum = 0.0;
        DDA_HIP(hipMemcpyAsync(d_bk, bk, sizeof(bk), hipMemcpyHostToDevice, s));
        launch_far_field(t->g, t->d_cell_site, P, t->kd, d_bk, d_bk + 3, d_bk + 4, 1, d_scr, d_sums, s);
        DDA_HIP(hipMemcpyAsync(&bsum, d_sums, sizeof(double), hipMemcpyDeviceToHost, s));
        DDA_HIP(hipStreamSynchronize(s));
        out[r].qbk = k4 * bsum / (pi * t->aeff * t->aeff);
      }
    } catch (...) {
      (void)hipStreamSynchronize(s);
      t->release(buf);
      throw;
    }
    t->release(buf);
    return DDA_OK;
  });
}

int dda_cross_sections(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev, const dda_c64 *p_host,
                       void *stream, dda_q *out) {
  return guarded([&]() -> int {
    DDA_REQUIRE(t && out, "NULL argument");
    DDA_REQUIRE(p_dev || p_host, "need p_dev or p_host");
    DDA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    DDA_HIP(hipSetDevice(t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamUse use_{t, s};
    std::vector<RhsDev> rd;
    std::vector<c64> ai;
    prepare_rhs(t, rhs, nrhs, rd, ai);
    ensure_krylov(t, nrhs, s);
    upload_rhs(t, rd, ai, s);
    const c64 *P = static_cast<const c64 *>(p_dev);
    if (!P) {
      DDA_HIP(hipMemcpyAsync(t->k.t, p_host, (size_t)t->k.n3 * nrhs * sizeof(c64), hipMemcpyHostToDevice, s));
      P = t->k.t;
    }
    launch_cross_sums(t->g, t->d_ijk, t->d_rhs, nrhs, t->kd, P, t->d_ainv, t->ncomp, t->d_comp, t->k.partial,
                      t->d_sums, s);
    std::vector<double> sums(3 * nrhs);
    DDA_HIP(hipMemcpyAsync(sums.data(), t->d_sums, sums.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DDA_HIP(hipStreamSynchronize(s));
    const double pi = 3.14159265358979323846;
    const double geo = pi * t->aeff * t->aeff;
    for (int r = 0; r < nrhs; ++r) {
      const double cext = 4.0 * pi * t->kd * sums[3 * r];
      const double cabs = 4.0 * pi * t->kd * sums[3 * r + 1];
      const double cpha = 2.0 * pi * t->kd * sums[3 * r + 2];
      out[r].qext = cext / geo;
      out[r].qabs = cabs / geo;
      out[r].qsca = (cext - cabs) / geo;
      out[r].aeff = t->aeff;
      out[r].qpha = cpha / geo;
    }
    return DDA_OK;
  });
}

int dda_fft_pencils(int32_t n, int64_t batch, int32_t sign, int32_t precision, double scale, const void *in_dev,
                    void *out_dev, void *stream, int32_t device) {
  return guarded([&]() -> int {
    DDA_REQUIRE(sign == -1 || sign == 1, "sign must be -1 or +1");
    DDA_REQUIRE(batch >= 0, "batch must be >= 0");
    if (batch == 0) return DDA_OK;
    DDA_REQUIRE(in_dev && out_dev, "NULL argument");
    DDA_REQUIRE(precision == DDA_FP64 || precision == DDA_MIXED, "unknown precision");
    DDA_REQUIRE(n >= 1 && n <= kMaxLen && next_smooth(n) == n, "n must be 2/3/5-smooth and <= 512");
    DDA_HIP(hipSetDevice(device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const AxisPlan p = make_axis_plan(n);
    dda_target tmp;         // owns the temporary twiddle tables
    tmp.device = device;
    StreamUse use_{&tmp, s};  // destroyed first: tmp then waits for the transform before releasing
    make_twiddles(&tmp, tmp.tx, n);
    if (precision == DDA_FP64)
      launch_fft_rows<double>(static_cast<const c64 *>(in_dev), static_cast<c64 *>(out_dev), batch, p, tmp.tx.d64,
                              sign, scale, s);
    else
      launch_fft_rows<float>(static_cast<const c32 *>(in_dev), static_cast<c32 *>(out_dev), batch, p, tmp.tx.d32,
                             sign, float(scale), s);
    DDA_HIP(hipStreamSynchronize(s));
    return DDA_OK;
  });
}

}  // extern "C"
