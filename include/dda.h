/*
 * dda.h -- C ABI of the MI355X discrete-dipole-approximation (DDA) solver.
 *
 * The library solves A P = E for the polarizations P of N point dipoles on a
 * cubic lattice (DDSCAT 7.3 user guide, Draine & Flatau 2013, §12 "Choice of
 * Iterative Algorithm", eq. AP=E), with
 *
 *     (A P)_j = P_j / alpha_j - sum_{l != j} G(r_j - r_l) P_l ,
 *
 * G the free-space dipole field tensor (cited in §1 and §12 from Draine 1988
 * and Draine & Flatau 1994) and alpha_j the dipole polarizability (§14).  The
 * sum is a discrete convolution evaluated with zero-padded 3-D FFTs of the six
 * independent tensor components (Goodman, Draine & Flatau 1990; §13 "Choice
 * of FFT Algorithm" for the 2/3/5-smooth grid extents).  The solver is
 * BiCGSTAB (van der Vorst 1992; the PBCGST option of §12), started from P = 0,
 * stopped on the true relative residual |E - A P| / |E| <= tol.  Cross sections
 * follow the efficiencies Q = C / (pi a_eff^2) of §3.1.
 *
 * Units: lattice spacing d = 1; Gaussian units; time dependence exp(-i w t)
 * (an absorbing material has Im m > 0).
 *
 * Conventions for every entry point:
 *   - Return value: DDA_OK (0) on success, a negative DDA_E* code on error, a
 *     positive DDA_W* code for a completed call with a warning.  No C++
 *     exception crosses this interface.  dda_last_error() returns a message
 *     for the last failing call on the calling thread.
 *   - Host pointers ("host") are read during the call only; the caller owns
 *     them.  Device pointers ("device") are HIP device addresses on the
 *     target's device; the caller owns them and they must stay valid until
 *     the work queued on the given stream has finished.
 *   - A stream argument is a hipStream_t passed as void*; NULL is the
 *     device's default (null) stream.  Calls on one handle must not overlap
 *     in time (one thread, one stream per handle); distinct handles may run
 *     concurrently on distinct streams.
 *   - Complex numbers are dda_c64 {re, im} (16 bytes, FP64).
 *   - Polarization / field vectors are laid out [nrhs][n_sites][3] dda_c64,
 *     site order as given to dda_setup_target, component order (x, y, z) of
 *     the Target Frame.
 */
#ifndef DDA_H
#define DDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define DDA_OK 0
#define DDA_EINVAL (-1)       /* invalid argument (message via dda_last_error) */
#define DDA_ENOMEM (-2)       /* device allocation failed or footprint too large */
#define DDA_EDEVICE (-3)      /* HIP runtime error */
#define DDA_ENOTSUP (-4)      /* valid but unsupported (e.g. grid extent > 512) */
#define DDA_NOT_CONVERGED 1   /* dda_solve: some RHS stopped at max_iter or broke down */
#define DDA_WVALIDITY 2       /* dda_setup_target: |m|kd >= 1 or |m-1| > 2 (§2) */

/* ---- enumerations ------------------------------------------------------ */
/* Polarizability prescription (§14). */
#define DDA_ALPHA_LDR 0       /* LATTDR: lattice dispersion relation (Draine & Goodman 1993) */
#define DDA_ALPHA_CMRR 1      /* Clausius-Mossotti with radiative reaction */
#define DDA_ALPHA_FCD 2       /* FLTRCD polarizability (requires kd < pi) */
#define DDA_ALPHA_GKDLDR 3    /* GKDLDR: lattice dispersion relation of Gutkowicz-Krusin & Draine 2004 */

/* Arithmetic of the FFT product inside the Krylov iteration. */
#define DDA_FP64 0            /* complex FP64 throughout */
#define DDA_MIXED 1           /* complex FP32 FFT product; FP64 Krylov vectors,
                                 inner products, residual refinement and sums */
#define DDA_MIXED_V32 2       /* dda_solve with DDA_SOLVER_COCG or DDA_SOLVER_BICGSTAB: the
                                 FP32 product of DDA_MIXED, and the search direction p and
                                 its product (COCG's q = A p, BiCGSTAB's v = A p) stored in
                                 complex FP32 (arithmetic on them in FP64); the residuals
                                 (r, and BiCGSTAB's shadow rh, s and t = A s), the iterate x,
                                 every inner product, the FP64 true residual and the
                                 refinement as in DDA_MIXED (§6: single precision where it
                                 suffices, double where accuracy is decided; an FP32 r loses
                                 COCG's bilinear r^T r to cancellation on metallic targets) */

/* Krylov solvers (§12, "Choice of Iterative Algorithm") */
#define DDA_SOLVER_BICGSTAB 0   /* BiCGSTAB, van der Vorst 1992 (the guide's PBCGST) */
#define DDA_SOLVER_BICGSTAB2 1  /* BiCGstab(2), Sleijpen & Fokkema 1993 (the guide's PBCGS2) */
#define DDA_SOLVER_COCG 2       /* conjugate orthogonal CG, van der Vorst & Melissen 1990: CG with
                                   the bilinear form x^T y, valid because A is complex symmetric;
                                   one product per iteration (not among the guide's options) */
#define DDA_SOLVER_QMR 3        /* QMR for complex symmetric A, Freund 1992 (the guide's QMRCCG),
                                   computed as the quasi-minimal-residual smoothing of COCG
                                   (the same iterates); one product per iteration */

/* Built-in target shapes (§21, SHPAR conventions of the guide). */
#define DDA_SHAPE_ELLIPSOID 1 /* shpar = diameters along x, y, z (a sphere: all equal) */
#define DDA_SHAPE_RCTGLPRSM 2 /* shpar = x, y, z extents in dipoles */
#define DDA_SHAPE_CYLINDER1 3 /* shpar = length, diameter, axis (1 = x, 2 = y, 3 = z) */
#define DDA_SHAPE_HEX_PRISM 4 /* shpar = length, vertex-to-vertex width, orientation 1..6 */

/* ---- types --------------------------------------------------------------- */
typedef struct { double re, im; } dda_c64;

typedef struct {
  int32_t nx, ny, nz;      /* bounding box in lattice units; every site inside */
  int64_t n_sites;         /* N >= 1 */
  const int32_t *ijk;      /* host [N][3] site indices, 0 <= i < nx etc., unique */
  const uint8_t *comp;     /* host [N] composition index, or NULL (all 0) */
  int32_t n_comp;          /* number of compositions, 1..255 */
  const dda_c64 *m;        /* host [n_comp] refractive index relative to the medium (§3.2) */
  double kd;               /* k d > 0 (wavenumber in the medium times lattice spacing) */
  int32_t alpha_kind;      /* DDA_ALPHA_* (below) */
  int32_t device;          /* HIP device ordinal */
} dda_target_desc;

/* Polarizabilities (§14; d = 1, m the composition's index, kd, and the RHS's
 * khat, e; alpha_CM = (3/4pi)(m^2-1)/(m^2+2) as printed in §14):
 *   DDA_ALPHA_LDR     1/alpha = 1/alpha_CM + (b1 + b2 m^2 + b3 m^2 S) kd^2 - (2/3) i kd^3,
 *                     S = sum_l khat_l^2 |e_l|^2, b1 = -1.891531, b2 = 0.1648469,
 *                     b3 = -1.7700004 (cited LATTDR; the b's are the second-order
 *                     coefficients of the dipole lattice's dispersion relation);
 *   DDA_ALPHA_GKDLDR  a diagonal tensor, 1/alpha_jj = 1/alpha_CM + (b1 + b2 m^2 +
 *                     b3 m^2 khat_j^2) kd^2 - (2/3) i kd^3 (the corrected lattice
 *                     dispersion relation §14 recommends, cited: every transverse
 *                     wave then propagates with K = m k to second order);
 *   DDA_ALPHA_CMRR    1/alpha = 1/alpha_CM - (2/3) i kd^3;
 *   DDA_ALPHA_FCD     1/alpha = 1/alpha_CM - [(4/3) kd^2 + (2/(3 pi)) ln((pi - kd)/(pi + kd)) kd^3
 *                     + (2/3) i kd^3] (the FLTRCD print of §14 read with the
 *                     kd^3 factor of its source and the radiative sign). */

typedef struct dda_target dda_target;   /* opaque handle; owns its device memory */

/* One right-hand side: incident direction and polarization in the Target Frame. */
typedef struct {
  double khat[3];          /* unit propagation direction (|khat| = 1 within 1e-12) */
  dda_c64 e[3];            /* polarization, normalised by the library; khat.e = 0 */
} dda_rhs;

typedef struct {
  double tol;              /* stop when |E - A P| / |E| <= tol (FP64 residual), e.g. 1e-5 */
  int32_t max_iter;        /* BiCGSTAB iteration cap per RHS (the guide's MXITER, §9) */
  int32_t precision;       /* DDA_FP64 or DDA_MIXED */
  double inner_tol;        /* MIXED: inner recursive-residual target relative to the
                              current true residual; 0 => tol (one refinement pass) */
  int32_t max_outer;       /* cap on true-residual checks / refinement passes per RHS */
  int32_t check_every;     /* iterations between host convergence checks (>= 1); 0 => the
                              first check after 8 (after 4 on FFT grids of at most 2^18
                              points), then (eager launches) where the decay of the recursive
                              residuals since the last check predicts that the slowest RHS
                              converges (4..64); -n => the same with the first check after
                              n (<= 64) iterations; with use_graph, 0 => 8 (4) and -n => n */
  int32_t use_graph;       /* 1: the check_every iterations between host checks run as one
                              captured HIP graph on a stream of the handle (ordered after and
                              before the caller's stream); 0: kernels are launched directly */
  int32_t solver;          /* DDA_SOLVER_BICGSTAB (the PBCGST option of §12),
                              DDA_SOLVER_BICGSTAB2 (BiCGstab(2), the PBCGS2 option the guide
                              recommends, §12; check_every then counts cycles of two BiCG
                              steps), DDA_SOLVER_COCG or DDA_SOLVER_QMR (the QMRCCG option) */
  int32_t fold_records;    /* tuning only, results are bit-identical: a product with at most this
                              many per-block partial records per RHS lets each block of the
                              kernel that needs its step length (BiCGSTAB alpha and omega, COCG
                              and QMR alpha) sum the records itself; above, one block computes
                              it first.  0 => 1024; < 0 => never */
  const void *x0;          /* NULL: the guide's start P = 0 (§12).  Otherwise a device
                              [nrhs][N][3] dda_c64 initial guess (read only): its FP64 true
                              residual is checked first (one product, counted as one outer
                              pass); an RHS already within tol returns x0 unchanged (up to
                              rounding with jacobi), the others iterate from it as from a
                              refinement restart */
  int32_t jacobi;          /* 1: symmetric diagonal (Jacobi) scaling, the diagonal
                              preconditioning of the PIM solvers §12 cites: the iterations solve
                              (S A S) y = S E with S = diag(alpha)^(1/2) (principal root, one
                              value per composition and component, so S A S has unit diagonal
                              and stays complex symmetric) and return P = S y; tol and
                              rel_resid then refer to |S (E - A P)| / |S E|, which for one
                              composition with a scalar alpha (LDR, CMRR, FCD) is |E - A P| / |E|.
                              0: none */
} dda_solve_opts;

typedef struct {
  int32_t status;          /* 0 converged, 1 max_iter, 2 breakdown without recovery */
  int32_t iters;           /* BiCGSTAB iterations or BiCG steps of BiCGstab(2) (two per
                              cycle), two products each; COCG / QMR iterations, one each */
  int32_t matvecs;         /* FFT products in the iteration precision */
  int32_t outer;           /* true-residual evaluations (FP64 products) */
  double rel_resid;        /* final true relative residual |E - A P| / |E| (FP64) */
} dda_solve_stats;

typedef struct {
  double qext, qabs, qsca; /* efficiencies Q = C / (pi a_eff^2) (§3.1); qsca = qext - qabs */
  double aeff;             /* effective radius in lattice units (§2) */
  double qpha;             /* phase-shift efficiency (§3.2, defined in Draine 1988):
                              C_pha = 2 pi k sum_j Re(conj(E_inc,j) . P_j) */
} dda_q;

/* Far-field averages of one solved RHS (§3.1 outputs). */
typedef struct {
  double qsca;             /* Q_sca = C_sca / (pi a_eff^2), C_sca = k^4 * integral |F_perp|^2 dOmega
                              by quadrature (an independent check of Q_ext - Q_abs) */
  double g;                /* <cos theta>, theta the scattering angle from khat */
  double cos2;             /* <cos^2 theta> */
  int32_t n_theta, n_phi;  /* quadrature: Gauss-Legendre nodes in cos theta, uniform phi */
  double qbk;              /* backscattering: k^4 |F_perp(-khat)|^2 / (pi a_eff^2), the differential
                              cross section (per sr) at theta = 180 deg over pi a_eff^2 (§3.1) */
} dda_far;

typedef struct {
  int32_t box[3];          /* nx, ny, nz */
  int32_t grid[3];         /* padded FFT extents Mx, My, Mz (2/3/5-smooth, >= 2n-1) */
  int64_t n_sites;
  double kd, aeff;
  uint64_t device_bytes;   /* device memory currently held by the handle */
  int32_t zpass_variant[2];/* radix-plan variant of the z-pass (0..3) in DDA_MIXED [0] and DDA_FP64
                              [1]: the autotuner's measured choice for Mz, or the one forced by
                              dda_set_plan_variant; 0 is the cost model's plan */
  int32_t xfwd_variant[2]; /* the same for the x-forward pass (0..1, for Mx) */
  int32_t xinv_variant[2]; /* the same for the x-inverse pass (0..1, for Mx) */
} dda_target_info;

/* ---- target geometry (host arithmetic) ------------------------------- */

/* Occupied sites of a built-in shape (§21).  Sites are centred lattice points
 * of n = nearest-integer(extent) per axis that satisfy the shape's inequality
 * (boundary included), shifted so the smallest index on each axis is 0, in
 * raster order (x fastest).  Call with ijk = NULL to get *n_sites and box;
 * then call again with ijk of capacity >= *n_sites triples.
 * Errors: DDA_EINVAL for an unknown shape, a non-positive extent or a bad
 * orientation code; DDA_EINVAL if capacity is too small. */
int dda_make_sites(int32_t shape, const double shpar[3], int64_t *n_sites,
                   int32_t box[3], int32_t *ijk, int64_t capacity);

/* a_eff = (3N/4pi)^(1/3) and kd = x / a_eff (§2). */
double dda_aeff(int64_t n_sites);
double dda_kd_from_x(double x, int64_t n_sites);

/* Target orientations for orientational averaging (§20): nbeta x ntheta x
 * nphi orientations with weights summing to 1, written as index
 * (it * nphi + ip) * nbeta + ib of the host arrays beta, theta, phi, weight
 * (radians; caller-allocated, nbeta * ntheta * nphi each).  beta and phi are
 * uniformly spaced over [min, max) (min + j (max - min) / n), theta uniformly
 * in cos(theta) between cos(theta_min) and cos(theta_max): for odd ntheta the
 * end points are included with Simpson weights (1, 4, 2, ..., 4, 1) /
 * (3 (ntheta - 1)), for even ntheta the midpoints of ntheta equal intervals
 * with equal weights; n = 1 takes the minimum.  The orientation average of
 * a quantity is sum weight_i Q_i.  Errors: DDA_EINVAL for a count < 1, NULL
 * outputs or non-finite angles. */
int dda_orientation_grid(double beta_min, double beta_max, int32_t nbeta, double theta_min, double theta_max,
                         int32_t ntheta, double phi_min, double phi_max, int32_t nphi, double *beta,
                         double *theta, double *phi, double *weight);

/* Incident direction and polarization in the Target Frame for target
 * orientation (beta, theta, phi) (radians, §19) and Lab-Frame polarization
 * e01 (normalised; x component must be 0).  which = 1 gives e01, which = 2 the
 * orthogonal state e02 = x_LF x conj(e01) (§24).  The target axes a1, a2 are
 * taken along x_TF, y_TF.  Errors: DDA_EINVAL for which not in {1,2} or a
 * zero / non-transverse e01. */
int dda_orient_rhs(double beta, double theta, double phi, const dda_c64 e01_lf[3],
                   int32_t which, dda_rhs *out);

/* ---- target handle ------------------------------------------------------- */

/* Validate the description, copy sites to the device, pick the padded grid
 * and build the Fourier transforms of the six Green-tensor components
 * (FP64 and FP32 copies).  Errors: DDA_EINVAL (N < 1, site outside the box or
 * duplicated, n_comp out of range, non-finite m, m^2 = -2, kd <= 0, FCD with
 * kd >= pi); DDA_ENOTSUP (padded extent > 512); DDA_ENOMEM; DDA_EDEVICE.
 * Returns DDA_WVALIDITY (with a valid handle) when |m|kd >= 1 or |m - 1| > 2
 * for some composition, the guide's validity criteria (§2). */
int dda_setup_target(const dda_target_desc *desc, dda_target **out);

/* Device bytes a target plus a solve of nrhs right-hand sides would hold
 * (setup transient included).  Same validation as dda_setup_target except
 * that sites are not read (ijk may be NULL). */
int dda_footprint_bytes(const dda_target_desc *desc, int32_t nrhs,
                        const dda_solve_opts *opts, uint64_t *bytes);

int dda_target_get_info(const dda_target *t, dda_target_info *info);

/* Plan autotuning (§13 "Choice of FFT Algorithm": the guide picks among FFT
 * implementations; here the choice is among radix plans of one transform
 * length).  The product's passes are numbered as in dda_profile_matvec:
 * 0 x-forward, 2 z-pass, 4 x-inverse (the y passes have one plan per length).
 * z-pass variants: 0 the cost model's plan (fewest LDS stages, then fewest
 * flops, largest radix first, radices bounded so that at least half the
 * threads of a block hold a butterfly), 1 the same with radices up to 16
 * whatever that bound, 2 the cheapest plan with one stage more than 0, 3 the
 * radices of 0 smallest first.  x-pass variants: 0 radices up to 8, 1 radices
 * up to 16.  Variants exist for compile-time lengths of 96 and above; others
 * always use variant 0.  Every variant gives the product to rounding.
 *
 * dda_set_plan_variant forces a pass's variant for this handle; -1 restores
 * the measured choice of the built-in table (written by autotune.py; variant
 * 0 for lengths it has not timed).  Errors: DDA_EINVAL (NULL, pass not 0, 2
 * or 4, variant out of range).  dda_set_zpass_variant(t, v) is
 * dda_set_plan_variant(t, 2, v). */
int dda_set_plan_variant(dda_target *t, int32_t pass, int32_t variant);
int dda_set_zpass_variant(dda_target *t, int32_t variant);

/* The radices, in execution order, of plan `variant` of pass 0, 2 or 4 for the
 * compile-time length L in `precision` (zeros after the last); returns the
 * number of stages, or a negative DDA_E* code (L not 2/3/5-smooth or above
 * 512, pass or variant out of range).  Lengths without a compile-time plan use
 * the run-time radix-8/4/2/5/3 plan in the product instead.
 * dda_zpass_plan(L, p, v, r) is dda_pass_plan(2, L, p, v, r). */
int dda_pass_plan(int32_t pass, int32_t L, int32_t precision, int32_t variant, int32_t radices[8]);
int dda_zpass_plan(int32_t L, int32_t precision, int32_t variant, int32_t radices[8]);

/* Solve A P = E for nrhs right-hand sides as one block (shared FFT grid and
 * Green transform, per-RHS polarizabilities, scalars and convergence).
 * p_dev: device [nrhs][N][3] dda_c64 receiving P, or NULL for a
 *   library-owned buffer (then read P back through p_host).
 * p_host: host [nrhs][N][3] copy of P, or NULL.
 * stats: host [nrhs], or NULL.
 * Returns DDA_OK when every RHS reached tol, DDA_NOT_CONVERGED when some did
 * not (per-RHS status in stats), or an error.  The call is synchronous: P is
 * complete on return.  Errors: DDA_EINVAL (nrhs < 1, |khat| != 1, khat.e != 0,
 * e = 0, tol <= 0, max_iter < 1, bad precision); DDA_ENOMEM; DDA_EDEVICE. */
int dda_solve(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const dda_solve_opts *opts,
              void *p_dev, dda_c64 *p_host, void *stream, dda_solve_stats *stats);

/* Q_ext, Q_abs, Q_sca (= Q_ext - Q_abs) and Q_pha of solved polarizations P,
 * from FP64 sums over the sites (cross sections of Draine 1988 / Draine &
 * Flatau 1994, efficiencies of §3.1 and §3.2).  P is read from p_dev (device) if non-NULL, else from
 * p_host (host).  out: host [nrhs].  Synchronous. */
int dda_cross_sections(dda_target *t, const dda_rhs *rhs, int32_t nrhs,
                       const void *p_dev, const dda_c64 *p_host, void *stream, dda_q *out);

/* Q_sca, <cos theta>, <cos^2 theta> and Q_bk of solved polarizations P
 * (device [nrhs][N][3]) from the far field F(n) = sum_j P_j exp(-i k n.r_j),
 * weighted by |F_perp|^2 (§3.1); Q_bk from F(-khat) alone.  Directions: Gauss-Legendre in cos theta about khat
 * with n_theta = ceil((3 + x)/etasca) + 1 nodes and 2 n_theta uniform phi,
 * x = k a_eff (the guide's ETASCA resolution parameter, §9: the number of
 * directions grows as [(3 + x)/ETASCA]^2; 0.5 is its recommended value).
 * out: host [nrhs].  Synchronous; allocates and frees a scratch buffer.
 * Errors: DDA_EINVAL (etasca <= 0 or so small that n_theta > 2048,
 * |khat| != 1); DDA_ENOMEM; DDA_EDEVICE. */
int dda_far_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev, double etasca,
                  void *stream, dda_far *out);

/* Scattering amplitude and Mueller matrices of one incidence (§26). */
typedef struct {
  dda_c64 f[2][2];         /* f_ml: m = 0 scattered polarization along theta_hat_s, 1 along
                              phi_hat_s; l = incident polarization e01, e02 (eq. f_ml_def) */
  dda_c64 s[4];            /* S_1, S_2, S_3, S_4 (eq. S_ampl_def) */
  double mueller[4][4];    /* S_ij = mueller[i-1][j-1] (Bohren & Huffman relations of §26) */
} dda_scat;

/* Amplitude and Mueller matrices (§26) in ndir scattering directions for the
 * two solved incident polarizations rhs[0] = e01 and rhs[1] = e02 of one
 * incident direction (p_dev: device [2][N][3], solved for those rhs).
 * lab (host [3][3]): the Lab Frame axes x_LF, y_LF, z_LF in the target frame,
 * with x_LF the common khat of both rhs.  theta_phi (host [ndir][2], radians):
 * the scattering direction n = cos(theta) x_LF + sin(theta) (cos(phi) y_LF +
 * sin(phi) z_LF); theta_hat and phi_hat are the derivatives of n.
 * f_ml = kd^3 e_m . sum_j P^(l)_j exp(-i kd n . r_j) (phase origin at the
 * origin of the site coordinates, as for the incident field), S_1..S_4 from
 * f_ml by the four relations of §26 with a = e01* . y_LF, b = e01* . z_LF,
 * c = e02* . y_LF, d = e02* . z_LF.  Synchronous.  Errors: DDA_EINVAL (NULL,
 * ndir < 1, a lab frame that is not orthonormal or whose x_LF is not khat of
 * both rhs); DDA_ENOMEM. */
int dda_scattering_matrix(dda_target *t, const dda_rhs rhs[2], const void *p_dev, const double lab[9],
                          int32_t ndir, const double *theta_phi, void *stream, dda_scat *out);

/* Near field (§29; the post-processor of §30 reads it).  For polarizations
 * p_dev (device [nrhs][N][3], solved for the same rhs) the field at every
 * lattice point q of the target's box extended by margin[a] >= 0 points on
 * both sides of axis a:
 *     E(q) = E_inc(q) + sum over sites l with r_l != q of G(r_q - r_l) P_l,
 * the dipole at q itself excluded, so at an occupied site E is the field that
 * polarizes that dipole (E = P / alpha for an exact solution).  With
 * macroscopic != 0 the field at occupied sites is multiplied by 3 / (eps + 2),
 * eps = m^2 of the site's composition (eq. macro_vs_micro of §29); the line
 * the guide prints in §30 is the field without that factor.
 * e_dev: device [nrhs][Z][Y][X][3] complex128, X = nx + 2 margin[0] (likewise
 * Y, Z); output point (i, j, k) is site coordinate (i - margin[0],
 * j - margin[1], k - margin[2]), and E_inc has the phase origin of the sites.
 * The sum is the FFT product of the extended box, in FP64, on a grid set up
 * for the call (freed before returning).  Queued on the stream; the call
 * returns after its own setup.  Errors: DDA_EINVAL (NULL, negative margin,
 * invalid rhs); DDA_ENOTSUP (an extended extent above 256); DDA_ENOMEM. */
int dda_near_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev,
                   const int32_t margin[3], int32_t macroscopic, void *e_dev, void *stream);

/* E and/or the magnetic field B at the same points (§29: the NRFLD = 2 option,
 * which stores B with E; nonmagnetic material, so B is both the micro- and the
 * macroscopic field).  Arguments as dda_near_field; e_dev or b_dev may be NULL
 * (not both).  b_dev: device [nrhs][Z][Y][X][3] dda_c64, the layout of e_dev,
 *   B(q) = B_inc(q) + sum_{l, r_l != q} k^2 (e^{ikR}/R) (1 - 1/(ikR)) n x P_l,
 * R = |r_q - r_l|, n = (r_q - r_l)/R, B_inc = khat x E_inc (Gaussian units,
 * d = 1).  The sum is a convolution computed with full FP64 3-D FFTs of the
 * padded extended box (two grids of 3 components held during the call, one
 * RHS at a time).  Errors as dda_near_field. */
int dda_near_field_eb(dda_target *t, const dda_rhs *rhs, int32_t nrhs, const void *p_dev,
                      const int32_t margin[3], int32_t macroscopic, void *e_dev, void *b_dev,
                      void *stream);

/* The product AP = A P for nrhs vectors (device [nrhs][N][3] in and out, may
 * not alias), in DDA_FP64 or DDA_MIXED (FP32 FFT convolution, FP64 diagonal
 * and output).  The polarizabilities are those of the given RHS.  Queued on
 * the stream; not synchronous. */
int dda_apply(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision,
              const void *p_dev, void *ap_dev, void *stream);

/* Allocation-free variant of dda_apply, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same product, same kernels, same
 * results as dda_apply (bit for bit), but the FFT work buffers and the per-RHS
 * 1/alpha live in one static device array of DDA_NOALLOC_SCRATCH_BYTES per GPU
 * (held by every process that loads the library, until it ends) instead of
 * the handle's workspaces; the call makes no device or pinned allocation and
 * creates no HIP object (the 1/alpha values reach the device as a kernel
 * argument).
 * Limits: nrhs * n_comp <= 32, and the work buffers of nrhs products,
 * nrhs * (3 nz nxt ny W + My nxt 3 nz W) * (8 B DDA_MIXED, 16 B DDA_FP64) with
 * W = 16 (MIXED) or 8 (FP64) and nxt = ceil(Mx / W), plus 4 KiB must fit in
 * DDA_NOALLOC_SCRATCH_BYTES (a 64^3 block: 37.7 MB per RHS MIXED, 75.5 MB
 * FP64); otherwise DDA_ENOTSUP, nothing queued.
 * Every call on one GPU shares that GPU's array, whichever handle it is made
 * with, and the array keeps the last call's contents: calls that overlap in
 * time on one GPU (other streams, other threads) race and must be ordered by
 * the caller.  Nothing in the array needs to start at zero.  dda_free_target
 * must not run before the work this call queued has finished (synchronize the
 * stream, unless the handle has already queued other work on it).
 * Arguments and errors otherwise as dda_apply.  Queued on the stream. */
#define DDA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int dda_apply_noalloc(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision,
                      const void *p_dev, void *ap_dev, void *stream);

/* Incident field E_j = e exp(i kd khat . r_j) at the sites (eq. AP=E),
 * device [nrhs][N][3] out.  Queued on the stream. */
int dda_incident_field(dda_target *t, const dda_rhs *rhs, int32_t nrhs, void *e_dev, void *stream);

void dda_free_target(dda_target *t);

/* Timing of the product AP = A P as dda_apply computes it, with HIP events
 * recorded on the given stream.  ms_per_pass (host [6]): [0..4] the average
 * milliseconds of one launch of each FFT pass (x-forward, y-forward, z-pass
 * with the Green multiply, y-inverse, x-inverse), each pass launched `reps`
 * times back to back on buffers a full product has just filled; [5] the
 * average of `reps` whole products.  ap_dev receives A P.  Synchronous. */
int dda_profile_matvec(dda_target *t, const dda_rhs *rhs, int32_t nrhs, int32_t precision, int32_t reps,
                       const void *p_dev, void *ap_dev, void *stream, double ms_per_pass[6]);

/* Timing of the FFT passes of the products inside dda_solve (the products of
 * the Krylov iterations and of the FP64 residual checks, §13), as they run in
 * the solve.  With every >= 1, every every-th product that a dda_solve on this
 * handle launches eagerly records a HIP event on the solve's stream before each
 * of its five passes and after the last (at most 512 products between two host
 * synchronisations of the solve; products replayed from a captured graph are
 * not timed); the solve reads the events back at its own synchronisations and
 * adds each pass's duration to per-precision sums.  every = 0 stops timing.
 * Each call resets the sums.  The first call with every >= 1 creates the
 * handle's 3072 events, which live as long as the handle.  Errors: DDA_EINVAL
 * (NULL, every < 0), DDA_EHIP. */
int dda_set_pass_timing(dda_target *t, int32_t every);

/* The sums of dda_set_pass_timing for the products in `precision` (DDA_MIXED:
 * the FP32 products; DDA_FP64: the FP64 ones): ms (host [5]) the total
 * milliseconds of each pass (x-forward, y-forward, z-pass, y-inverse,
 * x-inverse) and *products the number of timed products.  Errors: DDA_EINVAL
 * (NULL, unknown precision). */
int dda_get_pass_timing(const dda_target *t, int32_t precision, double ms[5], int64_t *products);

/* ---- diagnostics --------------------------------------------------------- */

/* Batched 1-D complex FFT (in_dev may equal out_dev) of length n (2/3/5-smooth, <= 512) on
 * the device: out[b][k] = scale * sum_j in[b][j] exp(sign * 2 pi i j k / n),
 * sign = -1 (forward) or +1 (inverse).  precision DDA_FP64 (dda_c64 data) or
 * DDA_MIXED (interleaved float pairs).  This is the FFT engine of the product
 * exposed for testing.  batch = 0 is a no-op (pointers may then be NULL).
 * Synchronous. */
int dda_fft_pencils(int32_t n, int64_t batch, int32_t sign, int32_t precision, double scale,
                    const void *in_dev, void *out_dev, void *stream, int32_t device);

/* Smallest 2/3/5-smooth integer >= n (the grid-extension rule of §13). */
int32_t dda_next_smooth(int32_t n);

/* Message for the last failing call on this thread ("" if none). */
const char *dda_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDA_H */
