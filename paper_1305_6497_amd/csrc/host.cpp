// Host-side arithmetic of the method: target sites, orientation and
// polarization, polarizabilities, FFT plans.  Compiled without floating-point
// contraction so the site rules give the same boundary decisions as a plain
// IEEE evaluation of the same inequalities.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "dda_internal.hpp"

namespace dda {

// ----------------------------------------------------------------- sites --
// §21 "Target Generation: Isolated Finite Targets".  Sampling: n = nearest
// integer of an extent, sites at centred positions u = i - (n-1)/2; a site is
// in the target when the shape's inequality holds at its centre (boundary
// included).  Twice the centred coordinate, 2u = 2i - (n-1), is an integer.
static int nsites(double s) { return (int)std::floor(s + 0.5); }

namespace {
struct SiteSink {
  std::vector<int32_t> ijk;
  void add(int x, int y, int z) {
    ijk.push_back(x);
    ijk.push_back(y);
    ijk.push_back(z);
  }
};

bool is_int(double v) { return std::floor(v) == v; }

// Shift to a zero minimum and report the tight box.  Input is already in
// raster order (x fastest) because every generator loops z, y, x.
void finish(std::vector<int32_t> &ijk, int32_t box[3]) {
  if (ijk.empty()) {
    box[0] = box[1] = box[2] = 0;
    return;
  }
  int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (size_t i = 0; i < ijk.size(); i += 3)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], ijk[i + a]);
      hi[a] = std::max(hi[a], ijk[i + a]);
    }
  for (size_t i = 0; i < ijk.size(); i += 3)
    for (int a = 0; a < 3; ++a) ijk[i + a] -= lo[a];
  for (int a = 0; a < 3; ++a) box[a] = hi[a] - lo[a] + 1;
}
}  // namespace

// ELLIPSOID: (x/S1)^2 + (y/S2)^2 + (z/S3)^2 <= 1/4, i.e. sum (2u_i/S_i)^2 <= 1.
static void ellipsoid(const double s[3], SiteSink &out) {
  const int n[3] = {nsites(s[0]), nsites(s[1]), nsites(s[2])};
  const bool exact = is_int(s[0]) && is_int(s[1]) && is_int(s[2]);
  const int64_t a = (int64_t)s[0], b = (int64_t)s[1], c = (int64_t)s[2];
  const int64_t wx = (b * c) * (b * c), wy = (a * c) * (a * c), wz = (a * b) * (a * b);
  const int64_t rhs = (a * b * c) * (a * b * c);
  for (int k = 0; k < n[2]; ++k) {
    const int64_t Z = 2 * k - (n[2] - 1);
    for (int j = 0; j < n[1]; ++j) {
      const int64_t Y = 2 * j - (n[1] - 1);
      for (int i = 0; i < n[0]; ++i) {
        const int64_t X = 2 * i - (n[0] - 1);
        bool in;
        if (exact) {
          in = X * X * wx + Y * Y * wy + Z * Z * wz <= rhs;
        } else {
          const double fx = double(X) / s[0], fy = double(Y) / s[1], fz = double(Z) / s[2];
          in = fx * fx + fy * fy + fz * fz <= 1.0;
        }
        if (in) out.add(i, j, k);
      }
    }
  }
}

static void rctglprsm(const double s[3], SiteSink &out) {
  const int n[3] = {nsites(s[0]), nsites(s[1]), nsites(s[2])};
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) out.add(i, j, k);
}

// Generic placement: a predicate over the shape's own axes (axial, t1, t2)
// with per-axis site counts nl[3]; perm[l] = Target-Frame axis of local axis l.
template <typename Pred>
static void place(const int nl[3], const int perm[3], Pred inside, SiteSink &out) {
  int ntf[3];
  for (int l = 0; l < 3; ++l) ntf[perm[l]] = nl[l];
  for (int k = 0; k < ntf[2]; ++k)
    for (int j = 0; j < ntf[1]; ++j)
      for (int i = 0; i < ntf[0]; ++i) {
        const int tf[3] = {i, j, k};
        const int loc[3] = {tf[perm[0]], tf[perm[1]], tf[perm[2]]};
        if (inside(loc)) out.add(i, j, k);
      }
}

// CYLINDER1: length S1 along the axis chosen by S3, diameter S2:
// (2u_t1)^2 + (2u_t2)^2 <= S2^2.
static void cylinder1(const double s[3], SiteSink &out) {
  const int axis = (int)s[2];
  DDA_REQUIRE(axis >= 1 && axis <= 3, "CYLINDER1: SHPAR3 must be 1, 2 or 3");
  static const int perms[3][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}};
  const int na = nsites(s[0]), nd = nsites(s[1]);
  const int nl[3] = {na, nd, nd};
  const double D = s[1];
  const bool exact = is_int(D);
  const int64_t D2 = (int64_t)D * (int64_t)D;
  place(nl, perms[axis - 1], [&](const int *loc) {
    const int64_t T1 = 2 * loc[1] - (nd - 1), T2 = 2 * loc[2] - (nd - 1);
    if (exact) return T1 * T1 + T2 * T2 <= D2;
    const double f1 = double(T1), f2 = double(T2);
    return f1 * f1 + f2 * f2 <= D * D;
  }, out);
}

// HEX_PRISM: length S1 along a1, vertex-to-vertex S2; a2 normal to a
// rectangular face.  Circumradius R = S2/2, apothem h = R sqrt(3)/2; inside
// when the projections on the three face normals (0, 60, 120 degrees from
// a2, in the a2-a3 plane) are all <= h in magnitude.
static void hex_prism(const double s[3], SiteSink &out) {
  const int orient = (int)s[2];
  DDA_REQUIRE(orient >= 1 && orient <= 6, "HEX_PRISM: SHPAR3 must be 1..6");
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  const double R = 0.5 * s[1];
  const double h = R * std::sqrt(3.0) / 2.0;
  const int na = nsites(s[0]), n2 = nsites(2.0 * h), n3 = nsites(2.0 * R);
  const int nl[3] = {na, n2, n3};
  const double c60 = 0.5, s60 = std::sqrt(3.0) / 2.0;
  place(nl, perms[orient - 1], [&](const int *loc) {
    const double U = double(2 * loc[1] - (n2 - 1)) / 2.0;
    const double Wc = double(2 * loc[2] - (n3 - 1)) / 2.0;
    return std::fabs(U) <= h && std::fabs(c60 * U + s60 * Wc) <= h && std::fabs(-c60 * U + s60 * Wc) <= h;
  }, out);
}

std::vector<int32_t> make_sites(int shape, const double shpar[3], int32_t box[3]) {
  SiteSink out;
  switch (shape) {
    case DDA_SHAPE_ELLIPSOID:
      DDA_REQUIRE(shpar[0] > 0 && shpar[1] > 0 && shpar[2] > 0, "ELLIPSOID: extents must be > 0");
      ellipsoid(shpar, out);
      break;
    case DDA_SHAPE_RCTGLPRSM:
      DDA_REQUIRE(shpar[0] >= 0.5 && shpar[1] >= 0.5 && shpar[2] >= 0.5, "RCTGLPRSM: extents must be >= 1");
      rctglprsm(shpar, out);
      break;
    case DDA_SHAPE_CYLINDER1:
      DDA_REQUIRE(shpar[0] > 0 && shpar[1] > 0, "CYLINDER1: extents must be > 0");
      cylinder1(shpar, out);
      break;
    case DDA_SHAPE_HEX_PRISM:
      DDA_REQUIRE(shpar[0] > 0 && shpar[1] > 0, "HEX_PRISM: extents must be > 0");
      hex_prism(shpar, out);
      break;
    default:
      throw Error{DDA_EINVAL, "unknown shape code"};
  }
  finish(out.ijk, box);
  return std::move(out.ijk);
}

// ------------------------------------------------------------ orientation --
// §19: x_LF, y_LF, z_LF in the basis of the target axes (a1, a2, a3), which
// are x_TF, y_TF, z_TF for the built-in targets used here.
void periodic_rule(double lo, double hi, int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.assign(n, 1.0 / n);
  for (int j = 0; j < n; ++j) x[j] = lo + j * (hi - lo) / n;
}

void cos_theta_rule(double lo, double hi, int n, std::vector<double> &theta, std::vector<double> &w) {
  theta.resize(n);
  w.resize(n);
  const double c0 = std::cos(lo), c1 = std::cos(hi);
  if (n == 1) {
    theta[0] = lo;
    w[0] = 1.0;
  } else if (n % 2 == 1) {
    for (int j = 0; j < n; ++j) {
      const double u = c0 + (c1 - c0) * j / (n - 1);
      theta[j] = std::acos(std::min(1.0, std::max(-1.0, u)));
      const double simpson = (j == 0 || j == n - 1) ? 1.0 : (j % 2 == 1 ? 4.0 : 2.0);
      w[j] = simpson / (3.0 * (n - 1));
    }
  } else {
    for (int j = 0; j < n; ++j) {
      const double u = c0 + (c1 - c0) * (j + 0.5) / n;
      theta[j] = std::acos(std::min(1.0, std::max(-1.0, u)));
      w[j] = 1.0 / n;
    }
  }
}

void orient_rhs(double beta, double theta, double phi, const c64 e01[3], int which, RhsDev &out) {
  DDA_REQUIRE(which == 1 || which == 2, "which must be 1 or 2");
  const std::complex<double> ey(e01[1].x, e01[1].y), ez(e01[2].x, e01[2].y);
  DDA_REQUIRE(e01[0].x == 0.0 && e01[0].y == 0.0, "e01 must be transverse to x_LF");
  const double nrm = std::sqrt(std::norm(ey) + std::norm(ez));
  DDA_REQUIRE(nrm > 0.0 && std::isfinite(nrm), "e01 must be non-zero and finite");
  std::complex<double> py = ey / nrm, pz = ez / nrm;
  if (which == 2) {            // e02 = x_LF x conj(e01) = (0, -conj(e01_z), conj(e01_y))  (§24)
    const std::complex<double> ny = -std::conj(pz), nz = std::conj(py);
    py = ny;
    pz = nz;
  }
  const double cb = std::cos(beta), sb = std::sin(beta);
  const double ct = std::cos(theta), st = std::sin(theta);
  const double cp = std::cos(phi), sp = std::sin(phi);
  const double xl[3] = {ct, -st * cb, st * sb};
  const double yl[3] = {st * cp, ct * cb * cp - sb * sp, -(ct * sb * cp + cb * sp)};
  const double zl[3] = {st * sp, ct * cb * sp + sb * cp, -(ct * sb * sp - cb * cp)};
  for (int a = 0; a < 3; ++a) {
    out.khat[a] = xl[a];
    const std::complex<double> e = py * yl[a] + pz * zl[a];
    out.e[a] = c64{e.real(), e.imag()};
  }
}

// --------------------------------------------------------- polarizability --
// §14.  Clausius-Mossotti alpha_CM = (3/4pi)(m^2-1)/(m^2+2) (d = 1).
// LATTDR (Draine & Goodman 1993, cited, not printed):
//   1/alpha = 1/alpha_CM + (b1 + b2 m^2 + b3 m^2 S) kd^2 - (2/3) i kd^3,
//   S = sum_l (khat_l e_l)^2.
// CM with radiative reaction: 1/alpha = 1/alpha_CM - (2/3) i kd^3.
// FLTRCD (reading of the garbled print: kd^3 on the log term, sign such that
// a lossless target does not absorb):
//   1/alpha = 1/alpha_CM - [(4/3) kd^2 + (2/(3 pi)) ln((pi-kd)/(pi+kd)) kd^3 + (2/3) i kd^3].
void alpha_inverse(int kind, c64 mc, double kd, const double khat[3], const c64 e[3], c64 out[3]) {
  using C = std::complex<double>;
  const C m(mc.x, mc.y);
  const C m2 = m * m;
  const double pi = 3.14159265358979323846;
  const C acm_inv = (4.0 * pi / 3.0) * (m2 + 2.0) / (m2 - 1.0);
  const double k2 = kd * kd, k3 = kd * kd * kd;
  const double b1 = -1.891531, b2 = 0.1648469, b3 = -1.7700004;
  C r[3];
  if (kind == DDA_ALPHA_LDR) {
    double S = 0.0;                       // sum_l khat_l^2 |e_l|^2
    for (int l = 0; l < 3; ++l) S += khat[l] * khat[l] * (e[l].x * e[l].x + e[l].y * e[l].y);
    r[0] = acm_inv + (b1 + b2 * m2 + b3 * m2 * S) * k2 - C(0.0, 2.0 / 3.0) * k3;
    r[1] = r[2] = r[0];
  } else if (kind == DDA_ALPHA_GKDLDR) {
    for (int l = 0; l < 3; ++l)
      r[l] = acm_inv + (b1 + b2 * m2 + b3 * m2 * (khat[l] * khat[l])) * k2 - C(0.0, 2.0 / 3.0) * k3;
  } else if (kind == DDA_ALPHA_CMRR) {
    r[0] = r[1] = r[2] = acm_inv - C(0.0, 2.0 / 3.0) * k3;
  } else {
    const double lg = std::log((pi - kd) / (pi + kd));
    r[0] = acm_inv - ((4.0 / 3.0) * k2 + (2.0 / (3.0 * pi)) * lg * k3 + C(0.0, 2.0 / 3.0) * k3);
    r[1] = r[2] = r[0];
  }
  for (int l = 0; l < 3; ++l) out[l] = c64{r[l].real(), r[l].imag()};
}

// --------------------------------------------------------------- FFT plans --
int next_smooth(int n) {
  if (n <= 1) return 1;
  for (int m = n;; ++m) {
    int v = m;
    for (int p : {2, 3, 5})
      while (v % p == 0) v /= p;
    if (v == 1) return m;
  }
}

// Radix plan of a transform: radix 8 while it divides, then 4, 2, 5, 3
// (the radices fft_lds.hpp implements).
// Nodes: roots of P_n by Newton's method from cos(pi (i + 3/4) / (n + 1/2)),
// with P_n and P_n' from the three-term recurrence; weights
// 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  DDA_REQUIRE(n >= 1, "need at least one node");
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n == 1 ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    if (n == 1) dp = 1.0;
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n == 1 ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    }
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

FastDiv make_fastdiv(uint32_t d) {
  DDA_REQUIRE(d >= 1, "division by zero");
  FastDiv f;
  if ((d & (d - 1)) == 0) {
    f.sh = 0;
    while ((1u << f.sh) < d) ++f.sh;
    f.m = 0;
  } else {
    f.sh = -1;
    f.m = (uint32_t)((uint64_t(1) << 32) / d + 1);
  }
  return f;
}

AxisPlan make_axis_plan(int L) {
  DDA_REQUIRE(L >= 1 && L <= kMaxLen, "FFT length out of range");
  AxisPlan p{};
  p.L = L;
  p.nstages = 0;
  int n = L;
  auto take = [&](int r) {
    while (n % r == 0) {
      if (p.nstages >= kMaxStages) throw Error{DDA_ENOTSUP, "too many FFT stages"};
      p.radix[p.nstages++] = r;
      n /= r;
    }
  };
  take(8);
  take(4);
  take(2);
  take(5);
  take(3);
  if (n != 1) throw Error{DDA_EINVAL, "FFT length must be 2/3/5-smooth"};
  int ns = 1;
  for (int s = 0; s < p.nstages; ++s) {
    const int R = p.radix[s];
    p.ns[s] = ns;
    p.lr[s] = L / R;
    p.twstep[s] = L / (ns * R);
    p.ns_div[s] = make_fastdiv((uint32_t)ns);
    p.lr_div[s] = make_fastdiv((uint32_t)(L / R));
    ns *= R;
  }
  return p;
}

}  // namespace dda
