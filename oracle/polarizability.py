"""Dipole polarizabilities, lattice units (d = 1), Gaussian units.

§14 "Choice of DDA Method" of the DDSCAT 7.3 guide names the prescriptions:

* Clausius-Mossotti, alpha_CM = (3 d^3 / 4 pi) (m^2 - 1)/(m^2 + 2)  (printed
  in §14, FLTRCD subsection).
* LATTDR, the lattice dispersion relation of Draine & Goodman (1993).  The
  guide cites it but does not print it.  Reading (from the cited paper):

      alpha = alpha_CM / (1 + (alpha_CM/d^3) [ (b1 + b2 m^2 + b3 m^2 S)(kd)^2
                                               - (2/3) i (kd)^3 ])

  with b1 = -1.891531, b2 = 0.1648469, b3 = -1.7700004 and
  S = sum_l khat_l^2 |e_l|^2 over the three Target-Frame components of the
  unit propagation vector khat and polarization vector e.  For a linear
  polarization (e real up to a phase) this is the cited sum_l (khat_l e_l)^2;
  written with |e_l|^2 it does not change when e is multiplied by a phase
  factor, which leaves every physical quantity unchanged.  The -(2/3) i (kd)^3
  term is the radiative reaction; its sign is pinned by the requirement that
  a lossless (real m) target absorbs nothing.  The b-constants are pinned by
  the lattice sums of ``lattice_sums``: they are the coefficients of the
  second-order terms of the infinite lattice's dispersion relation.
* GKDLDR, the lattice dispersion relation as corrected by Gutkowicz-Krusin &
  Draine (2004), the option §14 recommends; cited, not printed.  Reading: the
  polarizability is a diagonal tensor in the lattice axes that depends on the
  propagation direction only,

      1/alpha_jj = 1/alpha_CM + (b1 + b2 m^2 + b3 m^2 khat_j^2)(kd)^2 - (2/3) i (kd)^3,

  with the LATTDR constants.  It cancels the lattice's anisotropic
  second-order term component by component, so that every transverse wave,
  whatever its polarization, propagates with K = m k to second order, where
  the scalar LATTDR achieves this only for the projection on e.  Pinned by the
  lattice sums (every transverse wave a mode) and by the efficiencies the
  guide prints for its GKDLDR example (appendix .avg file, Q_pha included).
* CM with radiative reaction: alpha = alpha_CM / (1 - (2/3) i k^3 alpha_CM).
* FLTRCD, the filtered coupled dipole polarizability of §14.  The printed
  correction D is garbled: its log term lacks the (kd)^3 factor of the cited
  source, and its sign makes a lossless target absorb.  Reading used here:

      alpha = alpha_CM / (1 - (alpha_CM/d^3) [ (4/3)(kd)^2
                 + (2/(3 pi)) ln((pi - kd)/(pi + kd)) (kd)^3 + (2/3) i (kd)^3 ])

  Only the polarizability is modelled (the filtered Green function of the
  full FCD method is outside this oracle).  The bracket is the k-dependent
  part of the field that the point dipole's field, band-limited to
  wavenumbers below pi/d, puts on the dipole itself; a test computes that
  integral by quadrature and pins every term of the reading with it.

All functions return the inverse polarizability 1/alpha (complex128), which
is what enters the diagonal of A in eq. (AP=E): a scalar, or for GKDLDR the
three diagonal elements of the tensor.
"""

import math

import numpy as np

LDR_B1 = -1.891531
LDR_B2 = 0.1648469
LDR_B3 = -1.7700004


def alpha_cm(m):
    """Clausius-Mossotti polarizability for d = 1."""
    m2 = np.asarray(m, dtype=complex) ** 2
    return (3.0 / (4.0 * math.pi)) * (m2 - 1.0) / (m2 + 2.0)


def ldr_s(khat, e):
    """S = sum_l khat_l^2 |e_l|^2 for the LDR correction (Target Frame; e a unit vector)."""
    khat = np.asarray(khat, dtype=float)
    e = np.asarray(e, dtype=complex)
    return float(np.sum(khat ** 2 * np.abs(e) ** 2))


def alpha_inv_ldr(m, kd, khat, e):
    """1/alpha for LATTDR (reading above)."""
    m2 = np.asarray(m, dtype=complex) ** 2
    s = ldr_s(khat, e)
    return 1.0 / alpha_cm(m) + (LDR_B1 + LDR_B2 * m2 + LDR_B3 * m2 * s) * kd ** 2 - (2.0 / 3.0) * 1j * kd ** 3


def alpha_inv_gkdldr(m, kd, khat):
    """Diagonal of the inverse polarizability tensor for GKDLDR, complex [1, 3]
    (one tensor for every site of the composition)."""
    m2 = complex(m) ** 2
    a2 = np.asarray(khat, dtype=float).reshape(1, 3) ** 2
    return 1.0 / alpha_cm(m) + (LDR_B1 + LDR_B2 * m2 + LDR_B3 * m2 * a2) * kd ** 2 - (2.0 / 3.0) * 1j * kd ** 3


def alpha_inv_cmrr(m, kd):
    """1/alpha for Clausius-Mossotti with radiative reaction."""
    return 1.0 / alpha_cm(m) - (2.0 / 3.0) * 1j * kd ** 3


def alpha_inv_fcd(m, kd):
    """1/alpha for FLTRCD (reading above); requires kd < pi."""
    lg = math.log((math.pi - kd) / (math.pi + kd))
    return 1.0 / alpha_cm(m) - ((4.0 / 3.0) * kd ** 2 + (2.0 / (3.0 * math.pi)) * lg * kd ** 3
                               + (2.0 / 3.0) * 1j * kd ** 3)


def alpha_inv(kind, m, kd, khat, e):
    """Dispatch on the guide's option name: LATTDR, GKDLDR, CMRR, FLTRCD
    (GKDLDR returns the tensor diagonal [1, 3], the others a scalar)."""
    if kind == "LATTDR":
        return alpha_inv_ldr(m, kd, khat, e)
    if kind == "GKDLDR":
        return alpha_inv_gkdldr(m, kd, khat)
    if kind == "CMRR":
        return alpha_inv_cmrr(m, kd)
    if kind == "FLTRCD":
        return alpha_inv_fcd(m, kd)
    raise ValueError(kind)
