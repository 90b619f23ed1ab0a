"""Dipole polarizabilities, lattice units (d = 1), Gaussian units.

§14 "Choice of DDA Method" of the DDSCAT 7.3 guide names the prescriptions:

* Clausius-Mossotti, alpha_CM = (3 d^3 / 4 pi) (m^2 - 1)/(m^2 + 2)  (printed
  in §14, FLTRCD subsection).
* LATTDR, the lattice dispersion relation of Draine & Goodman (1993).  The
  guide cites it but does not print it.  Reading (from the cited paper):

      alpha = alpha_CM / (1 + (alpha_CM/d^3) [ (b1 + b2 m^2 + b3 m^2 S)(kd)^2
                                               - (2/3) i (kd)^3 ])

  with b1 = -1.891531, b2 = 0.1648469, b3 = -1.7700004 and
  S = sum_l (khat_l e_l)^2 over the three Target-Frame components of the unit
  propagation vector khat and polarization vector e.  The -(2/3) i (kd)^3
  term is the radiative reaction; its sign is pinned by the requirement that
  a lossless (real m) target absorbs nothing.  The b-constants are quoted
  from the literature and are "parity unpinned" by the guide.
* CM with radiative reaction: alpha = alpha_CM / (1 - (2/3) i k^3 alpha_CM).
* FLTRCD, the filtered coupled dipole polarizability of §14.  The printed
  correction D is garbled: its log term lacks the (kd)^3 factor of the cited
  source, and its sign makes a lossless target absorb.  Reading used here:

      alpha = alpha_CM / (1 - (alpha_CM/d^3) [ (4/3)(kd)^2
                 + (2/(3 pi)) ln((pi - kd)/(pi + kd)) (kd)^3 + (2/3) i (kd)^3 ])

  Only the polarizability is modelled (the filtered Green function of the
  full FCD method is outside this oracle).  Pinned by the kd -> 0 limit and
  the lossless test; otherwise parity unpinned.

All functions return the inverse polarizability 1/alpha (complex128), which
is what enters the diagonal of A in eq. (AP=E).
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
    """S = sum_l (khat_l e_l)^2 for the LDR correction (Target Frame)."""
    khat = np.asarray(khat, dtype=complex)
    e = np.asarray(e, dtype=complex)
    return complex(np.sum((khat * e) ** 2))


def alpha_inv_ldr(m, kd, khat, e):
    """1/alpha for LATTDR (reading above)."""
    m2 = np.asarray(m, dtype=complex) ** 2
    s = ldr_s(khat, e)
    return 1.0 / alpha_cm(m) + (LDR_B1 + LDR_B2 * m2 + LDR_B3 * m2 * s) * kd ** 2 - (2.0 / 3.0) * 1j * kd ** 3


def alpha_inv_cmrr(m, kd):
    """1/alpha for Clausius-Mossotti with radiative reaction."""
    return 1.0 / alpha_cm(m) - (2.0 / 3.0) * 1j * kd ** 3


def alpha_inv_fcd(m, kd):
    """1/alpha for FLTRCD (reading above); requires kd < pi."""
    lg = math.log((math.pi - kd) / (math.pi + kd))
    return 1.0 / alpha_cm(m) - ((4.0 / 3.0) * kd ** 2 + (2.0 / (3.0 * math.pi)) * lg * kd ** 3
                               + (2.0 / 3.0) * 1j * kd ** 3)


def alpha_inv(kind, m, kd, khat, e):
    """Dispatch on the guide's option name: LATTDR, CMRR, FLTRCD."""
    if kind == "LATTDR":
        return alpha_inv_ldr(m, kd, khat, e)
    if kind == "CMRR":
        return alpha_inv_cmrr(m, kd)
    if kind == "FLTRCD":
        return alpha_inv_fcd(m, kd)
    raise ValueError(kind)
