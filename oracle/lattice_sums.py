"""Dipole lattice sums: the dispersion relation that LATTDR and GKDLDR match.

TEST INFRASTRUCTURE (part of the oracle): used only by the tests that pin the
polarizability prescriptions of §14.

The LATTDR and GKDLDR options of §14 ("Choice of DDA Method") choose the
dipole polarizability so that an infinite cubic lattice of point dipoles
(spacing d = 1) carries a plane wave with the dispersion relation of the
continuum it represents, K = m k, up to second order in kd.  The guide cites
the derivations (Draine & Goodman 1993; Gutkowicz-Krusin & Draine 2004) and
prints neither.  This module states the condition itself, so that the
coefficients of the prescriptions can be checked against it rather than
against a retyped formula.

A polarization wave P_R = P exp(i K.R) on the lattice points R is a free mode
(no incident field) when every dipole is driven by the field of all others:

    P / alpha = T(K, k) P,   T(K, k) = sum_{R != 0} G(R) exp(i K.R),

with G = (k^2 + grad grad) exp(ikr)/r the dipole field tensor of the product
A P (eq. AP=E).  The sum converges only conditionally; it is evaluated with
Ewald's split of exp(ikr)/r at a parameter eta (the Helmholtz form of the
split, as in the lattice-sum literature):

    exp(ikr)/r = f_s(r) + f_l(r),
    f_s(r) = [exp(ikr) erfc(eta r + i a) + exp(-ikr) erfc(eta r - i a)] / (2r),
    a = k / (2 eta),

f_s decays like a Gaussian and is summed over lattice points; the lattice sum
of f_l is a sum over reciprocal vectors q = K + 2 pi n (unit cell volume 1)

    sum_R exp(i K.R) f_l(|r - R|) = 4 pi sum_q exp(i q.r) exp(-(q^2 - k^2)/(4 eta^2)) / (q^2 - k^2).

Applying k^2 + grad grad and taking r -> 0 with the R = 0 term removed gives

    T = 4 pi sum_q (k^2 I - q q) exp(-(q^2 - k^2)/(4 eta^2)) / (q^2 - k^2)
        + sum_{R != 0} exp(i K.R) [k^2 f_s I + f_s'' n n + (f_s' / r)(I - n n)]
        + (k^2 h0 + 2 h2) I,

where h(r) = f_s(r) - exp(ikr)/r = h0 + h2 r^2 + ... is regular at r = 0;
h0 and h2 follow from the Taylor series of erf about i a (written out in
``_self_term``).  The result does not depend on eta (a test checks this), and
its imaginary part is exactly -(2/3) k^3 I when no q has |q| = k.
"""

import math

import numpy as np
import scipy.special as ssp


def _short_range(rho, k, eta):
    """f_s and its first two derivatives at distances rho > 0 (arrays)."""
    a = k / (2.0 * eta)
    ep, em = np.exp(1j * k * rho), np.exp(-1j * k * rho)
    psp = ssp.erfc(eta * rho + 1j * a)
    psm = ssp.erfc(eta * rho - 1j * a)
    v = ep * psp + em * psm
    w = ep * psp - em * psm
    # exp(+-ikr) times the Gaussian derivative of erfc(eta r +- i a): both
    # equal exp(a^2 - eta^2 r^2) because 2 eta a = k
    g = np.exp(a * a - (eta * rho) ** 2)
    v1 = 1j * k * w - (4.0 * eta / math.sqrt(math.pi)) * g
    v2 = -k * k * v + (8.0 * eta ** 3 * rho / math.sqrt(math.pi)) * g
    f0 = v / (2.0 * rho)
    f1 = v1 / (2.0 * rho) - v / (2.0 * rho ** 2)
    f2 = v2 / (2.0 * rho) - v1 / rho ** 2 + v / rho ** 3
    return f0, f1, f2


def _self_term(k, eta):
    """h0 and h2 of h(r) = f_s(r) - exp(ikr)/r = h0 + h2 r^2 + O(r^4).

    With u(r) = 2 r h(r) = -exp(ikr)(1 + erf(eta r + i a)) + exp(-ikr)(1 - erf(eta r - i a))
    (odd in r), h0 = u'(0)/2 and h2 = u'''(0)/12.  The derivatives of
    erf(eta r +- i a) at r = 0 are c1 = (2 eta/sqrt(pi)) e^{a^2}, -+ i c2 with
    c2 = (4 eta^2 a/sqrt(pi)) e^{a^2}, and c3 = -(4 eta^3/sqrt(pi))(1 + 2 a^2) e^{a^2};
    erf(+- i a) = +- i erfi(a).
    """
    a = k / (2.0 * eta)
    ea = math.exp(a * a)
    sp = math.sqrt(math.pi)
    E = ssp.erfi(a)
    c1 = 2.0 * eta / sp * ea
    c2 = 4.0 * eta ** 2 * a / sp * ea
    c3 = -4.0 * eta ** 3 / sp * (1.0 + 2.0 * a * a) * ea
    h0 = -1j * k * (1.0 + 1j * E) - c1
    h2 = (1j * k ** 3 * (1.0 + 1j * E) + 3.0 * k * k * c1 - 3.0 * k * c2 - c3) / 6.0
    return h0, h2


def dipole_lattice_sum(K, k, eta=math.sqrt(math.pi), nmax=6):
    """T(K, k) = sum_{R != 0} G(R) exp(i K.R) on the unit cubic lattice, complex [3, 3].

    K: real wave vector [3] (|K + 2 pi n| != k for every integer n), k > 0.
    """
    K = np.asarray(K, dtype=float)
    n = np.arange(-nmax, nmax + 1)
    N = np.stack(np.meshgrid(n, n, n, indexing="ij"), axis=-1).reshape(-1, 3).astype(float)
    eye = np.eye(3)
    # reciprocal-space part
    q = K[None, :] + 2.0 * math.pi * N
    q2 = np.sum(q * q, axis=1)
    wgt = 4.0 * math.pi * np.exp(-(q2 - k * k) / (4.0 * eta * eta)) / (q2 - k * k)
    T = np.einsum("i,ab->ab", wgt * k * k, eye) - np.einsum("i,ia,ib->ab", wgt, q, q)
    T = T.astype(complex)
    # real-space part (R != 0)
    R = N[np.any(N != 0, axis=1)]
    rho = np.sqrt(np.sum(R * R, axis=1))
    f0, f1, f2 = _short_range(rho, k, eta)
    nn = R[:, :, None] * R[:, None, :] / (rho ** 2)[:, None, None]
    ph = np.exp(1j * (R @ K))
    H = (k * k * f0 + f1 / rho)[:, None, None] * eye[None] + (f2 - f1 / rho)[:, None, None] * nn
    T += np.einsum("i,iab->ab", ph, H)
    # the R = 0 term: the regular remainder of the split
    h0, h2 = _self_term(k, eta)
    T += (k * k * h0 + 2.0 * h2) * eye
    return T
