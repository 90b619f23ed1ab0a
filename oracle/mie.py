"""Mie-theory efficiencies of a homogeneous sphere.

§2 "Applicability of the DDA" judges DDA accuracy by comparison with Mie
theory for spheres (Bohren & Huffman 1983, cited in the guide); as kd -> 0
the DDA cross sections of a dipole pseudosphere must approach these.

Textbook series, e^{-i w t}:  with psi_n(x) = x j_n(x), xi_n(x) = x h_n^(1)(x)
and D_n(z) = psi_n'(z)/psi_n(z) (by downward recurrence,
D_{n-1} = n/z - 1/(D_n + n/z)),

    a_n = [(D_n(mx)/m + n/x) psi_n - psi_{n-1}] / [(D_n(mx)/m + n/x) xi_n - xi_{n-1}]
    b_n = [(m D_n(mx) + n/x) psi_n - psi_{n-1}] / [(m D_n(mx) + n/x) xi_n - xi_{n-1}]
    Q_ext = (2/x^2) sum (2n+1) Re(a_n + b_n)
    Q_sca = (2/x^2) sum (2n+1) (|a_n|^2 + |b_n|^2),   Q_abs = Q_ext - Q_sca

summed to n_max = x + 4 x^(1/3) + 2 (Wiscombe 1980).  The asymmetry parameter
g = <cos theta> (the guide's <cos theta>, §3.1 output) is the textbook sum

    g Q_sca = (4/x^2) sum [ n(n+2)/(n+1) Re(a_n a*_{n+1} + b_n b*_{n+1})
                            + (2n+1)/(n(n+1)) Re(a_n b*_n) ].
"""

import math

import numpy as np
import scipy.special as ssp


def mie_coefficients(m, x):
    """Arrays a[n], b[n] for n = 0..n_max (index 0 unused, zero)."""
    m = complex(m)
    nmax = int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    mx = m * x
    nstart = int(max(nmax, abs(mx))) + 16
    D = np.zeros(nstart + 1, dtype=complex)
    for n in range(nstart, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)
    n = np.arange(0, nmax + 1)
    psi = x * ssp.spherical_jn(n, x)
    xi = x * (ssp.spherical_jn(n, x) + 1j * ssp.spherical_yn(n, x))
    a = np.zeros(nmax + 1, dtype=complex)
    b = np.zeros(nmax + 1, dtype=complex)
    for k in range(1, nmax + 1):
        da = D[k] / m + k / x
        db = m * D[k] + k / x
        a[k] = (da * psi[k] - psi[k - 1]) / (da * xi[k] - xi[k - 1])
        b[k] = (db * psi[k] - psi[k - 1]) / (db * xi[k] - xi[k - 1])
    return a, b


def mie_q(m, x):
    """Return dict(qext, qsca, qabs, g) for relative index m and size parameter x."""
    a, b = mie_coefficients(m, x)
    nmax = len(a) - 1
    k = np.arange(1, nmax + 1)
    qe = 2.0 / (x * x) * float(np.sum((2 * k + 1) * (a[1:] + b[1:]).real))
    qs = 2.0 / (x * x) * float(np.sum((2 * k + 1) * (np.abs(a[1:]) ** 2 + np.abs(b[1:]) ** 2)))
    a1 = np.append(a, 0.0)
    b1 = np.append(b, 0.0)
    gq = float(np.sum(k * (k + 2) / (k + 1) * (a1[k] * np.conj(a1[k + 1]) + b1[k] * np.conj(b1[k + 1])).real))
    gq += float(np.sum((2 * k + 1) / (k * (k + 1)) * (a[k] * np.conj(b[k])).real))
    g = 4.0 / (x * x) * gq / qs if qs > 0 else 0.0
    return dict(qext=qe, qsca=qs, qabs=qe - qs, g=g)
