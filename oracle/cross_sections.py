"""Cross sections and efficiencies from a solved polarization P.

§3.1 "What Does It Calculate?" defines the efficiencies
Q = C / (pi a_eff^2) for extinction, absorption and scattering.  The sums
that give C from the dipole moments are cited (Draine 1988; Draine & Flatau
1994), not printed.  Reading, with |E_0| = 1 and d = 1:

    C_ext = 4 pi k sum_j Im( conj(E_inc,j) . P_j )
    C_abs = 4 pi k sum_j [ Im( P_j . conj(1/alpha_j) conj(P_j) ) - (2/3) k^3 |P_j|^2 ]

(for a diagonal 1/alpha tensor the first term is sum_c Im(conj(1/alpha_jc)) |P_jc|^2)
    C_sca = k^4 * integral dOmega | sum_j (I - n n) P_j e^{-i k n.r_j} |^2
          = 4 pi k^4 sum_j sum_l conj(P_j) . K(k R_jl) . P_l

with R_jl = r_j - r_l and, using the angular integral
integral dOmega (I - n n) e^{i k n.R} = 4 pi K(kR),

    K(x) = (j0(x) - j1(x)/x) I + j2(x) Rhat Rhat,    K(0) = (2/3) I

(spherical Bessel functions j_n).  ``c_sca_quadrature`` evaluates the same
far-field integral by brute-force angular quadrature, as an independent check
of ``c_sca_exact``.

``far_field`` does the same quadrature about the incident direction khat and
also returns the angular averages of §3.1, weighted by the scattered
intensity |F_perp(n)|^2 with cos theta = n . khat:

    g = <cos theta>,   <cos^2 theta>.

§3.1 also lists Q_bk, the differential scattering cross section for
backscattering (area per steradian) over pi a_eff^2, and §3.2 Q_pha, the
phase-shift cross section over pi a_eff^2 (defined in Draine 1988, cited).
Readings:

    dC_sca/dOmega (n) = k^4 | sum_j (I - n n) P_j e^{-i k n.r_j} |^2,
    Q_bk = dC_sca/dOmega (n = -khat) / (pi a_eff^2),
    C_pha = 2 pi k sum_j Re( conj(E_inc,j) . P_j ),

the last being the phase delay per unit column density that the real part of
the response imposes on the transmitted wave, as C_ext is (twice) the
amplitude attenuation (for one dipole C_pha = 2 pi k Re alpha, the
dilute-medium refractive index n - 1 = 2 pi N alpha in these units).

The guide chooses its scattering directions by the parameter ETASCA (number
of directions proportional to [(3 + x)/ETASCA]^2) without printing the rule.
Reading: Gauss-Legendre in cos theta with n_theta = ceil((3 + x)/ETASCA) + 1
nodes and a uniform phi grid of 2 n_theta points, which integrates the
band-limited far-field intensity (degree about 2x in each angle) exactly for
ETASCA <= 1.
"""

import math

import numpy as np
import scipy.special as ssp

from . import interaction


def c_ext(kd, E_inc, P):
    return 4.0 * math.pi * kd * float(np.sum(np.imag(np.conj(E_inc) * P)))


def c_pha(kd, E_inc, P):
    """Phase-shift cross section (module docstring)."""
    return 2.0 * math.pi * kd * float(np.sum(np.real(np.conj(E_inc) * P)))


def dc_sca_domega(sites, kd, P, n):
    """Differential scattering cross section in direction(s) n [..., 3] (unit)."""
    sites = np.asarray(sites, dtype=float)
    n = np.asarray(n, dtype=float).reshape(-1, 3)
    F = np.exp(-1j * kd * (n @ sites.T)) @ np.asarray(P, dtype=complex)          # [m, 3]
    Fperp = F - np.sum(n * F, axis=1, keepdims=True) * n
    return kd ** 4 * np.sum(np.abs(Fperp) ** 2, axis=1)


def c_abs(kd, alpha_inv_sites, P):
    P = np.asarray(P, dtype=complex)
    ai = interaction.alpha_inv_diag(alpha_inv_sites, P.shape[0])
    p2 = np.abs(P) ** 2
    term = np.imag(np.conj(ai)) * p2 - (2.0 / 3.0) * kd ** 3 * p2
    return 4.0 * math.pi * kd * float(np.sum(term))


def _k_tensor(x, Rhat):
    """K(x) of the module docstring for arrays x[...] > 0, Rhat[..., 3]."""
    j0 = ssp.spherical_jn(0, x)
    j1 = ssp.spherical_jn(1, x)
    j2 = ssp.spherical_jn(2, x)
    a = j0 - j1 / x
    return a[..., None, None] * np.eye(3) + j2[..., None, None] * (Rhat[..., :, None] * Rhat[..., None, :])


def c_sca_exact(sites, kd, P, block=512):
    """Exact C_sca of the dipole array by the O(N^2) double sum."""
    sites = np.asarray(sites, dtype=float)
    P = np.asarray(P, dtype=complex)
    n = sites.shape[0]
    total = (2.0 / 3.0) * float(np.sum(np.abs(P) ** 2))        # j == l terms
    for j0 in range(0, n, block):
        j1 = min(n, j0 + block)
        R = sites[j0:j1, None, :] - sites[None, :, :]
        r = np.sqrt(np.sum(R * R, axis=-1))
        same = r == 0
        r_safe = np.where(same, 1.0, r)
        K = _k_tensor(kd * r_safe, R / r_safe[..., None])
        K[same] = 0.0
        total += float(np.real(np.einsum("ja,jlab,lb->", np.conj(P[j0:j1]), K, P)))
    return 4.0 * math.pi * kd ** 4 * total


def c_sca_quadrature(sites, kd, P, n_theta=96, n_phi=192):
    """C_sca by Gauss-Legendre (cos theta) x trapezoid (phi) quadrature."""
    sites = np.asarray(sites, dtype=float)
    P = np.asarray(P, dtype=complex)
    mu, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - mu * mu)
    n = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(mu, np.ones_like(phi))], axis=-1)            # [T, F, 3]
    phase = np.exp(-1j * kd * np.einsum("tfc,jc->tfj", n, sites))
    F = np.einsum("tfj,ja->tfa", phase, P)
    F = F - n * np.sum(n * F, axis=-1, keepdims=True)
    integrand = np.sum(np.abs(F) ** 2, axis=-1)
    total = np.sum(w[:, None] * integrand) * (2.0 * math.pi / n_phi)
    return kd ** 4 * float(total)


def far_field_directions(x, etasca=0.5):
    """(n_theta, n_phi) of the reading of ETASCA in the module docstring."""
    nt = int(math.ceil((3.0 + x) / etasca)) + 1
    return nt, 2 * nt


def far_field(sites, kd, P, khat, n_theta, n_phi):
    """dict(c_sca, g, cos2) by quadrature about khat (see module docstring)."""
    sites = np.asarray(sites, dtype=float)
    P = np.asarray(P, dtype=complex)
    khat = np.asarray(khat, dtype=float)
    khat = khat / np.linalg.norm(khat)
    # an orthonormal frame (e1, e2, khat)
    t = np.array([1.0, 0.0, 0.0]) if abs(khat[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = t - khat * np.dot(t, khat)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(khat, e1)
    mu, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - mu * mu)
    n = (mu[:, None, None] * khat + (st[:, None] * np.cos(phi))[..., None] * e1
         + (st[:, None] * np.sin(phi))[..., None] * e2)                    # [T, F, 3]
    phase = np.exp(-1j * kd * np.einsum("tfc,jc->tfj", n, sites))
    F = np.einsum("tfj,ja->tfa", phase, P)
    F = F - n * np.sum(n * F, axis=-1, keepdims=True)
    inten = np.sum(np.abs(F) ** 2, axis=-1) * w[:, None] * (2.0 * math.pi / n_phi)
    tot = float(np.sum(inten))
    g = float(np.sum(inten * mu[:, None])) / tot
    cos2 = float(np.sum(inten * (mu * mu)[:, None])) / tot
    return dict(c_sca=kd ** 4 * tot, g=g, cos2=cos2)


def efficiencies(n_sites, kd, E_inc, alpha_inv_sites, P, sites=None, exact_sca=False):
    """Dict of Q_ext, Q_abs, Q_sca (= Q_ext - Q_abs unless exact_sca), Q_pha and a_eff."""
    aeff = (3.0 * n_sites / (4.0 * math.pi)) ** (1.0 / 3.0)
    geo = math.pi * aeff * aeff
    ce = c_ext(kd, E_inc, P)
    ca = c_abs(kd, alpha_inv_sites, P)
    cs = c_sca_exact(sites, kd, P) if exact_sca else ce - ca
    return dict(qext=ce / geo, qabs=ca / geo, qsca=cs / geo, qpha=c_pha(kd, E_inc, P) / geo, aeff=aeff)
