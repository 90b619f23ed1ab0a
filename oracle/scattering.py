"""Scattering amplitude matrix and Mueller matrix (§26 of the DDSCAT 7.3 guide).

The Lab Frame has x_LF along the incident direction; a scattering direction
(theta_s, phi_s) is n = cos(theta_s) x_LF + sin(theta_s) (cos(phi_s) y_LF +
sin(phi_s) z_LF), with the scattered polarization basis e_1 = theta_hat_s and
e_2 = phi_hat_s = -sin(phi_s) y_LF + cos(phi_s) z_LF (so cos(phi_s) =
phi_hat_s . z_LF and sin(phi_s) = -phi_hat_s . y_LF, as §26 states).

For the solutions P^(l) of the two incident polarizations e_01, e_02
(|E_0| = 1, phase origin at the origin of the site coordinates), the far
field of the dipole array is E_s = k^2 (exp(ikr)/r) sum_j (P_j)_perp
exp(-i k n . r_j) (d = 1), so the matrix f_ml of eq. f_ml_def is

    f_ml = k^3 e_m . F^(l),    F^(l) = sum_j P^(l)_j exp(-i k n . r_j).

The amplitude matrix S_1..S_4 follows from f_ml, the projections
a = e_01* . y_LF, b = e_01* . z_LF, c = e_02* . y_LF, d = e_02* . z_LF and
phi_s by the four relations §26 prints (from eq. fml_rel_S_v4), and the 16
Mueller elements S_ij from S_1..S_4 by the Bohren & Huffman relations it
lists.  P = (S_21^2 + S_31^2)^(1/2) / S_11 is the linear polarization of the
scattered light for unpolarized incident light.
"""

import numpy as np


def directions(theta, phi, lab):
    """Unit vectors (n, theta_hat, phi_hat), each [m, 3] in the site frame.

    ``lab`` = (x_LF, y_LF, z_LF) expressed in the site frame.
    """
    x, y, z = (np.asarray(v, dtype=float) for v in lab)
    t = np.asarray(theta, dtype=float)[:, None]
    p = np.asarray(phi, dtype=float)[:, None]
    n = np.cos(t) * x + np.sin(t) * (np.cos(p) * y + np.sin(p) * z)
    th = -np.sin(t) * x + np.cos(t) * (np.cos(p) * y + np.sin(p) * z)
    ph = -np.sin(p) * y + np.cos(p) * z
    return n, th, ph


def f_matrix(sites, kd, P1, P2, theta, phi, lab):
    """f_ml, complex [m, 2, 2] (index [dir, m, l])."""
    sites = np.asarray(sites, dtype=float)
    n, th, ph = directions(theta, phi, lab)
    phase = np.exp(-1j * kd * (n @ sites.T))                # [m, N]
    out = np.empty((len(n), 2, 2), dtype=complex)
    for l, P in enumerate((P1, P2)):
        F = phase @ np.asarray(P, dtype=complex)             # [m, 3]
        out[:, 0, l] = kd ** 3 * np.sum(th * F, axis=1)
        out[:, 1, l] = kd ** 3 * np.sum(ph * F, axis=1)
    return out


def amplitude_matrix(f, phi, e01, e02, lab):
    """S_1, S_2, S_3, S_4 (complex [m] each) from f_ml by §26."""
    _, y, z = (np.asarray(v, dtype=float) for v in lab)
    e01c = np.conj(np.asarray(e01, dtype=complex))
    e02c = np.conj(np.asarray(e02, dtype=complex))
    a, b = e01c @ y, e01c @ z
    c, d = e02c @ y, e02c @ z
    cs, sn = np.cos(phi), np.sin(phi)
    f11, f12, f21, f22 = f[:, 0, 0], f[:, 0, 1], f[:, 1, 0], f[:, 1, 1]
    S1 = -1j * (f21 * (b * cs - a * sn) + f22 * (d * cs - c * sn))
    S2 = -1j * (f11 * (a * cs + b * sn) + f12 * (c * cs + d * sn))
    S3 = 1j * (f11 * (b * cs - a * sn) + f12 * (d * cs - c * sn))
    S4 = 1j * (f21 * (a * cs + b * sn) + f22 * (c * cs + d * sn))
    return S1, S2, S3, S4


def mueller(S1, S2, S3, S4):
    """The 4 x 4 Mueller matrix, real [m, 4, 4] (S[:, i-1, j-1] = S_ij)."""
    a1, a2, a3, a4 = (np.abs(s) ** 2 for s in (S1, S2, S3, S4))
    M = np.empty(np.shape(S1) + (4, 4))
    M[..., 0, 0] = (a1 + a2 + a3 + a4) / 2
    M[..., 0, 1] = (a2 - a1 + a4 - a3) / 2
    M[..., 0, 2] = np.real(S2 * np.conj(S3) + S1 * np.conj(S4))
    M[..., 0, 3] = np.imag(S2 * np.conj(S3) - S1 * np.conj(S4))
    M[..., 1, 0] = (a2 - a1 + a3 - a4) / 2
    M[..., 1, 1] = (a1 + a2 - a3 - a4) / 2
    M[..., 1, 2] = np.real(S2 * np.conj(S3) - S1 * np.conj(S4))
    M[..., 1, 3] = np.imag(S2 * np.conj(S3) + S1 * np.conj(S4))
    M[..., 2, 0] = np.real(S2 * np.conj(S4) + S1 * np.conj(S3))
    M[..., 2, 1] = np.real(S2 * np.conj(S4) - S1 * np.conj(S3))
    M[..., 2, 2] = np.real(S1 * np.conj(S2) + S3 * np.conj(S4))
    M[..., 2, 3] = np.imag(S2 * np.conj(S1) + S4 * np.conj(S3))
    M[..., 3, 0] = np.imag(S4 * np.conj(S2) + S1 * np.conj(S3))
    M[..., 3, 1] = np.imag(S4 * np.conj(S2) - S1 * np.conj(S3))
    M[..., 3, 2] = np.imag(S1 * np.conj(S2) - S3 * np.conj(S4))
    M[..., 3, 3] = np.real(S1 * np.conj(S2) - S3 * np.conj(S4))
    return M


def polarization(M):
    """(S_21^2 + S_31^2)^(1/2) / S_11 for each direction."""
    return np.sqrt(M[..., 1, 0] ** 2 + M[..., 2, 0] ** 2) / M[..., 0, 0]
