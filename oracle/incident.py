"""Incident wave: orientation algebra, polarization states, field at the dipoles.

* §19 "Target Orientation": the angles (beta, Theta, Phi) fix the target
  axes a1, a2, a3 in the Lab Frame; equivalently the Lab-Frame unit vectors
  x_LF (propagation), y_LF, z_LF are written in the (a1, a2, a3) basis.
  This module uses the second set of relations, which directly give the
  incident direction and polarization in the Target Frame.
* §19 / §24 "Incident Polarization State": e01 lies in the y_LF, z_LF plane
  and is normalised; the orthogonal state is e02 = x_LF x conj(e01).
* §12, eq. (AP=E): E is the incident field at the N sites,
  E_j = e exp(i k khat . r_j) with |E_0| = 1 and r_j the site position in
  lattice units (d = 1).
"""

import numpy as np


def lab_axes_in_target_basis(beta, theta, phi):
    """x_LF, y_LF, z_LF as components along (a1, a2, a3)  (§19)."""
    cb, sb = np.cos(beta), np.sin(beta)
    ct, st = np.cos(theta), np.sin(theta)
    cp, sp = np.cos(phi), np.sin(phi)
    x_lf = np.array([ct, -st * cb, st * sb])
    y_lf = np.array([st * cp, ct * cb * cp - sb * sp, -(ct * sb * cp + cb * sp)])
    z_lf = np.array([st * sp, ct * cb * sp + sb * cp, -(ct * sb * sp - cb * cp)])
    return x_lf, y_lf, z_lf


def target_axes_tf(a1=(1.0, 0.0, 0.0), a2=(0.0, 1.0, 0.0)):
    """Target axes a1, a2, a3 = a1 x a2 as Target-Frame vectors (§18/§19)."""
    a1 = np.asarray(a1, float)
    a2 = np.asarray(a2, float)
    return np.stack([a1, a2, np.cross(a1, a2)])


def polarization_pair(e01_lf):
    """Normalised e01 and e02 = x_LF x conj(e01), both in Lab-Frame components."""
    e01 = np.asarray(e01_lf, dtype=complex)
    if abs(e01[0]) > 0:
        raise ValueError("e01 must be transverse to x_LF")
    e01 = e01 / np.sqrt(np.vdot(e01, e01).real)
    xhat = np.array([1.0, 0.0, 0.0])
    e02 = np.cross(xhat, np.conj(e01))
    return e01, e02


def incident_in_tf(beta, theta, phi, e_lf, a1=(1.0, 0.0, 0.0), a2=(0.0, 1.0, 0.0)):
    """Propagation direction khat and polarization e in the Target Frame.

    e_lf gives the (complex) polarization in Lab-Frame components (x, y, z);
    its x component must vanish.
    """
    x_lf, y_lf, z_lf = lab_axes_in_target_basis(beta, theta, phi)
    A = target_axes_tf(a1, a2)          # rows: a1, a2, a3 in TF
    to_tf = lambda v: v @ A             # sum_i v_i a_i
    khat = to_tf(x_lf)
    e_lf = np.asarray(e_lf, dtype=complex)
    e = e_lf[0] * to_tf(x_lf) + e_lf[1] * to_tf(y_lf) + e_lf[2] * to_tf(z_lf)
    return khat, e


def incident_field(sites, kd, khat, e):
    """E_j = e exp(i kd khat . r_j), complex128 [N, 3]  (eq. AP=E, |E0| = 1)."""
    r = np.asarray(sites, dtype=float)
    phase = np.exp(1j * kd * (r @ np.asarray(khat, float)))
    return phase[:, None] * np.asarray(e, dtype=complex)[None, :]
