"""Near fields: E (and B) at lattice points in and around the target (§29 of
the DDSCAT 7.3 guide) and along a line (§30, the post-processor).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

For a solved polarization P the field at a lattice point q, the dipole at q
itself excluded, is (d = 1, the Green tensor of ``interaction``)

    E(q) = E_inc(q) + sum_{l : r_l != q} G(r_q - r_l) P_l,

so at an occupied site E = P / alpha, the field that polarizes that dipole.
The guide calls the stored field macroscopic and relates the two inside a
material of dielectric function eps by E_macro = 3 / (eps + 2) E_micro
(eq. macro_vs_micro); in vacuum they are equal.  Its printed Au-sphere line
(§30) agrees with E above at every point, inside the sphere too, and not with
the converted field (reading: E is the lattice field, the conversion is an
option, ``macroscopic``).  Points between lattice points are interpolated
trilinearly from the eight surrounding lattice points (reading: the guide
does not name the scheme; nearest-point values miss the printed line by up to
0.1 outside the target, trilinear values agree to 6e-4).
"""

import numpy as np

from .interaction import green_tensor


def lattice_field(sites, kd, P, points, khat, e, origin=(0.0, 0.0, 0.0)):
    """E_inc + E_sca at integer lattice points, complex128 [len(points), 3].

    ``sites`` and ``points`` are integer lattice coordinates; ``P`` is
    [N, 3]; the incident phase is kd khat . (r - origin).  Direct sum, the
    definition above.
    """
    sites = np.asarray(sites, dtype=np.int64)
    points = np.asarray(points, dtype=np.int64)
    P = np.asarray(P, dtype=complex)
    out = np.empty((len(points), 3), dtype=complex)
    block = max(1, 500_000 // max(1, len(sites)))            # bounded temporaries
    for i0 in range(0, len(points), block):
        q = points[i0:i0 + block]
        R = (q[:, None, :] - sites[None, :, :]).astype(float)      # [b, N, 3]
        self_term = np.all(R == 0.0, axis=-1)
        R[self_term] = 1.0                                         # placeholder, zeroed below
        G = green_tensor(R, kd)
        G[self_term] = 0.0
        out[i0:i0 + block] = np.einsum("qnab,nb->qa", G, P)
    r = points.astype(float) - np.asarray(origin, dtype=float)[None, :]
    phase = np.exp(1j * kd * (r @ np.asarray(khat, dtype=float)))
    return out + phase[:, None] * np.asarray(e, dtype=complex)[None, :]


def macroscopic(E, points, sites, eps_sites):
    """3 / (eps + 2) E at the points that are occupied sites, E elsewhere."""
    index = {tuple(s): j for j, s in enumerate(np.asarray(sites, dtype=np.int64))}
    eps = np.broadcast_to(np.asarray(eps_sites, dtype=complex), (len(index),))
    f = np.array([3.0 / (eps[index[tuple(p)]] + 2.0) if tuple(p) in index else 1.0
                  for p in np.asarray(points, dtype=np.int64)])
    return E * f[:, None]


def trilinear_corners(positions):
    """For real positions [n, 3] the 8 corner lattice points [n, 8, 3] and weights [n, 8]."""
    x = np.asarray(positions, dtype=float)
    i0 = np.floor(x).astype(np.int64)
    w = x - i0
    corners, weights = [], []
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                corners.append(i0 + np.array([dx, dy, dz]))
                weights.append((w[:, 0] if dx else 1 - w[:, 0]) * (w[:, 1] if dy else 1 - w[:, 1])
                               * (w[:, 2] if dz else 1 - w[:, 2]))
    return np.stack(corners, axis=1), np.stack(weights, axis=1)


def field_on_line(field_at, positions):
    """Trilinear interpolation: ``field_at(points [m, 3]) -> [m, 3]`` gives the
    lattice field; returns [n, 3] at the real positions."""
    corners, weights = trilinear_corners(positions)
    flat = corners.reshape(-1, 3)
    uniq, inv = np.unique(flat, axis=0, return_inverse=True)
    vals = field_at(uniq)[inv.ravel()].reshape(corners.shape[0], 8, 3)
    return np.einsum("nk,nka->na", weights, vals)


def magnetic_field(sites, kd, P, points, khat, e, origin=(0.0, 0.0, 0.0)):
    """B_inc + B_sca at real-valued points, complex128 [len(points), 3].

    §29 stores, with E, the magnetic field B_sca of all the oscillating dipoles
    except one sitting at the point, and the incident B_inc (nonmagnetic
    material: B is both the micro- and the macroscopic field).  In the units of
    ``interaction`` (Gaussian, time factor exp(-i omega t), d = 1) the field of
    a point dipole p at distance R along the unit vector n (source to point) is
    the textbook one,

        B = k^2 (exp(ikR) / R) (1 - 1 / (ikR)) n x p,

    and the plane wave E_inc = e exp(ik khat . r) carries B_inc = khat x E_inc.
    Direct sum over the dipoles.
    """
    sites = np.asarray(sites, dtype=float)
    points = np.asarray(points, dtype=float)
    P = np.asarray(P, dtype=complex)
    out = np.empty((len(points), 3), dtype=complex)
    block = max(1, 500_000 // max(1, len(sites)))
    for i0 in range(0, len(points), block):
        q = points[i0:i0 + block]
        R = q[:, None, :] - sites[None, :, :]                      # [b, N, 3]
        r = np.sqrt(np.sum(R * R, axis=-1))
        self_term = r == 0.0
        r = np.where(self_term, 1.0, r)
        n = R / r[..., None]
        f = kd * kd * np.exp(1j * kd * r) / r * (1.0 - 1.0 / (1j * kd * r))
        f = np.where(self_term, 0.0, f)
        out[i0:i0 + block] = np.sum(f[..., None] * np.cross(n, P[None, :, :]), axis=1)
    rr = points - np.asarray(origin, dtype=float)[None, :]
    kh = np.asarray(khat, dtype=float)
    phase = np.exp(1j * kd * (rr @ kh))
    binc = np.cross(kh, np.asarray(e, dtype=complex))
    return out + phase[:, None] * binc[None, :]
