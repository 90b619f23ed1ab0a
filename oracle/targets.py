"""Occupied lattice sites of built-in target shapes, and the size relations.

Follows the DDSCAT 7.3 user guide:

* §18 "Target Geometry: The Target Frame": a target is a list of occupied
  sites (i, j, k) of a cubic lattice of spacing d (d = 1 here).
* §21 "Target Generation: Isolated Finite Targets": ELLIPSOID, RCTGLPRSM,
  CYLINDER1 and HEX_PRISM, each defined by SHPAR_1..SHPAR_3.
* §2 "Applicability of the DDA": V = N d^3, a_eff = (3V/4pi)^(1/3),
  x = k a_eff.

Reading of the lattice placement (the guide gives the continuous shapes, not
how they are sampled): along an axis of extent S there are n = nearest integer
to S sites at centred positions u = i - (n-1)/2, i = 0..n-1, and a site belongs
to the target when its centre satisfies the shape's inequality, with equality
included.  This reading reproduces every pseudosphere count the guide prints
(N = 304, 17904, 59728 in §2 and the ELLIPSOID example of §21).  When every
SHPAR is an integer the ellipsoid test is evaluated in exact integer
arithmetic, so boundary ties cannot depend on rounding.

Sites are returned as int64 [N, 3] (x, y, z) shifted so that the smallest
occupied index on every axis is 0, sorted in raster order with x fastest
(then y, then z); ``box_of`` gives the tight bounding box.
"""

import math

import numpy as np


def _nsites(s):
    """Number of lattice sites spanning extent s (nearest integer, half up)."""
    return int(math.floor(s + 0.5))


def _centred_axis(n):
    """Twice the centred coordinate, 2u = 2i - (n-1), as integers."""
    return 2 * np.arange(n, dtype=np.int64) - (n - 1)


def _finish(mask):
    """Turn a boolean occupancy mask over the centred grid into sorted sites."""
    ix, iy, iz = np.nonzero(mask)
    sites = np.stack([ix, iy, iz], axis=1).astype(np.int64)
    if sites.shape[0] == 0:
        return sites
    sites -= sites.min(axis=0)
    order = np.lexsort((sites[:, 0], sites[:, 1], sites[:, 2]))
    return sites[order]


def ellipsoid(s1, s2, s3):
    """ELLIPSOID (§21): (x/S1)^2 + (y/S2)^2 + (z/S3)^2 <= 1/4, d = 1.

    A sphere of diameter D is S1 = S2 = S3 = D.
    """
    s = (s1, s2, s3)
    n = [_nsites(v) for v in s]
    t = [_centred_axis(k) for k in n]          # 2u on each axis
    X, Y, Z = np.meshgrid(t[0], t[1], t[2], indexing="ij")
    if all(float(v).is_integer() for v in s):
        a, b, c = (int(v) for v in s)
        # (2u_x/S1)^2 + ... <= 1  times (S1 S2 S3)^2, all integers.
        lhs = X * X * (b * c) ** 2 + Y * Y * (a * c) ** 2 + Z * Z * (a * b) ** 2
        mask = lhs <= (a * b * c) ** 2
    else:
        mask = (X / s1) ** 2 + (Y / s2) ** 2 + (Z / s3) ** 2 <= 1.0
    return _finish(mask)


def sphere(diameter):
    """Sphere = ELLIPSOID with three equal SHPAR (§21)."""
    return ellipsoid(diameter, diameter, diameter)


def rctglprsm(s1, s2, s3):
    """RCTGLPRSM (§21): rectangular solid of S1 x S2 x S3 dipoles."""
    n = [_nsites(v) for v in (s1, s2, s3)]
    mask = np.ones(n, dtype=bool)
    return _finish(mask)


def _axis_perm(axis):
    """Map the shape's own (axial, transverse-1, transverse-2) axes to TF x/y/z."""
    return {1: (0, 1, 2), 2: (1, 2, 0), 3: (2, 0, 1)}[axis]


def _place(mask_local, perm):
    """Place a mask built in (axial, t1, t2) order into TF axes: local axis l -> perm[l]."""
    return np.transpose(mask_local, [perm.index(i) for i in range(3)])


def cylinder1(length, diameter, axis=1):
    """CYLINDER1 (§21): length SHPAR1, diameter SHPAR2, axis along x/y/z (SHPAR3).

    Reading (the guide does not spell out the sampling): n = nearest integer
    of each extent on centred positions; a site is inside when
    (2u_t1)^2 + (2u_t2)^2 <= SHPAR2^2.  The axial extent needs no test.
    """
    na, nd = _nsites(length), _nsites(diameter)
    ta = _centred_axis(na)
    td = _centred_axis(nd)
    A, T1, T2 = np.meshgrid(ta, td, td, indexing="ij")
    if float(diameter).is_integer():
        mask = T1 * T1 + T2 * T2 <= int(diameter) ** 2
    else:
        mask = T1.astype(float) ** 2 + T2.astype(float) ** 2 <= float(diameter) ** 2
    mask = _place(mask, _axis_perm(axis))
    return _finish(mask)


def hex_prism(length, vertex_to_vertex, orient=1):
    """HEX_PRISM (§21): prism length SHPAR1, hexagon vertex-to-vertex SHPAR2.

    Orientation SHPAR3 = 1: prism axis a1 || x_TF, a2 || y_TF normal to one
    rectangular face.  Other orientations permute the axes (2: a2 || z,
    3: a1 || y & a2 || x, 4: a1 || y & a2 || z, 5: a1 || z & a2 || x,
    6: a1 || z & a2 || y).

    Reading of the sampling: the hexagon has circumradius R = SHPAR2/2 and
    apothem h = R*sqrt(3)/2; along a2 (face normal) the extent is 2h, along
    the third axis (through the vertices) it is 2R; n = nearest integer of
    each extent on centred positions; a site is inside when its projection
    on each of the three face normals (at 0, 60 and 120 degrees from a2) has
    magnitude <= h.
    """
    R = 0.5 * float(vertex_to_vertex)
    h = R * math.sqrt(3.0) / 2.0
    na = _nsites(length)
    n2 = _nsites(2.0 * h)
    n3 = _nsites(2.0 * R)
    ta = _centred_axis(na).astype(float) / 2.0
    t2 = _centred_axis(n2).astype(float) / 2.0
    t3 = _centred_axis(n3).astype(float) / 2.0
    A, U, W = np.meshgrid(ta, t2, t3, indexing="ij")
    c60, s60 = 0.5, math.sqrt(3.0) / 2.0
    mask = (np.abs(U) <= h) & (np.abs(c60 * U + s60 * W) <= h) & (np.abs(-c60 * U + s60 * W) <= h)
    # (a1, a2, a3) -> TF axis indices for the six orientations.
    perms = {1: (0, 1, 2), 2: (0, 2, 1), 3: (1, 0, 2), 4: (1, 2, 0), 5: (2, 0, 1), 6: (2, 1, 0)}
    mask = _place(mask, perms[orient])
    return _finish(mask)


def box_of(sites):
    """Tight bounding box (nx, ny, nz) of a site list whose minimum index is 0."""
    return tuple(int(v) + 1 for v in sites.max(axis=0))


def aeff(n_sites):
    """Effective radius in lattice units, a_eff = (3N/4pi)^(1/3) (§2, d = 1)."""
    return (3.0 * n_sites / (4.0 * math.pi)) ** (1.0 / 3.0)


def kd_from_x(x, n_sites):
    """k d from the size parameter x = k a_eff (§2), with d = 1."""
    return x / aeff(n_sites)


def make(shape, shpar):
    """Dispatch on the guide's shape keyword with its SHPAR tuple."""
    s = tuple(shpar)
    if shape == "ELLIPSOID":
        return ellipsoid(*s[:3])
    if shape == "RCTGLPRSM":
        return rctglprsm(*s[:3])
    if shape == "CYLINDER1":
        return cylinder1(s[0], s[1], int(s[2]) if len(s) > 2 else 1)
    if shape == "HEX_PRISM":
        return hex_prism(s[0], s[1], int(s[2]) if len(s) > 2 else 1)
    raise ValueError(f"unknown shape {shape!r}")
