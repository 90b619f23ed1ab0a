"""Orientational averaging (§20 of the DDSCAT 7.3 guide).

The average of Q over random orientations is
    <Q> = 1/(8 pi^2) int dbeta int dcos(Theta) int dPhi Q(beta, Theta, Phi),
sampled at Theta uniformly spaced in cos(Theta) and beta, Phi uniformly
spaced, with weights WGTB = 1/NBETA and WGTA for (Theta, Phi): 1/(NTHETA
NPHI) for even NTHETA, Simpson weights for odd NTHETA.

Readings (the guide prints the weights, not the points): beta and Phi take
min + j (max - min)/n, j = 0..n-1 (the periodic trapezoid rule over a full
period); for odd NTHETA the points include both ends of the cos(Theta) range
and the Simpson weights (1, 4, 2, ..., 4, 1) are divided by 3 (NTHETA - 1) so
that they sum to one (the printed (1/3, 4/3, 2/3)/NTHETA sums to
(NTHETA - 1)/NTHETA); for even NTHETA the points are the midpoints of NTHETA
equal intervals (the rule for which equal weights are exact for linear
functions).  NTHETA = 1 takes Theta_min with weight 1.
"""

import numpy as np


def periodic(lo, hi, n):
    x = lo + np.arange(n) * (hi - lo) / n
    return x, np.full(n, 1.0 / n)


def cos_theta(lo, hi, n):
    if n == 1:
        return np.array([lo]), np.array([1.0])
    c0, c1 = np.cos(lo), np.cos(hi)
    if n % 2 == 1:
        u = c0 + (c1 - c0) * np.arange(n) / (n - 1)
        w = np.where(np.arange(n) % 2 == 1, 4.0, 2.0)
        w[0] = w[-1] = 1.0
        return np.arccos(np.clip(u, -1.0, 1.0)), w / (3.0 * (n - 1))
    u = c0 + (c1 - c0) * (np.arange(n) + 0.5) / n
    return np.arccos(np.clip(u, -1.0, 1.0)), np.full(n, 1.0 / n)


def grid(beta, theta, phi):
    """(beta, theta, phi, weight) arrays, beta fastest then phi then theta;
    each argument is a (min, max, count) range in radians."""
    b, wb = periodic(*beta)
    t, wt = cos_theta(*theta)
    p, wp = periodic(*phi)
    T, P, B = np.meshgrid(t, p, b, indexing="ij")
    W = wt[:, None, None] * wp[None, :, None] * wb[None, None, :]
    return B.ravel(), T.ravel(), P.ravel(), W.ravel()


def average(values, weights):
    """sum_i w_i Q_i over the orientations (axis 0)."""
    return np.tensordot(np.asarray(weights, dtype=float), np.asarray(values), axes=(0, 0))
