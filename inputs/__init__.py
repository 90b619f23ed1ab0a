"""Seeded synthetic workloads shared by the oracle side and the GPU side.

This module only describes workloads and draws random numbers.  It holds no
arithmetic of the dipole method itself (no site rule, no polarizability, no
field or cross section): each side turns these descriptions into sites,
fields and results with its own code.

Workloads stand in for the guide's example calculations; there is no public
dataset for this method.  Shapes use the guide's keywords and SHPAR
conventions (§21 of the DDSCAT 7.3 user guide).
"""

import math

import numpy as np

# Named single-target workloads.  ``x`` is the size parameter k a_eff; the
# number of dipoles N (hence kd = x / a_eff) follows from the site rule.
WORKLOADS = {
    # FP64 single solve: pseudosphere of diameter 20 (radius 10) in a 20^3 box.
    "sphere_d20": dict(shape="ELLIPSOID", shpar=(20, 20, 20), m=complex(1.33, 0.01), x=1.0,
                       polarizations=2, orientations=1, precision="fp64"),
    # Mixed-precision single solve: 64^3 block, FFT grid 128^3.
    "block_64": dict(shape="RCTGLPRSM", shpar=(64, 64, 64), m=complex(1.5, 0.1), x=10.0,
                     polarizations=1, orientations=1, precision="mixed"),
    # Batched multi-RHS: ellipsoid with semi-axes 48 x 32 x 24.
    "ellipsoid_96x64x48": dict(shape="ELLIPSOID", shpar=(96, 64, 48), m=complex(1.7, 0.05), x=8.0,
                               polarizations=2, orientations=32, precision="mixed"),
    # Large single target: sphere of diameter 133.
    "sphere_d133": dict(shape="ELLIPSOID", shpar=(133, 133, 133), m=complex(1.33, 0.001), x=25.0,
                        polarizations=2, orientations=1, precision="mixed"),
    # The guide's worked example (§8 and the .avg appendix): 16 x 32 x 32 Au block.
    "au_block_16x32x32": dict(shape="RCTGLPRSM", shpar=(16, 32, 32), m=complex(0.9656, 1.8628),
                              x=3.093665, polarizations=2, orientations=1, precision="fp64"),
}

ORIENTATION_SEED = 1305
SERVING_SEED = 4242


def orientation_angles(n, seed=ORIENTATION_SEED):
    """n orientations uniform on SO(3): beta, phi ~ U[0, 2pi), cos(theta) ~ U[-1, 1].

    Returns float64 arrays (beta, theta, phi) drawn from NumPy's PCG64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = rng.uniform(0.0, 2.0 * math.pi, n)
    cos_theta = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    return beta, np.arccos(cos_theta), phi


def random_polarization(n_sites, n_rhs=1, seed=0):
    """Random complex128 vectors [n_rhs, n_sites, 3] with unit-variance parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((n_rhs, n_sites, 3))
    im = rng.standard_normal((n_rhs, n_sites, 3))
    return re + 1j * im


SERVING_SHAPES = ("ELLIPSOID_SPHERE", "CYLINDER1", "HEX_PRISM", "ELLIPSOID")


def serving_requests(n=1000, seed=SERVING_SEED, rate=1.0, accept=None,
                     extent=(16, 96), re_m=(1.1, 2.5), im_m=(0.0, 0.5), x=(1.0, 15.0)):
    """Poisson-arrival request stream of mixed targets.

    Each request: shape uniform over sphere / finite cylinder / hexagonal
    prism / ellipsoid; extents uniform integers in ``extent`` per free axis;
    Re m, Im m and x uniform.  ``accept(req) -> bool`` lets the caller reject a
    draw (e.g. one outside the method's validity range); a rejected draw is
    redrawn from the same stream and counted in ``req['redraws']``.
    Arrival times are cumulative Exp(rate) gaps (seconds).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    lo, hi = extent
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        redraws = 0
        while True:
            kind = SERVING_SHAPES[int(rng.integers(0, 4))]
            if kind == "ELLIPSOID_SPHERE":
                d = int(rng.integers(lo, hi + 1))
                shape, shpar = "ELLIPSOID", (d, d, d)
            elif kind == "CYLINDER1":
                shape, shpar = "CYLINDER1", (int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1)), 1)
            elif kind == "HEX_PRISM":
                shape, shpar = "HEX_PRISM", (int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1)), 1)
            else:
                shape, shpar = "ELLIPSOID", tuple(int(v) for v in rng.integers(lo, hi + 1, 3))
            m = complex(rng.uniform(*re_m), rng.uniform(*im_m))
            xs = float(rng.uniform(*x))
            req = dict(id=i, arrival=t, shape=shape, shpar=shpar, m=m, x=xs, redraws=redraws)
            if accept is None or accept(req):
                break
            redraws += 1
        out.append(req)
    return out
