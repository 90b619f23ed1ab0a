"""The 3N x 3N matrix A of eq. (AP=E) and its product with a polarization P.

§12 "Choice of Iterative Algorithm" states the problem A P = E; the guide
cites Draine (1988) and Draine & Flatau (1994) for A without printing it.
Reading (the free-space dipole field, Gaussian units, e^{-i w t}, d = 1):
for j != l, with R = r_j - r_l, R = |R|, n = R/R,

    A_jl = -G_jl,
    G_jl = (e^{ikR}/R) [ k^2 (I - n n) + ((ikR - 1)/R^2) (I - 3 n n) ],

the field at r_j radiated by a unit dipole at r_l; and A_jj = 1/alpha_j, a
multiple of I, or for the GKDLDR polarizability of §14 a diagonal tensor.
So (A P)_j = alpha_j^{-1} P_j - sum_{l != j} G_jl P_l.

The inverse polarizabilities may be given as one scalar, one per site [N],
or as tensor diagonals, one for all sites [1, 3] or one per site [N, 3].

Two products are given:

* ``direct_matvec``: the sum above written out, O(N^2) (the definition).
* ``fft_matvec``: the same sum as a linear convolution on the lattice,
  evaluated by zero-padded 3-D FFTs (Goodman, Draine & Flatau 1990, cited in
  §1 and used by the FFT options of §13).  Each tensor component
  G_ab(Delta) is laid out on a periodic grid of M_i = 2 N_i points per axis
  at index (Delta mod M_i) for |Delta_i| < N_i, with G(0) = 0 and zero at the
  one unused index M_i/2; then (G*P)_a = IFFT( sum_b FFT(G_ab) FFT(P_b) )
  restricted to the N_x x N_y x N_z box.  (M_i = 2 N_i is the extent the
  method names; any M_i >= 2 N_i - 1 gives the same sum.)
"""

import numpy as np
import scipy.fft as sfft


def alpha_inv_diag(alpha_inv_sites, n):
    """1/alpha as the diagonal of each site's tensor, complex [n, 3].

    A scalar or a 1-D array (one value per site) is a multiple of I; a 2-D
    array [1, 3] or [n, 3] holds tensor diagonals."""
    ai = np.asarray(alpha_inv_sites, dtype=complex)
    if ai.ndim <= 1:
        return np.repeat(np.broadcast_to(ai, (n,))[:, None], 3, axis=1)
    return np.broadcast_to(ai, (n, 3)).copy()


def green_tensor(R, kd):
    """G for an array of offset vectors R[..., 3] (lattice units); R != 0.

    Returns complex128 [..., 3, 3].
    """
    R = np.asarray(R, dtype=float)
    r = np.sqrt(np.sum(R * R, axis=-1))
    n = R / r[..., None]
    nn = n[..., :, None] * n[..., None, :]
    eye = np.eye(3)
    k = kd
    pref = np.exp(1j * k * r) / r
    c1 = (k * k) * pref
    c2 = pref * (1j * k * r - 1.0) / (r * r)
    return c1[..., None, None] * (eye - nn) + c2[..., None, None] * (eye - 3.0 * nn)


def dense_matrix(sites, kd, alpha_inv_sites):
    """A as a dense complex128 [3N, 3N] array; unknown order (site, component)."""
    sites = np.asarray(sites, dtype=float)
    n = sites.shape[0]
    R = sites[:, None, :] - sites[None, :, :]
    off = ~np.eye(n, dtype=bool)
    G = np.zeros((n, n, 3, 3), dtype=complex)
    G[off] = green_tensor(R[off], kd)
    A = -G
    ai = alpha_inv_diag(alpha_inv_sites, n)
    for j in range(n):
        A[j, j] = np.diag(ai[j])
    return A.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def direct_matvec(sites, kd, alpha_inv_sites, P, block=256):
    """(A P)_j by direct summation over all l != j.  P: complex [N, 3]."""
    sites = np.asarray(sites, dtype=float)
    P = np.asarray(P, dtype=complex)
    n = sites.shape[0]
    out = alpha_inv_diag(alpha_inv_sites, n) * P
    for j0 in range(0, n, block):
        j1 = min(n, j0 + block)
        R = sites[j0:j1, None, :] - sites[None, :, :]
        same = np.zeros((j1 - j0, n), dtype=bool)
        same[np.arange(j1 - j0), np.arange(j0, j1)] = True
        R[same] = 1.0                      # placeholder, zeroed below
        G = green_tensor(R, kd)
        G[same] = 0.0
        out[j0:j1] -= np.einsum("jlab,lb->ja", G, P)
    return out


def sampled_direct_field(sites, kd, P, rows):
    """sum_{l != j} G_jl P_l for the listed sites j only (for spot checks)."""
    sites = np.asarray(sites, dtype=float)
    P = np.asarray(P, dtype=complex)
    res = np.zeros((len(rows), 3), dtype=complex)
    for i, j in enumerate(rows):
        R = sites[j][None, :] - sites
        mask = np.ones(sites.shape[0], dtype=bool)
        mask[j] = False
        G = green_tensor(R[mask], kd)
        res[i] = np.einsum("lab,lb->a", G, P[mask])
    return res


# Unique components of the symmetric tensor, in the order used throughout.
COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def green_grid(box, kd, M=None):
    """The six components G_ab on the periodic M grid, complex128 [6, Mx, My, Mz]."""
    nx, ny, nz = box
    if M is None:
        M = (2 * nx, 2 * ny, 2 * nz)
    axes = []
    for ni, mi in zip(box, M):
        idx = np.arange(mi)
        delta = np.where(idx < ni, idx, idx - mi).astype(float)
        valid = (idx < ni) | (idx > mi - ni)
        axes.append((delta, valid))
    (dx, vx), (dy, vy), (dz, vz) = axes
    DX, DY, DZ = np.meshgrid(dx, dy, dz, indexing="ij")
    valid = vx[:, None, None] & vy[None, :, None] & vz[None, None, :]
    valid[0, 0, 0] = False
    R = np.stack([DX, DY, DZ], axis=-1)
    G = np.zeros(tuple(M) + (3, 3), dtype=complex)
    G[valid] = green_tensor(R[valid], kd)
    return np.stack([G[..., a, b] for a, b in COMPONENTS])


class FFTOperator:
    """A P by zero-padded FFT convolution (see module docstring)."""

    def __init__(self, sites, kd, alpha_inv_sites, workers=None):
        self.sites = np.asarray(sites, dtype=np.int64)
        self.box = tuple(int(v) + 1 for v in self.sites.max(axis=0))
        self.M = tuple(2 * b for b in self.box)
        self.kd = kd
        self.n = self.sites.shape[0]
        self.alpha_inv = alpha_inv_diag(alpha_inv_sites, self.n)
        self.workers = workers if workers is not None else -1
        G = green_grid(self.box, kd, self.M)
        self.Ghat = sfft.fftn(G, axes=(1, 2, 3), workers=self.workers)

    def field(self, P):
        """sum_{l != j} G_jl P_l at every site j, complex [N, 3]."""
        P = np.asarray(P, dtype=complex)
        ix, iy, iz = self.sites.T
        grid = np.zeros((3,) + self.M, dtype=complex)
        for a in range(3):
            grid[a][ix, iy, iz] = P[:, a]
        Phat = sfft.fftn(grid, axes=(1, 2, 3), workers=self.workers)
        out = np.empty((self.n, 3), dtype=complex)
        for a in range(3):
            acc = np.zeros(self.M, dtype=complex)
            for c, (p, q) in enumerate(COMPONENTS):
                if p == a:
                    acc += self.Ghat[c] * Phat[q]
                elif q == a:
                    acc += self.Ghat[c] * Phat[p]
            conv = sfft.ifftn(acc, workers=self.workers)
            out[:, a] = conv[ix, iy, iz]
        return out

    def matvec(self, P):
        P = np.asarray(P, dtype=complex)
        return self.alpha_inv * P - self.field(P)
