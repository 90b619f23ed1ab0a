"""FP64 CPU oracle for the discrete dipole approximation (DDA) solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
statement of what the GPU path computes.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product library
and its Python binding never do, and they share no code with it (the only
common module is ``inputs``, which draws seeded random workloads and holds no
DDA arithmetic).

Contents, each following the passage of the DDSCAT 7.3 user guide
(Draine & Flatau 2013) it cites:

* ``targets``        -- occupied lattice sites of the built-in shapes (§21),
                        effective radius and size parameter (§2).
* ``polarizability`` -- Clausius-Mossotti, lattice-dispersion-relation and
                        filtered-coupled-dipole polarizabilities (§14).
* ``incident``       -- orientation algebra (§19), polarization states (§24),
                        incident field at the dipoles (§12, eq. AP=E).
* ``interaction``    -- the 3N x 3N matrix A of eq. (AP=E): dense build,
                        direct-sum product, FFT-convolution product (§13).
* ``solvers``        -- dense LU, BiCGSTAB, BiCGstab(l), COCG and QMR (§12).
* ``cross_sections`` -- C_ext, C_abs, exact C_sca and the efficiencies
                        Q = C / (pi a_eff^2) (§3.1).
* ``mie``            -- Mie-theory efficiencies of a homogeneous sphere, the
                        kd -> 0 limit the DDA must approach (§2).
* ``near_field``     -- E at lattice points in and near the target and along
                        a line (§29, §30).
* ``scattering``     -- amplitude matrix f_ml, S_1..S_4 and the Mueller
                        matrix S_ij in Lab-Frame directions (§26).
* ``orientation``    -- orientation sampling and weights for averages (§20).

Everything is complex128 / float64.  Formulas the guide cites but does not
print (the dipole field tensor, the LDR coefficients, the cross-section sums,
BiCGSTAB) are written out from the cited physics; every such reading is named
in the docstring where it is used.
"""

from . import targets, polarizability, incident, interaction, solvers, cross_sections, mie, near_field, scattering, orientation  # noqa: F401
