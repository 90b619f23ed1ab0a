// Magnetic near field (§29 of the DDSCAT 7.3 guide): B = B_inc + h (*) P on
// the extended box, computed with full (unpruned) FP64 3-D FFTs: it is a
// one-off evaluation after a solve, not part of the iteration.
#pragma once

#include "dda_internal.hpp"

namespace dda {

// In-place unnormalised 3-D FFT of ncomp grids [ncomp][Mz][My][Mx] of the
// geometry g (dir -1 forward, +1 inverse).
void launch_fft3_full64(c64 *data, int ncomp, const Geometry &g, const Twiddles &tx, const Twiddles &ty,
                        const Twiddles &tz, const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int dir,
                        hipStream_t s);

// h = the dipole magnetic-field vector k^2 (e^{ikR}/R)(1 + i/(kR)) n on the
// periodic grid of g, transformed: 3 grids [3][Mz][My][Mx].
void launch_magnetic_kernel(const Geometry &g, double kd, c64 *h, const Twiddles &tx, const Twiddles &ty,
                            const Twiddles &tz, const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz,
                            hipStream_t s);

// full[c][mapM[i]] = P[i][c] for the n sites of one RHS (full zeroed before).
void launch_magnetic_embed(const c64 *P, int64_t n, const int64_t *mapM, c64 *full, int64_t M, hipStream_t s);

// full[:, j] = scale * h[:, j] x full[:, j] at every grid cell.
void launch_magnetic_cross(const c64 *h, c64 *full, int64_t M, double scale, hipStream_t s);

// B at the extended points of one RHS: B_inc + full at grid cell (z, y, x),
// point j = (z Y + y) X + x at site coordinate (x, y, z) - margin.
void launch_magnetic_field(const c64 *full, const Geometry &g, int X, int Y, int64_t ne, const int margin[3],
                           const RhsDev *rhs, double kd, c64 *B, hipStream_t s);

}  // namespace dda
