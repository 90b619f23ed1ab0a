// The five-pass FFT product in FP32 (see passes.hpp).  The x passes with FP32
// Krylov vectors are instantiated in matvec_f32v.hip (compiled in parallel).
#include "passes.hpp"

namespace dda {
extern template void launch_x_pass<float, c32, c32>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                                    hipStream_t);
extern template void launch_x_pass<float, c64, c32>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                                    hipStream_t);
template void launch_x_pass<float, c64, c64>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                             hipStream_t);
template void launch_matvec<float>(const Geometry &, const MatvecArgs &, hipStream_t, const hipEvent_t *, int, int);
}  // namespace dda
