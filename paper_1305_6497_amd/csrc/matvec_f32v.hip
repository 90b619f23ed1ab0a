// The x passes of the FP32 product on FP32 search directions and products
// (DDA_MIXED_V32): both vectors FP32 (COCG; BiCGSTAB's p -> v product), and an
// FP64 input with an FP32 v in the fused update (BiCGSTAB's s -> t product).
#include "passes.hpp"

namespace dda {
extern template void launch_x_pass<float, c64, c64>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                                    hipStream_t);
template void launch_x_pass<float, c32, c32>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                             hipStream_t);
template void launch_x_pass<float, c64, c32>(int, const Geometry &, const MatvecArgs &, const PassDims &,
                                             hipStream_t);
}  // namespace dda
