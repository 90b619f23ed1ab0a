// The x passes of the FP32 product on FP32 vectors p and q (DDA_MIXED_V32).
#include "passes.hpp"

namespace dda {
template void launch_x_pass<float, c32>(int, const Geometry &, const MatvecArgs &, const PassDims &, hipStream_t);
}  // namespace dda
