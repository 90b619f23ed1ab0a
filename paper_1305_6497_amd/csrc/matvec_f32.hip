// The five-pass FFT product in FP32 (see passes.hpp).
#include "passes.hpp"

namespace dda {
template void launch_matvec<float>(const Geometry &, const MatvecArgs &, hipStream_t, const hipEvent_t *, int, int);
}  // namespace dda
