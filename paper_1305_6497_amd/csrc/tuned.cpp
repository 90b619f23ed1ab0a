// Measured plan choices of the z-pass (see autotune.py): for each padded
// z extent and precision the radix-plan variant (plan_variant in fft_lds.hpp)
// that ran fastest on MI355X.  Lengths missing here use variant 0, the cost
// model's plan.
#include "dda_internal.hpp"

namespace dda {
namespace {

struct TunedPlan {
  int L, fp32, variant;
};

constexpr TunedPlan kTuned[] = {
    {0, 0, 0},                    // sentinel
#include "zpass_tuned.inc"
};

}  // namespace

int tuned_zpass_variant(int L, bool fp32) {
  for (const TunedPlan &t : kTuned)
    if (t.L == L && t.fp32 == (fp32 ? 1 : 0) && t.variant >= 0 && t.variant < kPlanVariantsHost) return t.variant;
  return 0;
}

}  // namespace dda
