// Measured plan choices (see autotune.py): for each pass, padded length and
// precision the radix-plan variant that ran fastest on MI355X (the z-pass:
// plan_variant in fft_lds.hpp; the x passes: rows_plan).  Lengths missing
// here use variant 0, the cost model's plan.
#include "dda_internal.hpp"

namespace dda {
namespace {

struct TunedPlan {
  int pass, L, fp32, variant;
};

constexpr TunedPlan kTuned[] = {
    {-1, 0, 0, 0},                // sentinel
#include "plan_tuned.inc"
};

}  // namespace

int tuned_variant(int pass, int L, bool fp32) {
  const int nvar = pass == kPassZ ? kPlanVariantsHost : kRowPlanVariantsHost;
  for (const TunedPlan &t : kTuned)
    if (t.pass == pass && t.L == L && t.fp32 == (fp32 ? 1 : 0) && t.variant >= 0 && t.variant < nvar)
      return t.variant;
  return 0;
}

}  // namespace dda
