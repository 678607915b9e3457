// Fused FP32 collision kernels (placeholder until written): returning false
// selects the generic pipeline.
#include "collision_common.hpp"

namespace blr {
struct PairPlan;
bool fast_collision_f32(blr_ctx, const DevTables&, const float*, const PairPlan&,
                        const std::vector<int>&, float*) {
  return false;
}
}  // namespace blr
