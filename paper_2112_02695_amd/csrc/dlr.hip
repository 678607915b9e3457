// Low-rank step: not written yet; the entry points report BLR_ERR_UNSUPPORTED.
#include "internal.hpp"

extern "C" {
blr_status blr_state_from_full(blr_ctx ctx, const blr_problem*, const double*, int32_t, blr_state*) {
  if (ctx) ctx->err = "blr_state_from_full: not built";
  return BLR_ERR_UNSUPPORTED;
}
blr_status blr_dlr_step(blr_ctx ctx, const blr_problem*, blr_state*, const blr_step_params*,
                        blr_step_info*) {
  if (ctx) ctx->err = "blr_dlr_step: not built";
  return BLR_ERR_UNSUPPORTED;
}
blr_status blr_steady_solve(blr_ctx ctx, const blr_problem*, blr_state*, const blr_solve_params*,
                            blr_solve_info*) {
  if (ctx) ctx->err = "blr_steady_solve: not built";
  return BLR_ERR_UNSUPPORTED;
}
}
