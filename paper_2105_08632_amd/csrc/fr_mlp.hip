// Learned block preconditioner (placeholder until the MLP kernels land).
#include "fr_solver.hpp"

fr_status pc_mlp_create(fr_precond_s* pc) {
  pc->ctx->err = "learned preconditioner not available";
  return FR_E_UNSUPPORTED;
}
fr_status pc_mlp_setup(fr_precond_s*, const void*, double, double) { return FR_E_UNSUPPORTED; }
fr_status pc_mlp_apply(fr_precond_s*, const void*, void*) { return FR_E_UNSUPPORTED; }
void pc_mlp_destroy(fr_precond_s*) {}
