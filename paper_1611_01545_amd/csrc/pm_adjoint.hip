// Adjoint of the particle-mesh step (placeholder until the adjoint kernels land).
#include "pm_codec.h"

pm_status run_step_vjp(pm_context*, const pm_species*, int, double, float* const*,
                       float* const*, float* const*, float* const*) {
  return PM_ERR_ARG;
}
pm_status run_loss_vjp(pm_context*, const pm_species*, int, const float*, double*,
                       float* const*) {
  return PM_ERR_ARG;
}
