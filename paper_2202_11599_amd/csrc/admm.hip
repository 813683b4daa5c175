// ADMM drivers (Algorithm NysADMM).
#include "internal.h"

extern "C" {

nys_status admm_step(nys_ctx, const nys_problem*, const nys_admm_opts*, nys_factor*,
                     nys_admm_state*, nys_admm_info*) {
  return NYS_ERR_INVALID;
}

nys_status admm_solve(nys_ctx, int, const nys_problem*, const nys_admm_opts*, nys_admm_state*,
                      nys_admm_info*) {
  return NYS_ERR_INVALID;
}

}  // extern "C"
