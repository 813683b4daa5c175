// Randomized Nystrom sketch and its FP64 core (Algorithm RandNysAppx).
#include "internal.h"

extern "C" {

nys_status nys_sketch(nys_ctx, const nys_dense*, const double*, double, const double*, int,
                      nys_dtype, nys_factor*) {
  return NYS_ERR_INVALID;
}

nys_status nys_sketch_adaptive(nys_ctx, const nys_dense*, const double*, double, const double*,
                               int, int, double, double, nys_dtype, nys_factor*) {
  return NYS_ERR_INVALID;
}

}  // extern "C"
