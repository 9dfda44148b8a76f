// Network forward (filled in below the solver path).
#include "batch.h"

namespace hp {

hp_status network_alloc(Batch& b) {
  (void)b;
  return HP_OK;
}

}  // namespace hp

extern "C" hp_status hp_infer_factors(hp_batch b, const float* d_weights, const float* d_rho, const float* d_sys,
                                      void* d_factors, int32_t compute) {
  (void)b; (void)d_weights; (void)d_rho; (void)d_sys; (void)d_factors; (void)compute;
  return hp::set_error(HP_E_STATE, "hp_infer_factors: not built yet");
}
