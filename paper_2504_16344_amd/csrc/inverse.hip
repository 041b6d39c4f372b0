// Data-space Hessian assembly and posterior mean (placeholders until the
// float64 Cholesky lands).
#include "p2o_internal.h"

extern "C" {

p2o_status p2o_hessian_assemble(p2o_handle h, double prior_var,
                                const double* noise_var, double* K,
                                void* stream) {
  (void)prior_var; (void)stream;
  if (!h || !noise_var || !K) return P2O_EINVAL;
  return P2O_EUNSUPPORTED;
}

p2o_status p2o_posterior_solve(p2o_handle h, double* K, const double* d,
                               double* m_out, int64_t nrhs, double prior_var,
                               int refine_steps, int64_t* failed_pivot,
                               void* stream) {
  (void)prior_var; (void)refine_steps; (void)failed_pivot; (void)stream;
  if (!h || !K || !d || !m_out || nrhs < 1) return P2O_EINVAL;
  return P2O_EUNSUPPORTED;
}

}  // extern "C"
