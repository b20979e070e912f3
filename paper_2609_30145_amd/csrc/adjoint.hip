// Reverse pass of the forward model (exact gradient of logL with respect to theta).
#include "kernels.h"
#include "runtime.h"

namespace sps {

sps_status run_adjoint(const sps_library *L, sps_obs *o, const double *theta, int B, int prec, double *grad,
                       hipStream_t s) {
  (void)L; (void)o; (void)theta; (void)B; (void)prec; (void)grad; (void)s;
  return fail(SPS_E_INVAL, "gradient pass not built yet");
}

}  // namespace sps
