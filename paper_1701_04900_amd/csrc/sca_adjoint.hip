// Implicit-differentiation adjoint of libsca.
#include <hip/hip_runtime.h>

#include "sca_internal.h"

using namespace sca;

extern "C" sca_status sca_adjoint(sca_problem* p, const sca_opts*, const void*, const void*, void*,
                                  double*, double, int64_t, void*) {
  (void)p;
  return set_error(SCA_EINVAL, "adjoint not available in this build");
}
