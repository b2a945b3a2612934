// Sparse (CSC) path of libsca.
#include <hip/hip_runtime.h>

#include "sca_internal.h"

using namespace sca;

void sca::launch_colnorm2_csc(sca_problem*, hipStream_t) {}
void sca::launch_round_csc(sca_problem*, const sca_opts*, void*, void*, hipStream_t, uint64_t,
                           const BRParams&) {}
void sca::launch_residual_csc(sca_problem*, const void*, void*, hipStream_t) {}
void sca::launch_probe_csc(sca_problem*, const void*, const BRParams&, hipStream_t) {}

extern "C" sca_status sca_problem_create_csr(sca_problem** out, sca_dtype, int64_t, int64_t,
                                             int64_t, const int64_t*, const int32_t*, const void*,
                                             const void*, double, double, double, const int64_t*,
                                             int64_t, void*) {
  if (out) *out = nullptr;
  return set_error(SCA_EINVAL, "sparse path not available in this build");
}
