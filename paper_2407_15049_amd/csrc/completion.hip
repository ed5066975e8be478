// Matrix-completion kernels (C = I, sampled-entry constraints).
#include "device.h"
#include "kernels.h"

namespace lrsdp {

int spmm_completion(hipStream_t, const DevCompletion &, int, const void *, int64_t, const double *, void *) {
    return set_error(LRSDP_EUNSUPPORTED, "completion SpMM not available in this build");
}

}  // namespace lrsdp
