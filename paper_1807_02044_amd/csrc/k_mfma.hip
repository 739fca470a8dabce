// k_mfma.hip - fused TAD path on the matrix cores (not built yet).
#include "fbs_internal.h"

namespace fbs {

bool mfma_supported(const Geom&) { return false; }

hipError_t launch_mfma(const Geom&, const Tables&, const uint8_t*, const uint8_t*, int32_t*,
                       float*, float*, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace fbs
