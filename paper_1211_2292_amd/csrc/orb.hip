// Orthogonal Recursive Bisection order on the device (placeholder until the
// device implementation lands).
#include "internal.h"

namespace nbi {

int orb_order(const void *, int, int, int, int32_t *, hipStream_t)
{
    set_error("nbody_orb_order is not available in this build");
    return NBODY_E_UNSUPPORTED;
}

void orb_release() {}

}  // namespace nbi
