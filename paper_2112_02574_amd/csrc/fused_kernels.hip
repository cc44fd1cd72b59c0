// fused_kernels.hip -- the fused one-kernel-per-step design (z-marching).
#include "site_ops.h"

namespace scmc {

bool fused_supported(const StepKey &, const int *) { return false; }

hipError_t launch_fused(const StepKey &, const Member &, const void *, void *,
                        const int *, hipStream_t) {
    return hipErrorInvalidValue;
}

hipError_t launch_batch_fused(const StepKey &, const Member *, const Tile *,
                              int, const void *, void *, const int *, int,
                              hipStream_t) {
    return hipErrorInvalidValue;
}

bool node_fused(const StepKey &, const int *, NodeLaunch *, const Member &) {
    return false;
}

bool node_batch_fused(const StepKey &, const int *, int, NodeLaunch *) {
    return false;
}

}  // namespace scmc
