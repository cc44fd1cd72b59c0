// fused_inst.hip -- instantiates the fused-step kernels of one storage format
// and stencil order (SCMC_INST_STORE, SCMC_INST_ORDER, set by the build).
#define SCMC_FUSED_DEFINE
#include "fused_impl.h"

namespace scmc {
template struct FusedOps<SCMC_INST_STORE, SCMC_INST_ORDER>;
}  // namespace scmc
