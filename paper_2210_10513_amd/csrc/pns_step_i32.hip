// Step kernels for int32_t coefficients with int32_t local fields.
#include "pns_step.h"

namespace pns {

hipError_t launch_steps_i32(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe)
{
    using namespace step;
    PNS_TILE_LIST(PNS_DISPATCH_TILE, int32_t, int32_t)
    PNS_TILE_LIST_WIDE(PNS_DISPATCH_TILE, int32_t, int32_t)
    return hipErrorInvalidConfiguration;
}

}  // namespace pns
