// Step kernels for float coefficients with double local fields.
#include "pns_step.h"

namespace pns {

hipError_t launch_steps_f32(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe)
{
    using namespace step;
    PNS_TILE_LIST(PNS_DISPATCH_TILE, float, double)
    return hipErrorInvalidConfiguration;
}

}  // namespace pns
