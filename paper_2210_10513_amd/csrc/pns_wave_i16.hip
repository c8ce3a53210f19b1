// Window kernels of one, two or four waves per chain for int16_t
// coefficients with int32_t fields.
#include "pns_wave.h"

namespace pns {

hipError_t launch_waves_i16(bool instr, int block, int groups, int grid, hipStream_t st, const StepArgs& a,
                            bool probe)
{
    PNS_WAVE_TILE_LIST(PNS_WAVE_DISPATCH_TILE, int16_t)
    return hipErrorInvalidConfiguration;
}

}  // namespace pns
