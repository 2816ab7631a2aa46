// fsc_step2_e8.hip -- instantiations of the two-step kernel (D2Q9, StencilE8_2D, float).
#include "fsc_step2_kernel.h"

namespace fsc {

hipError_t launch_step2_e8(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 128)
        return P.noise ? launch_two<StencilE8_2D, float, true, 128>(P, s)
                       : launch_two<StencilE8_2D, float, false, 128>(P, s);
    if (P.tile.tx == 256)
        return P.noise ? launch_two<StencilE8_2D, float, true, 256>(P, s)
                       : launch_two<StencilE8_2D, float, false, 256>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
