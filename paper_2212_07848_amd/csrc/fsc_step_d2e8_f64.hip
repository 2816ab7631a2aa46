// fsc_step_d2e8_f64.hip -- instantiations of the fused step (D2Q9, StencilE8_2D, double).
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d2e8_f64(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 128 && P.tile.ty == 1 && P.tile.pf == 1)
        return P.noise ? launch_one<D2Q9, StencilE8_2D, double, true, 128, 1, 1>(P, s)
                       : launch_one<D2Q9, StencilE8_2D, double, false, 128, 1, 1>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
