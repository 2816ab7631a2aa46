// fsc_step_d3e4_f64.hip -- instantiations of the fused step (D3Q19, StencilE4_3D, double).
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d3e4_f64(const StepLaunch &P, hipStream_t s) {
    // no prefetch (the default): the register-lean form stays within the 256
    // architectural VGPRs; with one plane of prefetch the noisy form also
    // parks 38 values in accumulation registers
    if (P.tile.tx == 32 && P.tile.ty == 8 && P.tile.pf == 0)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, double, true, 32, 8, 0>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, double, false, 32, 8, 0>(P, s);
    if (P.tile.tx == 32 && P.tile.ty == 8 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, double, true, 32, 8, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, double, false, 32, 8, 1>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
