// fsc_step_d3e4.hip -- instantiations of the fused step for D3Q19 with StencilE4_3D.
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d3e4(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 32 && P.tile.ty == 8) return launch_prec<D3Q19, StencilE4_3D, 32, 8>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 4) return launch_prec<D3Q19, StencilE4_3D, 64, 4>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
