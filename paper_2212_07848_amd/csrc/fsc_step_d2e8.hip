// fsc_step_d2e8.hip -- instantiations of the fused step for D2Q9 with StencilE8_2D.
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d2e8(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 128 && P.tile.ty == 1) return launch_prec<D2Q9, StencilE8_2D, 128, 1>(P, s);
    if (P.tile.tx == 256 && P.tile.ty == 1) return launch_prec<D2Q9, StencilE8_2D, 256, 1>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 1) return launch_prec<D2Q9, StencilE8_2D, 64, 1>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
