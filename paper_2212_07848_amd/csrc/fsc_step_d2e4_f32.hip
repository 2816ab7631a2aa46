// fsc_step_d2e4_f32.hip -- instantiations of the fused step (D2Q9, StencilE4_2D, float).
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d2e4_f32(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 128 && P.tile.ty == 1 && P.tile.pf == 2)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 128, 1, 2>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 128, 1, 2>(P, s);
    if (P.tile.tx == 256 && P.tile.ty == 1 && P.tile.pf == 2)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 256, 1, 2>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 256, 1, 2>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 1 && P.tile.pf == 2)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 64, 1, 2>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 64, 1, 2>(P, s);
    if (P.tile.tx == 128 && P.tile.ty == 1 && P.tile.pf == 1)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 128, 1, 1>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 128, 1, 1>(P, s);
    if (P.tile.tx == 256 && P.tile.ty == 1 && P.tile.pf == 1)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 256, 1, 1>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 256, 1, 1>(P, s);
    // the single steps of a run on the 192-wide two-step tiling
    if (P.tile.tx == 192 && P.tile.ty == 1 && P.tile.pf == 1)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 192, 1, 1>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 192, 1, 1>(P, s);
    // the single steps of a run on the 250-wide two-step tiling (halos in the tile's lanes)
    if (P.tile.tx == 250 && P.tile.ty == 1 && P.tile.pf == 1)
        return P.noise ? launch_one<D2Q9, StencilE4_2D, float, true, 250, 1, 1>(P, s)
                       : launch_one<D2Q9, StencilE4_2D, float, false, 250, 1, 1>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
