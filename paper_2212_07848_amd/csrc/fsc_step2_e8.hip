// fsc_step2_e8.hip -- instantiations of the two-step kernel (D2Q9, StencilE8_2D, float).
#include "fsc_step2_kernel.h"

namespace fsc {

hipError_t launch_step2_e8(const StepLaunch &P, hipStream_t s) {
    // the prefetch field selects the LDS schedule: 0 one barrier per row
    // (4-row f(t+1) ring), 1 two barriers per row (3-row ring, less LDS)
    if (P.tile.pf != 0 && P.tile.pf != 1) return hipErrorInvalidValue;
    const bool two = P.tile.pf == 1;
    if (P.tile.tx == 128)
        return P.noise ? (two ? launch_two<StencilE8_2D, float, true, 128, 2>(P, s)
                              : launch_two<StencilE8_2D, float, true, 128, 1>(P, s))
                       : (two ? launch_two<StencilE8_2D, float, false, 128, 2>(P, s)
                              : launch_two<StencilE8_2D, float, false, 128, 1>(P, s));
    if (P.tile.tx == 192)
        return P.noise ? (two ? launch_two<StencilE8_2D, float, true, 192, 2>(P, s)
                              : launch_two<StencilE8_2D, float, true, 192, 1>(P, s))
                       : (two ? launch_two<StencilE8_2D, float, false, 192, 2>(P, s)
                              : launch_two<StencilE8_2D, float, false, 192, 1>(P, s));
    if (P.tile.tx == 256)
        return P.noise ? (two ? launch_two<StencilE8_2D, float, true, 256, 2>(P, s)
                              : launch_two<StencilE8_2D, float, true, 256, 1>(P, s))
                       : (two ? launch_two<StencilE8_2D, float, false, 256, 2>(P, s)
                              : launch_two<StencilE8_2D, float, false, 256, 1>(P, s));
    // tile columns and their halos in the same lanes: 246 output columns per 246 + 4R + 2 = 256 lanes
    if (P.tile.tx == 246)
        return P.noise ? (two ? launch_two<StencilE8_2D, float, true, 246, 2, true>(P, s)
                              : launch_two<StencilE8_2D, float, true, 246, 1, true>(P, s))
                       : (two ? launch_two<StencilE8_2D, float, false, 246, 2, true>(P, s)
                              : launch_two<StencilE8_2D, float, false, 246, 1, true>(P, s));
    return hipErrorInvalidValue;
}

}  // namespace fsc
