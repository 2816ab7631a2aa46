// fsc_step_d3e4_f32.hip -- instantiations of the fused step (D3Q19, StencilE4_3D, float).
#include "fsc_step_kernel.h"

namespace fsc {

hipError_t launch_step_d3e4_f32(const StepLaunch &P, hipStream_t s) {
    if (P.tile.tx == 32 && P.tile.ty == 8 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 32, 8, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 32, 8, 1>(P, s);
    if (P.tile.tx == 32 && P.tile.ty == 8 && P.tile.pf == 2)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 32, 8, 2>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 32, 8, 2>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 4 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 64, 4, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 64, 4, 1>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 4 && P.tile.pf == 2)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 64, 4, 2>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 64, 4, 2>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 8 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 64, 8, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 64, 8, 1>(P, s);
    if (P.tile.tx == 32 && P.tile.ty == 16 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 32, 16, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 32, 16, 1>(P, s);
    if (P.tile.tx == 128 && P.tile.ty == 4 && P.tile.pf == 1)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 128, 4, 1>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 128, 4, 1>(P, s);
    // whole 256-wide rows, four per tile (one 16-wave workgroup per CU)
    if (P.tile.tx == 256 && P.tile.ty == 4 && P.tile.pf == 0)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 256, 4, 0>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 256, 4, 0>(P, s);
    // no prefetch (ring of R + 1 planes): fewer registers, more waves per SIMD
    if (P.tile.tx == 128 && P.tile.ty == 4 && P.tile.pf == 0)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 128, 4, 0>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 128, 4, 0>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 8 && P.tile.pf == 0)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 64, 8, 0>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 64, 8, 0>(P, s);
    if (P.tile.tx == 64 && P.tile.ty == 4 && P.tile.pf == 0)
        return P.noise ? launch_one<D3Q19, StencilE4_3D, float, true, 64, 4, 0>(P, s)
                       : launch_one<D3Q19, StencilE4_3D, float, false, 64, 4, 0>(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
