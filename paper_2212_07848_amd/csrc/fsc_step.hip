// fsc_step.hip -- dispatch of the fused step kernel (fsc_step_kernel.h) over
// lattice, stencil, precision, noise and tile shape.
#include "fsc_internal.h"

namespace fsc {

hipError_t launch_step_d2e4(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d2e8(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d3e4(const StepLaunch &P, hipStream_t s);

__global__ void k_step_advance(uint64_t *step_base, uint64_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step_base[0] += k;
}

hipError_t launch_step_advance(uint64_t *step_base, uint64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step_base, k);
    return hipGetLastError();
}

int tile_shapes(int D, int stencil, TileShape *out, int max) {
    static const TileShape s2[] = {{128, 1}, {256, 1}, {64, 1}};
    static const TileShape s3[] = {{32, 8}, {64, 4}};
    const TileShape *t = D == 2 ? s2 : s3;
    const int n = D == 2 ? 3 : 2;
    (void)stencil;
    for (int i = 0; i < n && i < max; ++i) out[i] = t[i];
    return n;
}

hipError_t launch_step(const StepLaunch &P, hipStream_t s) {
    if (P.D == 2 && P.stencil == 4) return launch_step_d2e4(P, s);
    if (P.D == 2 && P.stencil == 8) return launch_step_d2e8(P, s);
    if (P.D == 3 && P.stencil == 4) return launch_step_d3e4(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
