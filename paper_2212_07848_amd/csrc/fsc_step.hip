// fsc_step.hip -- dispatch of the fused step kernel (fsc_step_kernel.h) over
// lattice, stencil, precision, noise and tile shape.
#include "fsc_internal.h"

namespace fsc {

hipError_t launch_step_d2e4_f32(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d2e4_f64(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d2e8_f32(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d2e8_f64(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d3e4_f32(const StepLaunch &P, hipStream_t s);
hipError_t launch_step_d3e4_f64(const StepLaunch &P, hipStream_t s);
hipError_t launch_step2_e4(const StepLaunch &P, hipStream_t s);
hipError_t launch_step2_e8(const StepLaunch &P, hipStream_t s);

__global__ void k_step_advance(uint64_t *step_base, uint64_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step_base[0] += k;
}

hipError_t launch_step_advance(uint64_t *step_base, uint64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step_base, k);
    return hipGetLastError();
}

// Compiled tile shapes {tx, ty, prefetch depth}; the first is the default.
int tile_shapes(int D, int stencil, int precision, TileShape *out, int max) {
    // two-step tilings: the prefetch field selects the LDS schedule (0: one
    // barrier per row, 1: two barriers and a smaller ring)
    static const TileShape f2[] = {{128, 1, 2},    {256, 1, 2},    {64, 1, 2},
                                   {128, 1, 1},    {256, 1, 1},    {128, 1, 0, 2},
                                   {256, 1, 0, 2}, {128, 1, 1, 2}, {256, 1, 1, 2},
                                   {192, 1, 0, 2}, {192, 1, 1, 2}};
    // two-step tilings whose lanes hold the tile's columns and both halos
    // (4R + 2 columns, so the width depends on the stencil), and their
    // single-step partners
    static const TileShape f2e4[] = {{250, 1, 0, 2}, {250, 1, 1, 2}, {250, 1, 1}};
    static const TileShape f2e8[] = {{246, 1, 0, 2}, {246, 1, 1, 2}, {246, 1, 1}};
    static const TileShape d2[] = {{128, 1, 1}};
    static const TileShape f3[] = {{32, 8, 1},  {32, 8, 2}, {64, 4, 1},  {64, 4, 2}, {64, 8, 1},
                                   {32, 16, 1}, {128, 4, 1}, {128, 4, 0}, {64, 8, 0}, {64, 4, 0},
                                   {256, 4, 0}};
    static const TileShape d3[] = {{32, 8, 0}, {32, 8, 1}};
    const TileShape *t = D == 2 ? (precision == 0 ? f2 : d2) : (precision == 0 ? f3 : d3);
    const int n = D == 2 ? (precision == 0 ? 11 : 1) : (precision == 0 ? 11 : 2);
    for (int i = 0; i < n && i < max; ++i) out[i] = t[i];
    if (D == 2 && precision == 0) {
        const TileShape *x = stencil == 8 ? f2e8 : f2e4;
        for (int i = 0; i < 3; ++i)
            if (n + i < max) out[n + i] = x[i];
        return n + 3;
    }
    return n;
}

hipError_t launch_step(const StepLaunch &P, hipStream_t s) {
    const bool f = P.precision == 0;
    if (P.tile.steps == 2) {
        if (P.D != 2 || !f) return hipErrorInvalidValue;
        return P.stencil == 8 ? launch_step2_e8(P, s) : launch_step2_e4(P, s);
    }
    if (P.D == 2 && P.stencil == 4) return f ? launch_step_d2e4_f32(P, s) : launch_step_d2e4_f64(P, s);
    if (P.D == 2 && P.stencil == 8) return f ? launch_step_d2e8_f32(P, s) : launch_step_d2e8_f64(P, s);
    if (P.D == 3 && P.stencil == 4) return f ? launch_step_d3e4_f32(P, s) : launch_step_d3e4_f64(P, s);
    return hipErrorInvalidValue;
}

}  // namespace fsc
