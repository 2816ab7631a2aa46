// fsc_internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

#include <vector>

#include "fsc_device.h"

namespace fsc {

// Host-side range around a library call, shown by profilers that collect
// markers (rocprofv3 --marker-trace); without one attached it costs a call.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// Tile shape of the fused step kernel: a TX x TY cross-section (TY = 1 in 2D)
// marching along the slowest axis.
struct TileShape {
    int tx, ty, pf;     // cross-section tile and register prefetch depth (planes)
    int steps = 1;      // time steps per launch: 1, or 2 (two-step kernel, 2D FP32)
};

// Launch of one step over every replica of an ensemble.
struct StepLaunch {
    const RepDesc *reps;       // device
    const int *tile_begin;     // device, [nrep]
    int nrep;
    int total_tiles;
    int parity;                // source buffer index
    const uint64_t *step_base; // device
    uint32_t step_off;
    int D, stencil, precision; // selects the instantiation
    bool noise;
    bool wide;                 // a replica's buffers reach 4 GiB (single-step kernel only)
    TileShape tile;
};

// One launch of the tile's kernel: one step, or two when L.tile.steps == 2
// (then the state goes from buf[parity] at step_base + step_off to
// buf[parity ^ 1] at two steps later).  hipErrorInvalidValue when no
// instantiation matches.
hipError_t launch_step(const StepLaunch &L, hipStream_t s);
// Tile shapes compiled for a lattice/stencil; the first is the default.
int tile_shapes(int D, int stencil, int precision, TileShape *out, int max);

// Adds k to the device step counter (one thread).
hipError_t launch_step_advance(uint64_t *step_base, uint64_t k, hipStream_t s);

// ---------------------------------------------------------------------------
// Measurement kernels (fsc_measure.hip).
// ---------------------------------------------------------------------------
struct Geometry {
    int D, nx, ny, nz;
    int64_t N;
};

// Real density deviation dn(x) (float or double by precision).
hipError_t launch_density_real(const Geometry &g, int precision, const void *buf, void *out,
                               hipStream_t s);
// FP64 state reductions into out[8] (see fsc_stats); `partials` holds
// stats_partials_len() doubles.
size_t stats_partials_len();
hipError_t launch_stats(const Geometry &g, int precision, const void *buf, double rho0,
                        double *partials, double *out, hipStream_t s);

// In-place complex FFT of every line along the contiguous axis of a
// [n2][n1][n0] array, then a rotation to [n0][n2][n1]; after D calls the
// array is back in its original axis order and transformed along every axis.
// `twiddle` holds n0/2 complex values exp(-2 pi i k / n0) (power-of-two n0)
// or n0 values (other n0).  `tmp` is a second complex buffer of equal size.
hipError_t launch_fft_axis(int precision, void *data, void *tmp, const void *twiddle, int n0,
                           int n1, int n2, hipStream_t s);
hipError_t launch_twiddles(int precision, void *tw, int n, hipStream_t s);
size_t twiddle_len(int n);

// Adds |X(k)|^2 / N of one spectrum to the FP64 axis and radial accumulators.
struct BinTargets {
    double *axis_sum, *axis_sq;  // [D][n_axis]
    double *rad_sum, *rad_sq;    // [n_rad] or null
    int n_axis, n_rad;
    // time series (null when disabled): per-sample sum P and sum |k| P, and
    // rows [cap][2 + n_rad] = (step, L, per-shell sums of P) at row *series_n
    double *mom;
    double *series;
    const int *series_n;
    int series_cap;
};
hipError_t launch_bin(const Geometry &g, int precision, const void *spec, const BinTargets &t,
                      hipStream_t s);
// One replica's part of a batched S(k) sample: a device table filled by the
// host.  The sampled density is dn(x) = sum_i f_i(x) - rho0 of the streamed
// state, gathered from the stored post-collision buffer buf[parity].
struct MeasRep {
    const void *buf[2];   // population buffers
    void *cbuf, *ctmp;    // complex work buffers of N elements each
    const void *tw[3];    // twiddles per axis (see launch_twiddles)
    Geometry g;
    BinTargets t;         // accumulators; t.mom == nullptr: no time series
    double invN;
    int *series_n;        // the time series' row counter (t.series_n, writable)
    double *modes;        // mode recorder rows [cap][D][nm][2], or null
    int *modes_n;
    int modes_nm, modes_cap;
};
// kinds of work in one sample; MK_FFT + d and MK_ROT + d for axis pass d
constexpr int MK_DENSITY = 0, MK_FFT = 1, MK_ROT = 4, MK_BIN = 7, MK_MODES = 8, MK_COUNT = 9;
struct MeasPlan {
    int nrep = 0, D = 2;
    size_t esz = 4;          // bytes of one real (set by the caller)
    std::vector<int> pre;    // [MK_COUNT][nrep + 1]: first block of each replica per kind
    size_t shm_fft[3] = {0, 0, 0}, shm_bin = 0;
    bool any_series = false;
};
// Fills the block prefixes and LDS sizes of P from the host copy of the
// replica table; -1 if a side exceeds 8192 or a grid exceeds 2^31 blocks.
int measure_plan(const MeasRep *reps, int nrep, MeasPlan &P);
// One S(k) sample of every replica in P (density, FFT passes, binning, mode
// records, series rows), in at most 4 + 2 D launches.  The sampled state is
// step_base[0] + step_off.
hipError_t launch_measure(const MeasPlan &P, const MeasRep *dev_reps, const int *dev_pre, int precision,
                          int parity, const uint64_t *step_base, uint32_t step_off, hipStream_t s);

// Block means of the density over f x f blocks (2D) into out[(ny/f) x (nx/f)].
hipError_t launch_coarsen(const Geometry &g, int precision, const void *buf, double rho0, int f,
                          float *out, hipStream_t s);
// Real field -> interleaved complex float.
hipError_t launch_field_cplx(const float *f, int n, void *c, hipStream_t s);
// Zeroes `words` 32-bit words of device memory with a fill kernel.
hipError_t launch_zero_words(void *p, int64_t words, hipStream_t s);

// Plain copy of `bytes` (multiple of 16) bytes.
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);

// Device Philox / normals checks.
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                         hipStream_t s);
hipError_t launch_normals(int D, int precision, uint64_t seed, uint32_t replica,
                          const int64_t *node, const int64_t *step, int64_t n, double *out,
                          hipStream_t s);

}  // namespace fsc
