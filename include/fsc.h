/*
 * fsc.h -- C ABI of the MI355X (gfx950) fluctuating Shan-Chen lattice
 * Boltzmann library.
 *
 * Method: Lulli, Biferale, Falcucci, Sbragaglia, Yang, Shan, "Metastable and
 * Unstable Dynamics in multi-phase lattice Boltzmann", arXiv:2212.07848.
 *   - the fluctuating lattice Boltzmann equation, Eq. (12):
 *       f_i(x + c_i, t + 1) - f_i(x, t) = Omega_i + F_i + eta_i
 *     with Omega a relaxation collision, F_i the Guo forcing of the Shan-Chen
 *     force and eta_i Gaussian noise whose covariance is diagonal in moment
 *     space and zero on the conserved moments (text following Eq. 16);
 *   - the Shan-Chen force, Eq. (1): F(x) = G psi(x) sum_a w(|e_a|^2) psi(x+e_a) e_a,
 *     with psi = exp(-1/n) and weights normalised to sum_a w e_ax^2 = 1, so that
 *     the bulk pressure is Eq. (2): p = n T - (G/2) psi^2, T = c_s^2 = 1/3;
 *   - the structure factor S(k) = <|dn(k)|^2> measured against Eq. (16).
 *
 * Conventions shared by every call:
 *   - Every call returns an int: FSC_OK (0) or a negative FSC_E_* code; no
 *     exception crosses the ABI.  fsc_last_error() gives a message for the
 *     last failure on a context; fsc_strerror() names a code.
 *   - Lattices are periodic.  D = 2 uses D2Q9 (nz = 1), D = 3 uses D3Q19.
 *   - Population order (the index i of every f array):
 *       D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *       D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *              (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *              (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *   - Host population arrays are double, layout f[i][z][y][x] (x fastest),
 *     Q * nx * ny * nz values, holding the populations right after streaming
 *     at the context's current time step.  Node index = x + nx*(y + ny*z).
 *   - Host buffers are owned by the caller and only read/written during the
 *     call.  Device buffers are owned by the library unless passed in through
 *     fsc_create_external (then the caller keeps ownership and must keep them
 *     alive until fsc_destroy).
 *   - All device work is enqueued on the hipStream_t given at creation.  A
 *     lattice or ensemble created with NULL makes a stream of its own (its
 *     step chunks are captured into HIP graphs, which the null stream cannot
 *     hold); the surrogate and the field functions take NULL as the device's
 *     default stream.  Calls that return host data synchronise the stream.
 *     A context is not thread safe; distinct contexts are independent.
 */
#ifndef FSC_H
#define FSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSC_OK 0
#define FSC_E_INVAL (-1)    /* invalid argument or parameter combination */
#define FSC_E_HIP (-2)      /* a HIP runtime call failed */
#define FSC_E_OOM (-3)      /* device or host allocation failed */
#define FSC_E_DIVERGED (-4) /* non-finite or non-positive density detected */
#define FSC_E_STATE (-5)    /* call not valid in the current state */
#define FSC_E_NOTSUP (-6)   /* combination not supported by the library */
#define FSC_E_IO (-7)       /* checkpoint file missing, unreadable, truncated or corrupt */
#define FSC_E_RANGE (-8)    /* input larger than a fixed-size library buffer allows */

#define FSC_E4 4 /* 2D: |e|^2 in {1,2} (8 neighbours); 3D: {1,2} (18) */
#define FSC_E8 8 /* 2D only: |e|^2 in {1,2,4,5,8} (24 neighbours, 5x5 block) */

#define FSC_FP32_SHIFTED 0 /* populations stored as float deviations f_i - w_i rho0 */
#define FSC_FP64 1         /* populations stored as double deviations f_i - w_i rho0 */

#define FSC_SK_AXIS 0   /* bins [D][n/2 + 1]: modes +-m along each lattice axis */
#define FSC_SK_RADIAL 1 /* bins [nb]: shells b = round(|m|), equal sides only */

/*
 * Run parameters.  Layout is fixed: 6 x int32, 7 x double, uint64, 2 x uint32
 * (96 bytes, natural alignment).
 *   D, nx, ny, nz  lattice dimension and sides (nz = 1 when D = 2); sides >= 1
 *   stencil        FSC_E4 or FSC_E8 (interaction set of Eq. 1)
 *   precision      FSC_FP32_SHIFTED or FSC_FP64
 *   T_hat          reduced temperature T/T_c; used when G is NaN:
 *                  G = e^2 / (3 T_hat) (critical point of Eq. 3-4 with b = 1)
 *   G              coupling of Eq. (1), G > 0 attractive; NaN = from T_hat
 *   rho0           homogeneous initial density n0 (> 0), also the storage shift
 *   lambda_bulk    relaxation rate (1/tau) of the bulk (trace) moment
 *   lambda_shear   relaxation rate of the deviatoric second moments
 *   lambda_ghost   relaxation rate of the higher (kinetic) moments
 *                  all three in (0, 2); all equal 1 is BGK with tau = 1
 *   kBT            fluctuation energy k_B theta in lattice units (>= 0); 0 = no noise
 *   seed, replica  key of the counter-based noise generator (see fsc_normals)
 */
typedef struct fsc_params {
    int32_t D, nx, ny, nz;
    int32_t stencil, precision;
    double T_hat, G, rho0;
    double lambda_bulk, lambda_shear, lambda_ghost;
    double kBT;
    uint64_t seed;
    uint32_t replica, reserved;
} fsc_params;

typedef struct fsc_ctx fsc_ctx;
typedef struct fsc_ens fsc_ens;

/* ----------------------------------------------------------------------- */
/* Single lattice.                                                          */
/* ----------------------------------------------------------------------- */

/* Creates a context and allocates its two population buffers (pull
 * streaming ping-pong).  `stream` is a hipStream_t or NULL.  The state is
 * undefined until fsc_init_uniform or fsc_set_populations.  One population
 * (nx ny nz values) must stay below 4 GiB: up to about 1000^3 nodes in FP32,
 * 800^3 in FP64.  Errors: FSC_E_INVAL (bad parameters, lattice too large),
 * FSC_E_NOTSUP (E8 in 3D), FSC_E_OOM, FSC_E_HIP. */
int fsc_create(const fsc_params *p, void *stream, fsc_ctx **out);

/* As fsc_create, but uses two caller-owned device buffers of at least
 * Q * nx * ny * nz elements each (float for FSC_FP32_SHIFTED, double for
 * FSC_FP64), 256-byte aligned. */
int fsc_create_external(const fsc_params *p, void *stream, void *dev_buf_a, void *dev_buf_b,
                        fsc_ctx **out);

int fsc_destroy(fsc_ctx *ctx);
const char *fsc_last_error(const fsc_ctx *ctx);
const char *fsc_strerror(int code);

/* Copies the effective parameters (G resolved from T_hat) into *out. */
int fsc_get_params(const fsc_ctx *ctx, fsc_params *out);

/* Homogeneous initial condition of the runs (paper, simulation protocol):
 * f_i = w_i rho0, time step 0, S(k) accumulators cleared. */
int fsc_init_uniform(fsc_ctx *ctx);

/* Sets the streamed populations f (host, double, layout above) as the state
 * of Eq. (12) at time step `step` (0 <= step < 2^32).  Clears nothing else.
 * Values are stored as deviations f_i - w_i rho0 in the context's precision
 * (rounded to float for FSC_FP32_SHIFTED); they are not checked (a
 * non-finite or non-positive density shows in fsc_stats). */
int fsc_set_populations(fsc_ctx *ctx, const double *host_f, int64_t step);

/* Reads the streamed populations of the current state of Eq. (12) into
 * host_f (w_i rho0 + the stored deviation, in double) and the current time
 * step into *step (may be NULL).  Synchronises the stream. */
int fsc_get_populations(fsc_ctx *ctx, double *host_f, int64_t *step);

/* Advances the state by nsteps >= 0 time steps of Eq. (12) with the force of
 * Eq. (1) and the moment-space noise described after Eq. (16): one fused
 * kernel launch per step, or per pair of steps where the tiling in use is the
 * two-step kernel (2D FP32; bit-identical results, see fsc_tile_shapes).  The
 * noise of step t at node s uses counter (s, t, block, seed >> 32) and key
 * (seed & 0xffffffff, replica) (fsc_normals).  Enqueued on the context's
 * stream.  Fails with FSC_E_INVAL if the step count would pass 2^32. */
int fsc_step(fsc_ctx *ctx, int64_t nsteps);

/* Advances nsteps and accumulates one S(k) sample after every `sk_every`
 * steps (sk_every <= 0: no samples).  Whole chunks are replayed as one
 * captured hipGraph.  Equivalent to alternating fsc_step / fsc_measure_sk. */
int fsc_run(fsc_ctx *ctx, int64_t nsteps, int64_t sk_every);

int fsc_get_step(const fsc_ctx *ctx, int64_t *step);

/* Checkpoint of a single lattice: same file format and behaviour as
 * fsc_ens_save / fsc_ens_load below (one replica). */
int fsc_save(fsc_ctx *ctx, const char *path);
int fsc_load(fsc_ctx *ctx, const char *path);

/* Density n(x) = sum_i f_i of the current state (the field whose
 * fluctuations the paper's S(k) measures), host double [nz][ny][nx].
 * fsc_read_density is the same call under the name of the problem
 * statement's "measure rho".  Synchronises the stream. */
int fsc_density(fsc_ctx *ctx, double *host_rho);
int fsc_read_density(fsc_ctx *ctx, double *host_rho);

/* FP64 reductions of the current state, the quantities the collision
 * conserves (mass exactly, momentum up to the force, whose lattice sum
 * vanishes; the paper's protocol relies on the exact mass conservation):
 * out[0] = sum n, out[1..3] = sum j (x, y, z; z = 0 in 2D), out[4] = min n,
 * out[5] = max n over nodes with a number as density (NaN nodes are skipped),
 * out[6] = number of nodes with a non-finite or non-positive density,
 * out[7] = node count.  Returns FSC_E_DIVERGED (after filling out) when
 * out[6] > 0.  Synchronises the stream. */
int fsc_stats(fsc_ctx *ctx, double *out8);
/* The conserved sums alone: *mass = sum n, mom[0..D-1] = sum j.  Errors as
 * fsc_stats (FSC_E_DIVERGED after filling them). */
int fsc_conserved(fsc_ctx *ctx, double *mass, double *mom);

/* Structure factor.  One sample adds, for every wave vector k != 0 of the
 * lattice (k_d = 2 pi m_d / n_d), P(k) = |sum_x n(x) e^{-i k.x}|^2 / N to the
 * FP64 accumulators of its bins (sum and sum of squares); count holds the
 * number of (mode, sample) pairs per bin.
 *   FSC_SK_AXIS   nbins = D * (max side / 2 + 1); bin [d][m] collects the
 *                 modes with m_d = +-m and all other components 0.
 *   FSC_SK_RADIAL nbins = round(sqrt(D) * n / 2) + 1 when all sides equal n,
 *                 else 0; shell b collects the modes with round(|m|) = b,
 *                 decided in exact integer arithmetic.
 * Mean S(k) of a bin = sum / count. */
/* One sample fills both bin kinds from one FFT of the density; the kind is
 * chosen when reading (fsc_read_sk's `kind` plays the role of a measurement
 * mode).  S(k) is the quantity compared with Eq. (16); the sample is
 * enqueued on the context's stream. */
int fsc_sk_reset(fsc_ctx *ctx);
int fsc_measure_sk(fsc_ctx *ctx);
int fsc_sk_nbins(const fsc_ctx *ctx, int kind, int *nbins);
int fsc_read_sk(fsc_ctx *ctx, int kind, double *sum, double *sumsq, int64_t *count, int nbins);

/* Time series of S(k, t) and the domain length L(t) (unstable runs, where
 * the structure factor evolves).  With capacity > 0, every S(k) sample also
 * writes one row (step, L, S_1 .. S_{nb-1}) where S_b is that sample's mean of
 * P(k) over radial shell b (row_len = 2 + nb, nb = radial bin count; 0 shells
 * for non-cubic lattices) and
 *     L = 2 pi sum_k P(k) / sum_k |k| P(k)      (k != 0, |k| exact per mode),
 * the inverse first moment of the structure factor as a domain size.  Rows past
 * `capacity` are counted but not stored.  Enabling clears the series. */
int fsc_series_enable(fsc_ctx *ctx, int capacity);
/* Copies min(rows, max_rows) rows into out (row-major, row_len doubles each). */
int fsc_read_series(fsc_ctx *ctx, double *out, int max_rows, int *nrows, int *row_len);

/* ----------------------------------------------------------------------- */
/* Ensemble: many independent replicas (uneven sides, couplings, densities, */
/* seeds) advanced together, one kernel launch per step over all replicas'  */
/* tiles; fsc_ens_run replays captured hipGraphs.  All replicas must share   */
/* D, stencil and precision.                                                */
/* ----------------------------------------------------------------------- */
int fsc_ens_create(const fsc_params *reps, int nrep, void *stream, fsc_ens **out);
int fsc_ens_destroy(fsc_ens *ens);
const char *fsc_ens_last_error(const fsc_ens *ens);
int fsc_ens_init_uniform(fsc_ens *ens);
int fsc_ens_run(fsc_ens *ens, int64_t nsteps, int64_t sk_every);
int fsc_ens_get_step(const fsc_ens *ens, int64_t *step);
int fsc_ens_get_populations(fsc_ens *ens, int replica, double *host_f);
int fsc_ens_set_populations(fsc_ens *ens, int replica, const double *host_f);
int fsc_ens_stats(fsc_ens *ens, int replica, double *out8);
/* Density of one replica's current state, host double [nz][ny][nx]. */
int fsc_ens_density(fsc_ens *ens, int replica, double *host_rho);
int fsc_ens_sk_nbins(const fsc_ens *ens, int replica, int kind, int *nbins);
int fsc_ens_read_sk(fsc_ens *ens, int replica, int kind, double *sum, double *sumsq,
                    int64_t *count, int nbins);
int fsc_ens_sk_reset(fsc_ens *ens);

/* Checkpoint and resume.  fsc_ens_save writes the current step, every
 * replica's parameters, its populations exactly as stored and its FP64 S(k)
 * accumulators to a file at `path` (host file IO, caller-owned path; the
 * stream is synchronised).  fsc_ens_load restores them into an ensemble
 * created with the same parameters, in the same order: continuing from the
 * loaded state is bit-identical to continuing the saved run, because the
 * noise of Eq. 12 depends only on (seed, replica, node, step).  Errors:
 * FSC_E_IO (cannot open, truncated, not a checkpoint), FSC_E_INVAL (another
 * replica count or other parameters; nothing is changed), FSC_E_HIP.
 * Time-series rows (fsc_ens_series_enable) are not part of the file. */
int fsc_ens_save(fsc_ens *ens, const char *path);
int fsc_ens_load(fsc_ens *ens, const char *path);
/* Recorded mode amplitudes (for the dynamic structure factor).  Once
 * enabled, every S(k) sample (fsc_measure_sk, or the samples of fsc_run /
 * fsc_ens_run) also stores the complex amplitudes
 * dn^(k) = sum_x (n(x) - n0) e^{-i k.x} of the modes m = 1..nm along each
 * lattice axis (k = 2 pi m / side) as a row [D][nm][2] of doubles (real,
 * imaginary); rows past `capacity` are dropped.  Enabling (capacity >= 1,
 * 1 <= nm <= side/2) allocates and clears the rows; capacity 0 disables.
 * fsc_read_modes copies min(recorded, max_rows) rows to `out` and returns
 * the number recorded in *nrows.  Errors: FSC_E_INVAL, FSC_E_OOM, FSC_E_HIP. */
int fsc_modes_enable(fsc_ctx *ctx, int nm, int capacity);
int fsc_read_modes(fsc_ctx *ctx, double *out, int max_rows, int *nrows);
int fsc_ens_modes_enable(fsc_ens *ens, int nm, int capacity);
int fsc_ens_read_modes(fsc_ens *ens, int replica, double *out, int max_rows, int *nrows);
int fsc_ens_series_enable(fsc_ens *ens, int capacity);
int fsc_ens_read_series(fsc_ens *ens, int replica, double *out, int max_rows, int *nrows,
                        int *row_len);

/* ----------------------------------------------------------------------- */
/* Exact linear theory for any wave vector.                                 */
/* ----------------------------------------------------------------------- */

/* Stationary structure factor of the fluctuating step linearised around the
 * homogeneous state n0 = p->rho0 (Eq. 12 with the force of Eq. 1 linearised):
 * S(k) = 1^T X 1, X = sum_j A^j Qn (A^j)^H, where A(k) is the linearised
 * step (collision with the Guo source, then streaming) and Qn(k) the
 * covariance of the noise; on a lattice axis with the E4 stencil this is
 * Eq. 16.  host_k: nk wave vectors [nk][D] in lattice units (k = 2 pi m / L);
 * host_s: nk doubles (out).  Uses p's D, stencil, T_hat or G, rho0, rates and
 * kBT (sides are ignored).  FP64 on the GPU, one workgroup per wave vector;
 * synchronous on `stream` (NULL: the default stream).  Errors: FSC_E_INVAL,
 * FSC_E_OOM, FSC_E_HIP. */
int fsc_linear_sk(const fsc_params *p, const double *host_k, int64_t nk, double *host_s,
                  void *stream);
/* The same averaged over the radial shells b = round(|m|) of all wave
 * vectors m != 0 of p's square (2D) or cubic (3D) lattice, as the radial bins
 * of fsc_read_sk: host_shell_mean[b] and, if not NULL, host_count[b] modes,
 * b < nbins (shells beyond are dropped).  Uses the symmetry of the square /
 * cube (one wave vector per orbit).  FSC_E_INVAL unless the sides are
 * equal. */
int fsc_linear_sk_radial(const fsc_params *p, double *host_shell_mean, int64_t *host_count,
                         int nbins, void *stream);
/* Time correlation of the linearised dynamics in the stationary state:
 * C(k, tau) = <dn^(k, t + tau) dn^(k, t)*> / N = 1^T A^tau X 1 (C(k, 0) is
 * fsc_linear_sk), for nk wave vectors host_k [nk][D] and nlag lags
 * host_lags[] >= 0 in lattice steps (ascending); host_c [nk][nlag][2]
 * (real, imaginary; the imaginary part vanishes for the symmetric lattices
 * here).  Its Fourier transform over tau is the dynamic structure factor
 * S(k, omega) of the linearised step.  Errors as fsc_linear_sk. */
int fsc_linear_corr(const fsc_params *p, const double *host_k, int64_t nk, const int *host_lags,
                    int nlag, double *host_c, void *stream);

/* ----------------------------------------------------------------------- */
/* Learned coarse-grained surrogate (not in the paper).                     */
/*                                                                          */
/* A periodic convolutional network advances the block-averaged density of  */
/* a phase-separating 2D lattice by a fixed stride of k lattice steps:      */
/*   x_0 = (rho_t - mean)/in_scale                                          */
/*   x_1 = (rho_t - rho_{t-k})/out_scale          (in_ch = 2 only)          */
/*   a_0 = SiLU(conv(x)); a_l = SiLU(conv(a_l-1)), l = 1..layers-2 (32 ch);  */
/*   y = conv(a_layers-2); rho_{t+k} = rho_t + out_scale (y - <y>_image)    */
/* (each image's mean is conserved).  conv = 3x3 cross-correlation with     */
/* circular padding.  The 32 -> 32 layers run on BF16 matrix cores with     */
/* FP32 accumulation (forward, backward-data and backward-weight); the      */
/* parameters are FP32, trained by Adam on the loss                         */
/* mean((y - <y>) - (target - rho_t)/out_scale)^2.  Fields are device float  */
/* arrays [batch][H][W] (prev = rho_{t-k}, in = rho_t); calls run on the    */
/* stream given at creation (NULL: the device's default stream) and return  */
/* after enqueueing, except those returning host data.  The caller orders   */
/* its own writes of the inputs before, and reads of the outputs after,     */
/* on that stream.  Errors: FSC_E_INVAL (bad sizes, batch out of            */
/* range, prev missing for in_ch = 2), FSC_E_OOM, FSC_E_HIP.                */
/* ----------------------------------------------------------------------- */
typedef struct fsc_sur fsc_sur;

/* layers in [3, 16]; in_ch 1 or 2; W a multiple of 32; max_batch * H * W <
 * 2^26.  Weights and biases are drawn from `seed`, uniform in
 * +-1/sqrt(fan_in) (fan_in = 9 c_in). */
int fsc_sur_create(int layers, int in_ch, int H, int W, int max_batch, uint64_t seed,
                   void *stream, fsc_sur **out);
int fsc_sur_destroy(fsc_sur *s);
const char *fsc_sur_last_error(const fsc_sur *s);
/* Parameters: one float vector, per layer W[c_out][c_in][3][3] then b[c_out]. */
int fsc_sur_nparams(const fsc_sur *s, int64_t *n);
int fsc_sur_set_params(fsc_sur *s, const float *host, int64_t n); /* resets Adam state */
int fsc_sur_get_params(fsc_sur *s, float *host, int64_t n);
int fsc_sur_set_norm(fsc_sur *s, float mean, float in_scale, float out_scale);
/* dev_prev is ignored (may be NULL) when in_ch = 1. */
int fsc_sur_forward(fsc_sur *s, const float *dev_prev, const float *dev_in, float *dev_out,
                    int batch);
/* Gradient of the loss (host float[nparams], may be NULL) and the loss. */
int fsc_sur_grad(fsc_sur *s, const float *dev_prev, const float *dev_in, const float *dev_target,
                 int batch, float *host_grad, double *loss);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) at learning rate lr; *loss (may be
 * NULL) gets the loss before the update. */
int fsc_sur_train_step(fsc_sur *s, const float *dev_prev, const float *dev_in,
                       const float *dev_target, int batch, float lr, double *loss);

/* Rollout: `passes` forward passes in a row, traj [passes + 1][batch][H][W]
 * with traj[0] the start (set by the caller) and traj[k + 1] the prediction
 * from (traj[k - 1], traj[k]) (dev_prev in place of traj[-1]; ignored for
 * in_ch = 1).  The passes are captured once per (dev_prev, dev_traj, batch,
 * passes) into a hipGraph and replayed, so the launches of a rollout run
 * back to back; the replay is ordered after earlier and before later work
 * on the surrogate's stream.  Results equal `passes` calls of
 * fsc_sur_forward.  At most 8 captures are kept per surrogate: a ninth
 * drops the oldest (after waiting for a replay of it still running). */
int fsc_sur_rollout(fsc_sur *s, const float *dev_prev, float *dev_traj, int batch, int passes);

/* Inference (forward passes and rollouts) can run pairs of consecutive
 * 32 -> 32 layers as one launch that keeps the first layer's activations in
 * LDS (needs H % 4 == 0 and W % 64 == 0, else one launch per layer).  The
 * results are bit for bit those of one launch per layer.  mode 0: never;
 * 1: always; 2 (the default): when batch * H * W <= 8 * 128 * 128, where it
 * measured faster (its LDS halves the blocks per CU, which costs more than
 * it saves on larger batches).  Other modes: FSC_E_INVAL.  Changing the mode,
 * or the normalisation (fsc_sur_set_norm), drops the captured rollout
 * graphs (waiting for a replay still running). */
int fsc_sur_set_fusion(fsc_sur *s, int mode);

/* Training batch from a device snapshot stack S [K][R][H][W] (float; H, W
 * the surrogate's): image b (b < batch <= min(64, max_batch)) is
 *   out[b][y][x] = S[t[b] + dt][r[b]][(Y - sy) mod H][(X - sx) mod W],
 * (Y, X) = (x, y) if `transpose` (needs H == W), else (y, x): a periodic
 * shift and a transpose, symmetries of the periodic square lattice.  host_t,
 * host_r: batch indices (host int arrays); every t[b] + dt in [0, K), r[b]
 * in [0, R), else FSC_E_INVAL.  Enqueued on the surrogate's stream. */
int fsc_sur_gather(fsc_sur *s, const float *dev_snaps, int K, int R, const int *host_t,
                   const int *host_r, int batch, int dt, int sy, int sx, int transpose,
                   float *dev_out);

/* Data scales of a snapshot stack S [K][per_snap] (float, device), in FP64:
 * *host_in_std = sample standard deviation (n - 1) of S[t_first..K-1], and
 * *host_out_std = that of the increments S[k+1] - S[k], k = t_first..K-2
 * (the network's input and output scales).  `centre` is subtracted before
 * squaring (any value near the mean; it does not change the result beyond
 * rounding).  Synchronous on `stream` (NULL: the default stream). */
int fsc_stack_scales(const float *dev_snaps, int K, int64_t per_snap, int t_first, double centre,
                     double *host_in_std, double *host_out_std, void *stream);

/* Block-averaged density of the current state over factor x factor blocks
 * into dev_out[(ny/factor) x (nx/factor)] (2D lattices, sides divisible by
 * factor); enqueued on the lattice's stream. */
int fsc_coarsen(fsc_ctx *ctx, int factor, float *dev_out);
int fsc_ens_coarsen(fsc_ens *ens, int replica, int factor, float *dev_out);

/* S(k) of device fields [batch][n][n] (float): per radial shell the mean of
 * |sum_x f(x) e^{-ik.x}|^2 / n^2 (shells as FSC_SK_RADIAL, nbins from
 * fsc_field_nbins) and L = 2 pi sum P / sum |k| P.  Synchronous on `stream`. */
int fsc_field_nbins(int n, int *nbins);
int fsc_field_sk(const float *dev_fields, int batch, int ny, int nx, void *stream,
                 double *host_shell_mean, double *host_L, int nbins);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * same computation and results as fsc_field_sk, with every work area (complex
 * FFT lines, twiddles, FP64 accumulators, counter) in a fixed-size scratch
 * array that the library holds in device memory, about 16 MiB per device for
 * the life of the process.  It calls no hipMalloc or hipFree.  Fields up to
 * 1024 x 1024 (ny = nx <= 1024); larger ones return FSC_E_RANGE before any
 * device work.  All calls on one device share that device's scratch, and each
 * call re-initialises what it reads: calls that overlap in time on one device
 * (other host threads, or other streams) race and give wrong results, so the
 * caller serialises them.  Synchronous on `stream` (NULL: the current
 * device's default stream); the scratch of the stream's device is used. */
int fsc_field_sk_noalloc(const float *dev_fields, int batch, int ny, int nx, void *stream,
                         double *host_shell_mean, double *host_L, int nbins);

/* Matrix-core layout check: C = A (16x32) B (32x16) through one BF16 MFMA
 * with the operand placement the surrogate kernels use (host row-major). */
int fsc_mfma_probe(const float *host_a, const float *host_b, float *host_c);

/* ----------------------------------------------------------------------- */
/* Tiling of the fused step.                                                */
/* ----------------------------------------------------------------------- */

/* Times every compiled tile shape (cross-section tile, register prefetch
 * depth) and marching length on the context's own buffers and keeps the
 * fastest; the choice is cached per process and geometry.  Trial launches
 * alternate between the two buffers as a run does, on a temporary device copy
 * of the state that is put back afterwards (without room for the copy, every
 * trial reads the current buffer and writes the other).  The state is not
 * changed and results do not depend on the tiling.  fsc_step / fsc_run tune automatically
 * on first use when the lattice (or ensemble) has at least 2^20 nodes, unless
 * the environment sets FSC_AUTOTUNE=0 (FSC_AUTOTUNE=1 tunes at any size). */
int fsc_autotune(fsc_ctx *ctx);
int fsc_ens_autotune(fsc_ens *ens);

/* out[0..4] = tile x, tile y, prefetch depth, workgroups per launch, time
 * steps per launch (1, or 2 for the two-step kernel). */
int fsc_get_tiling(const fsc_ctx *ctx, int *out5);
int fsc_ens_get_tiling(const fsc_ens *ens, int *out5);

/* The tilings compiled for a lattice kind: writes up to `max` quadruples
 * (tile x, tile y, prefetch depth, steps per launch) to host out4[4 max] and
 * returns how many exist (the first is the default), or FSC_E_INVAL for an
 * unsupported kind.  Steps per launch 2 is the temporally blocked kernel of
 * 2D FP32 lattices: each launch advances two time steps with one read and
 * one write of the populations, keeping the intermediate state on chip; the
 * results equal two single steps bit for bit.  Runs then go in pairs of steps,
 * with single steps where an S(k) sample falls between two steps.  For these
 * tilings the prefetch field selects the on-chip schedule (0: one barrier per
 * row; 1: two barriers per row and 3/4 of the LDS).  The two-step widths 246
 * (E8) and 250 (E4) keep the tile's 4R + 2 halo columns in its own 256 lanes
 * instead of an extra wave. */
int fsc_tile_shapes(int D, int stencil, int precision, int *out4, int max);

/* Fixes the tiling instead of tuning it: one of the compiled tilings, and a
 * marching length chosen to give about target_blocks (>= 1) workgroups per
 * launch.  Results do not depend on it.  FSC_E_INVAL for a tiling that is not
 * compiled for the lattice, or a two-step tiling on a lattice narrower than
 * 2R + 2 columns (R = 1 for E4, 2 for E8) or with population buffers of
 * 4 GiB or more (those run single steps). */
int fsc_set_tiling(fsc_ctx *ctx, int tx, int ty, int pf, int steps, int64_t target_blocks);
int fsc_ens_set_tiling(fsc_ens *ens, int tx, int ty, int pf, int steps, int64_t target_blocks);

/* ----------------------------------------------------------------------- */
/* Diagnostics.                                                             */
/* ----------------------------------------------------------------------- */

/* Enqueues a plain device-to-device copy of `bytes` (a positive multiple of
 * 16) on `stream` with 16-byte accesses: the practical HBM read+write ceiling
 * that the step kernel's bandwidth is compared with, and the calibration of
 * the memory-traffic counters.  Asynchronous. */
int fsc_copy(const void *dev_src, void *dev_dst, int64_t bytes, void *stream);

/* ----------------------------------------------------------------------- */
/* Generator checks.                                                        */
/* ----------------------------------------------------------------------- */

/* Evaluates the device Philox4x32-10 (Salmon et al., SC'11) for n counters
 * (host arrays: ctr[4n], key[2n], out[4n]).  Synchronous. */
int fsc_philox(const uint32_t *host_ctr, const uint32_t *host_key, uint32_t *host_out, int64_t n);

/* The Q-D-1 standard normals the step kernel draws for each (node, step)
 * pair (host arrays node[n], step[n]; out[n][Q-D-1] as double), computed in
 * the given precision (FSC_FP32_SHIFTED: float, FSC_FP64: double).  The
 * paper fixes only that the noise is Gaussian and uncorrelated in space and
 * time; the generator is this library's: words w_0, w_1, .. are Philox4x32-10
 * outputs of blocks 0, 1, .. (one block for D2Q9, three for D3Q19) with key
 * (seed & 0xffffffff, replica) and counter (node, step, block, seed >> 32).
 * Pair k uses the radius uniform u_a = (floor(w_k / 2^9) + 1/2) / 2^23 and a
 * 16-bit angle uniform u_b = (h_k + 1/2) / 2^16:
 *   D2Q9 : h_0 = high half of w_3, h_1 = low half of w_3,
 *          h_2 = (low byte of w_0) * 256 + low byte of w_1;
 *   D3Q19: h_k = the k-th 16-bit half of w_8 .. w_11, high half first;
 * (z_2k, z_2k+1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b); normal m goes
 * to the m-th non-conserved moment.  Synchronous. */
int fsc_normals(int D, int precision, uint64_t seed, uint32_t replica, const int64_t *host_node,
                const int64_t *host_step, int64_t n, double *host_out);

#ifdef __cplusplus
}
#endif
#endif /* FSC_H */
