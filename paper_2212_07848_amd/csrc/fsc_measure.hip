// fsc_measure.hip -- density gathers, FP64 state reductions, and the
// structure-factor pipeline S(k) = <|dn(k)|^2> / N of Lulli et al.
// (arXiv:2212.07848, the quantity compared with Eq. 16):
//   density gather -> complex FFT along each axis (LDS radix-2 Cooley-Tukey
//   per line, or a direct DFT for other lengths) with axis rotations between
//   passes -> per-line binning with an LDS window of radial shells and FP64
//   accumulation.
#include "fsc_internal.h"

namespace fsc {

template <typename real>
struct cplx {
    real re, im;
};

// ---------------------------------------------------------------------------
// Density gather: the streamed state at x is f_i(x) = f*_i(x - c_i) of the
// stored post-collision buffer; dn = sum_i df_i.  One block = 256 x-values
// of one (y, z) row.
// ---------------------------------------------------------------------------
template <class L, typename real>
__device__ inline void gather_node(const real *src, const Geometry &g, int x, int y, int z,
                                   real (&f)[L::Q]) {
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x + 1 == g.nx ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y + 1 == g.ny ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z + 1 == g.nz ? 0 : z + 1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
        const int xs = cx == 1 ? xm : (cx == -1 ? xp : x);
        const int ys = cy == 1 ? ym : (cy == -1 ? yp : y);
        const int zs = cz == 1 ? zm : (cz == -1 ? zp : z);
        f[i] = src[int64_t(i) * g.N + xs + int64_t(g.nx) * (ys + int64_t(g.ny) * zs)];
    }
}

template <class L, typename real, bool CPLX>
__device__ inline void density_block(const Geometry &g, const real *__restrict__ src,
                                     real *__restrict__ out, int blk) {
    const int strips = (g.nx + 255) / 256;
    const int row = blk / strips;
    const int x = (blk % strips) * 256 + threadIdx.x;
    if (x >= g.nx) return;
    const int y = row % g.ny, z = row / g.ny;
    real f[L::Q];
    gather_node<L, real>(src, g, x, y, z, f);
    real dn = real(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) dn += f[i];
    const int64_t s = int64_t(row) * g.nx + x;
    if (CPLX) {
        out[2 * s] = dn;
        out[2 * s + 1] = real(0);
    } else {
        out[s] = dn;
    }
}

template <class L, typename real, bool CPLX>
__global__ void __launch_bounds__(256) k_density(Geometry g, const real *__restrict__ src,
                                                 real *__restrict__ out) {
    density_block<L, real, CPLX>(g, src, out, int(blockIdx.x));
}

template <class L, typename real>
static hipError_t density_impl(const Geometry &g, const void *buf, void *out, bool cplx,
                               hipStream_t s) {
    const int strips = (g.nx + 255) / 256;
    const int64_t blocks = int64_t(strips) * g.ny * g.nz;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (cplx)
        hipLaunchKernelGGL((k_density<L, real, true>), dim3(unsigned(blocks)), dim3(256), 0, s, g,
                           static_cast<const real *>(buf), static_cast<real *>(out));
    else
        hipLaunchKernelGGL((k_density<L, real, false>), dim3(unsigned(blocks)), dim3(256), 0, s, g,
                           static_cast<const real *>(buf), static_cast<real *>(out));
    return hipGetLastError();
}

static hipError_t density_dispatch(const Geometry &g, int precision, const void *buf, void *out,
                                   bool cplx, hipStream_t s) {
    if (g.D == 2)
        return precision == 0 ? density_impl<D2Q9, float>(g, buf, out, cplx, s)
                              : density_impl<D2Q9, double>(g, buf, out, cplx, s);
    return precision == 0 ? density_impl<D3Q19, float>(g, buf, out, cplx, s)
                          : density_impl<D3Q19, double>(g, buf, out, cplx, s);
}

hipError_t launch_density_real(const Geometry &g, int precision, const void *buf, void *out,
                               hipStream_t s) {
    return density_dispatch(g, precision, buf, out, false, s);
}

// ---------------------------------------------------------------------------
// FP64 reductions: sum dn, sum j, min/max n, bad-node count.  A fixed grid of
// STAT_BLOCKS blocks strides over rows; the partials are reduced by one block
// in a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int STAT_BLOCKS = 1024;
constexpr int STAT_W = 8;
size_t stats_partials_len() { return size_t(STAT_BLOCKS) * STAT_W; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// reduces acc[STAT_W] over a 256-thread block; thread 0 returns the result
__device__ inline void block_reduce_stats(double (&acc)[STAT_W]) {
    __shared__ double sh[4][STAT_W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < STAT_W; ++k) {
        double v = acc[k];
        v = (k == 4) ? wave_min(v) : (k == 5 ? wave_max(v) : wave_sum(v));
        if (lane == 0) sh[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < STAT_W; ++k) {
            double v = sh[0][k];
            for (int w = 1; w < 4; ++w)
                v = (k == 4) ? fmin(v, sh[w][k]) : (k == 5 ? fmax(v, sh[w][k]) : v + sh[w][k]);
            acc[k] = v;
        }
    }
}

template <class L, typename real>
__global__ void __launch_bounds__(256) k_stats(Geometry g, const real *__restrict__ src,
                                               double rho0, double *__restrict__ partials) {
    double acc[STAT_W] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 0.0};
    const int rows = g.ny * g.nz;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int y = row % g.ny, z = row / g.ny;
        for (int x = threadIdx.x; x < g.nx; x += 256) {
            real f[L::Q];
            gather_node<L, real>(src, g, x, y, z, f);
            double dn = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const double v = double(f[i]);
                dn += v;
#pragma unroll
                for (int q = 0; q < 3; ++q) j[q] += double(L::c(i, q)) * v;
            }
            const double n = rho0 + dn;
            acc[0] += dn;
            acc[1] += j[0];
            acc[2] += j[1];
            acc[3] += j[2];
            acc[4] = fmin(acc[4], n);
            acc[5] = fmax(acc[5], n);
            acc[6] += (isfinite(n) && n > 0.0) ? 0.0 : 1.0;
            acc[7] += 1.0;
        }
    }
    block_reduce_stats(acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < STAT_W; ++k) partials[blockIdx.x * STAT_W + k] = acc[k];
}

__global__ void __launch_bounds__(256) k_stats_final(const double *__restrict__ partials,
                                                     int nblocks, double n_rho0,
                                                     double *__restrict__ out) {
    double acc[STAT_W] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        const double *p = partials + b * STAT_W;
        for (int k = 0; k < STAT_W; ++k)
            acc[k] = (k == 4) ? fmin(acc[k], p[k]) : (k == 5 ? fmax(acc[k], p[k]) : acc[k] + p[k]);
    }
    block_reduce_stats(acc);
    if (threadIdx.x == 0) {
        out[0] = n_rho0 + acc[0];
        for (int k = 1; k < STAT_W; ++k) out[k] = acc[k];
    }
}

hipError_t launch_stats(const Geometry &g, int precision, const void *buf, double rho0,
                        double *partials, double *out, hipStream_t s) {
    const int rows = g.ny * g.nz;
    const int nb = rows < STAT_BLOCKS ? rows : STAT_BLOCKS;
    if (g.D == 2) {
        if (precision == 0)
            hipLaunchKernelGGL((k_stats<D2Q9, float>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const float *>(buf), rho0, partials);
        else
            hipLaunchKernelGGL((k_stats<D2Q9, double>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const double *>(buf), rho0, partials);
    } else {
        if (precision == 0)
            hipLaunchKernelGGL((k_stats<D3Q19, float>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const float *>(buf), rho0, partials);
        else
            hipLaunchKernelGGL((k_stats<D3Q19, double>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const double *>(buf), rho0, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, s, partials, nb,
                       double(g.N) * rho0, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FFT along the contiguous axis + rotation [n2][n1][n0] -> [n0][n2][n1].
// ---------------------------------------------------------------------------
size_t twiddle_len(int n) { return (n & (n - 1)) == 0 ? size_t(n > 1 ? n / 2 : 1) : size_t(n); }

template <typename real>
__global__ void k_twiddle(cplx<real> *tw, int n, int len) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double s, c;
    // exp(-2 pi i k / n), argument reduced exactly through sincospi
    sincospi(-2.0 * double(k) / double(n), &s, &c);
    tw[k].re = real(c);
    tw[k].im = real(s);
}

hipError_t launch_twiddles(int precision, void *tw, int n, hipStream_t s) {
    const int len = int(twiddle_len(n));
    const int nb = (len + 255) / 256;
    if (precision == 0)
        hipLaunchKernelGGL(k_twiddle<float>, dim3(nb), dim3(256), 0, s,
                           static_cast<cplx<float> *>(tw), n, len);
    else
        hipLaunchKernelGGL(k_twiddle<double>, dim3(nb), dim3(256), 0, s,
                           static_cast<cplx<double> *>(tw), n, len);
    return hipGetLastError();
}

// Iterative radix-2 Cooley-Tukey on one line staged in LDS (a[n]): bit-reversed
// load, then log2(n) butterfly stages with twiddles W_len^k = tw[k * n/len].
template <typename real>
__device__ inline void fft_line_pow2(cplx<real> *__restrict__ line, const cplx<real> *__restrict__ tw,
                                     int n, int logn, cplx<real> *a) {
    for (int i = threadIdx.x; i < n; i += 256) {
        const int r = logn == 0 ? 0 : int(__brev(unsigned(i)) >> (32 - logn));
        a[r] = line[i];
    }
    __syncthreads();
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1;
        const int stride = n / len;
        for (int j = threadIdx.x; j < n / 2; j += 256) {
            const int g = j / half, k = j - g * half;
            const int i0 = g * len + k, i1 = i0 + half;
            const cplx<real> w = tw[k * stride];
            const cplx<real> u = a[i0], v0 = a[i1];
            const cplx<real> v = {v0.re * w.re - v0.im * w.im, v0.re * w.im + v0.im * w.re};
            a[i0] = {u.re + v.re, u.im + v.im};
            a[i1] = {u.re - v.re, u.im - v.im};
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += 256) line[i] = a[i];
}

// Direct DFT of one line (any n): X_k = sum_j x_j tw[(j k) mod n].
template <typename real>
__device__ inline void dft_line(cplx<real> *__restrict__ line, const cplx<real> *__restrict__ tw, int n,
                                cplx<real> *a) {
    for (int i = threadIdx.x; i < n; i += 256) a[i] = line[i];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 256) {
        real sr = real(0), si = real(0);
        int idx = 0;
        for (int j = 0; j < n; ++j) {
            const cplx<real> w = tw[idx];
            sr += a[j].re * w.re - a[j].im * w.im;
            si += a[j].re * w.im + a[j].im * w.re;
            idx += k;
            if (idx >= n) idx -= n;
        }
        line[k] = {sr, si};
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_fft_pow2(cplx<real> *__restrict__ data,
                                                  const cplx<real> *__restrict__ tw, int n,
                                                  int logn) {
    extern __shared__ unsigned char smem_raw[];
    fft_line_pow2<real>(data + int64_t(blockIdx.x) * n, tw, n, logn,
                        reinterpret_cast<cplx<real> *>(smem_raw));
}

template <typename real>
__global__ void __launch_bounds__(256) k_dft(cplx<real> *__restrict__ data,
                                             const cplx<real> *__restrict__ tw, int n) {
    extern __shared__ unsigned char smem_raw[];
    dft_line<real>(data + int64_t(blockIdx.x) * n, tw, n, reinterpret_cast<cplx<real> *>(smem_raw));
}

// out[(i0 * n2 + i2) * n1 + i1] = in[(i2 * n1 + i1) * n0 + i0], via 32x32 LDS tiles;
// block (b0, b1, i2) of the (ceil(n0/32), ceil(n1/32), n2) grid
template <typename real>
__device__ inline void rotate_block(const cplx<real> *__restrict__ in, cplx<real> *__restrict__ out,
                                    int n0, int n1, int n2, int bx, int by, int i2,
                                    cplx<real> (&tile)[32][33]) {
    const int b0 = bx * 32, b1 = by * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i1 = b1 + r, i0 = b0 + tx;
        if (i1 < n1 && i0 < n0) tile[r][tx] = in[(int64_t(i2) * n1 + i1) * n0 + i0];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i0 = b0 + r, i1 = b1 + tx;
        if (i0 < n0 && i1 < n1) out[(int64_t(i0) * n2 + i2) * n1 + i1] = tile[tx][r];
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_rotate(const cplx<real> *__restrict__ in,
                                                cplx<real> *__restrict__ out, int n0, int n1,
                                                int n2) {
    __shared__ cplx<real> tile[32][33];
    rotate_block<real>(in, out, n0, n1, n2, int(blockIdx.x), int(blockIdx.y), int(blockIdx.z), tile);
}

hipError_t launch_fft_axis(int precision, void *data, void *tmp, const void *twiddle, int n0,
                           int n1, int n2, hipStream_t s) {
    const int64_t lines = int64_t(n1) * n2;
    if (lines > 0x7fffffff || n0 > 8192) return hipErrorInvalidValue;
    const bool pow2 = (n0 & (n0 - 1)) == 0;
    int logn = 0;
    while ((1 << logn) < n0) ++logn;
    const size_t esz = precision == 0 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    const size_t shm = esz * size_t(n0);
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    if (precision == 0) {
        auto *d = static_cast<cplx<float> *>(data);
        auto *t = static_cast<const cplx<float> *>(twiddle);
        if (n0 > 1) {
            if (pow2)
                hipLaunchKernelGGL(k_fft_pow2<float>, dim3(unsigned(lines)), dim3(256), shm, s, d, t,
                                   n0, logn);
            else
                hipLaunchKernelGGL(k_dft<float>, dim3(unsigned(lines)), dim3(256), shm, s, d, t, n0);
        }
        hipLaunchKernelGGL(k_rotate<float>, dim3((n0 + 31) / 32, (n1 + 31) / 32, n2), dim3(256),
                           0, s, d, static_cast<cplx<float> *>(tmp), n0, n1, n2);
    } else {
        auto *d = static_cast<cplx<double> *>(data);
        auto *t = static_cast<const cplx<double> *>(twiddle);
        if (n0 > 1) {
            if (pow2)
                hipLaunchKernelGGL(k_fft_pow2<double>, dim3(unsigned(lines)), dim3(256), shm, s, d,
                                   t, n0, logn);
            else
                hipLaunchKernelGGL(k_dft<double>, dim3(unsigned(lines)), dim3(256), shm, s, d, t,
                                   n0);
        }
        hipLaunchKernelGGL(k_rotate<double>, dim3((n0 + 31) / 32, (n1 + 31) / 32, n2), dim3(256),
                           0, s, d, static_cast<cplx<double> *>(tmp), n0, n1, n2);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Binning.  One block per x-line (fixed y, z) of the spectrum.
// ---------------------------------------------------------------------------
__device__ inline int isqrt_round(int64_t m) {
    // b = round(sqrt(m)) in exact integer arithmetic ((b - 1/2)^2 <= m < (b + 1/2)^2)
    int64_t b = int64_t(sqrt(double(m)));
    while (b * b > m) --b;
    while ((b + 1) * (b + 1) <= m) ++b;
    if (m - b * b > b) ++b;
    return int(b);
}

__device__ inline int signed_mode(int q, int n) { return q <= n / 2 ? q : q - n; }

template <typename real>
__device__ inline void bin_row(const Geometry &g, const cplx<real> *__restrict__ spec,
                               const BinTargets &t, double invN, int row, double *wnd,
                               double (&red)[2][4]) {
    const int y = row % g.ny, z = row / g.ny;
    const int my = signed_mode(y, g.ny), mz = signed_mode(z, g.nz);
    const int64_t base2 = int64_t(my) * my + int64_t(mz) * mz;
    const bool rad = t.n_rad > 0;
    const bool ser = t.mom != nullptr;
    const int srow = ser ? t.series_n[0] : 0;
    const bool ser_row = ser && t.series != nullptr && srow < t.series_cap;
    const double ky = 2.0 * M_PI * my / g.ny, kz = 2.0 * M_PI * mz / g.nz;
    int blo = 0, W = 0;
    if (rad) {
        const int half = g.nx / 2;
        blo = isqrt_round(base2);
        W = isqrt_round(base2 + int64_t(half) * half) - blo + 1;
        for (int k = threadIdx.x; k < 2 * W; k += 256) wnd[k] = 0.0;
        __syncthreads();
    }
    double sP = 0.0, skP = 0.0;
    for (int x = threadIdx.x; x < g.nx; x += 256) {
        const int mx = signed_mode(x, g.nx);
        const int64_t m2 = base2 + int64_t(mx) * mx;
        if (m2 == 0) continue;
        const cplx<real> v = spec[int64_t(row) * g.nx + x];
        const double P = (double(v.re) * double(v.re) + double(v.im) * double(v.im)) * invN;
        const int nz_cnt = (mx != 0) + (my != 0) + (mz != 0);
        if (nz_cnt == 1) {
            const int d = mx != 0 ? 0 : (my != 0 ? 1 : 2);
            const int m = abs(mx != 0 ? mx : (my != 0 ? my : mz));
            unsafeAtomicAdd(&t.axis_sum[d * t.n_axis + m], P);
            unsafeAtomicAdd(&t.axis_sq[d * t.n_axis + m], P * P);
        }
        if (rad) {
            const int b = isqrt_round(m2) - blo;
            atomicAdd(&wnd[b], P);
            atomicAdd(&wnd[W + b], P * P);
        }
        if (ser) {
            const double kx = 2.0 * M_PI * mx / g.nx;
            sP += P;
            skP += sqrt(kx * kx + ky * ky + kz * kz) * P;
        }
    }
    if (ser) {
        sP = wave_sum(sP);
        skP = wave_sum(skP);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) {
            red[0][wv] = sP;
            red[1][wv] = skP;
        }
    }
    if (rad || ser) __syncthreads();
    if (ser && threadIdx.x == 0) {
        unsafeAtomicAdd(&t.mom[0], red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        unsafeAtomicAdd(&t.mom[1], red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
    if (rad) {
        double *srow_bins = ser_row ? t.series + size_t(srow) * (2 + t.n_rad) + 2 : nullptr;
        for (int k = threadIdx.x; k < W; k += 256) {
            if (wnd[k] != 0.0 || wnd[W + k] != 0.0) {
                unsafeAtomicAdd(&t.rad_sum[blo + k], wnd[k]);
                unsafeAtomicAdd(&t.rad_sq[blo + k], wnd[W + k]);
                if (srow_bins) unsafeAtomicAdd(&srow_bins[blo + k], wnd[k]);
            }
        }
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_bin(Geometry g, const cplx<real> *__restrict__ spec,
                                             BinTargets t, double invN) {
    extern __shared__ double wnd[];  // [2][W]
    __shared__ double red[2][4];
    bin_row<real>(g, spec, t, invN, int(blockIdx.x), wnd, red);
}

hipError_t launch_bin(const Geometry &g, int precision, const void *spec, const BinTargets &t,
                      hipStream_t s) {
    const int64_t rows = int64_t(g.ny) * g.nz;
    if (rows > 0x7fffffff) return hipErrorInvalidValue;
    const size_t shm = t.n_rad > 0 ? sizeof(double) * 2 * size_t(g.nx / 2 + 3) : 0;
    const double invN = 1.0 / double(g.N);
    if (precision == 0)
        hipLaunchKernelGGL(k_bin<float>, dim3(unsigned(rows)), dim3(256), shm, s, g,
                           static_cast<const cplx<float> *>(spec), t, invN);
    else
        hipLaunchKernelGGL(k_bin<double>, dim3(unsigned(rows)), dim3(256), shm, s, g,
                           static_cast<const cplx<double> *>(spec), t, invN);
    return hipGetLastError();
}

// Closes one sample of a replica's time series: row *series_n gets (step, L)
// with L = 2 pi sum P / sum |k| P, the moments are cleared and the row advances.
__device__ inline void series_finalize(double *mom, double *series, int *series_n, int cap,
                                       int row_len, uint64_t step) {
    const int row = series_n[0];
    if (series != nullptr && row < cap) {
        series[size_t(row) * row_len] = double(step);
        series[size_t(row) * row_len + 1] = mom[1] > 0.0 ? 2.0 * M_PI * mom[0] / mom[1] : 0.0;
    }
    mom[0] = 0.0;
    mom[1] = 0.0;
    series_n[0] = row + 1;
}

// Mode recorder: the complex amplitudes of the modes m = 1..nm along each
// lattice axis of the transformed density (natural [z][y][x] order), as
// doubles, into row *rec_n of rec[cap][D][nm][2]; the row counter advances.
template <typename real>
__device__ inline void record_modes_block(const Geometry &g, const cplx<real> *__restrict__ spec,
                                          int nm, double *__restrict__ rec, int *__restrict__ rec_n,
                                          int cap) {
    const int row = rec_n[0];
    const int total = g.D * nm;
    if (row < cap) {
        for (int q = threadIdx.x; q < total; q += 256) {
            const int d = q / nm, m = q % nm + 1;
            const int64_t stride = d == 0 ? 1 : (d == 1 ? int64_t(g.nx) : int64_t(g.nx) * g.ny);
            const cplx<real> v = spec[int64_t(m) * stride];
            rec[(size_t(row) * total + q) * 2] = double(v.re);
            rec[(size_t(row) * total + q) * 2 + 1] = double(v.im);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) rec_n[0] = row + 1;
}

// ---------------------------------------------------------------------------
// One S(k) sample of every replica of an ensemble in a fixed number of
// launches (density, then per axis an FFT pass and a rotation, binning, mode
// records, series rows), whatever the number of replicas.  Each launch is a
// flat grid over the replicas: block b belongs to the replica r with
// pre[r] <= b < pre[r + 1] (a prefix table per kind of work).
// ---------------------------------------------------------------------------
__device__ inline int rep_of(const int *__restrict__ pre, int nrep, int b) {
    // largest r with pre[r] <= b; replicas without blocks of this kind have
    // pre[r] == pre[r + 1] and are never returned
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Arguments of the FFT pass d (transform of the contiguous axis, then the
// rotation (n0, n1, n2) -> (n1, n2, n0)); a unit middle axis makes the
// rotation a plain transpose of (n2 x n0).
struct PassDims {
    int n0, n1, n2;
};
__host__ __device__ inline PassDims pass_dims(const Geometry &g, int d) {
    int n0 = g.nx, n1 = g.ny, n2 = g.nz;
    for (int k = 0; k < d; ++k) {
        const int t = n0;
        n0 = n1;
        n1 = n2;
        n2 = t;
    }
    return n1 == 1 ? PassDims{n0, n2, 1} : PassDims{n0, n1, n2};
}

template <class L, typename real>
__global__ void __launch_bounds__(256) k_density_batch(const MeasRep *__restrict__ mr,
                                                       const int *__restrict__ pre, int nrep, int par) {
    const int r = rep_of(pre, nrep, int(blockIdx.x));
    const MeasRep &m = mr[r];
    density_block<L, real, true>(m.g, static_cast<const real *>(m.buf[par]), static_cast<real *>(m.cbuf),
                                 int(blockIdx.x) - pre[r]);
}

// pass d works in place on cbuf (d even) or ctmp (d odd) and rotates into the other
template <typename real>
__global__ void __launch_bounds__(256) k_fft_batch(const MeasRep *__restrict__ mr,
                                                   const int *__restrict__ pre, int nrep, int d) {
    extern __shared__ unsigned char smem_raw[];
    const int r = rep_of(pre, nrep, int(blockIdx.x));
    const MeasRep &m = mr[r];
    const PassDims p = pass_dims(m.g, d);
    if (p.n0 <= 1) return;
    cplx<real> *line = static_cast<cplx<real> *>((d & 1) ? m.ctmp : m.cbuf) +
                       int64_t(int(blockIdx.x) - pre[r]) * p.n0;
    const cplx<real> *tw = static_cast<const cplx<real> *>(m.tw[d]);
    cplx<real> *a = reinterpret_cast<cplx<real> *>(smem_raw);
    if ((p.n0 & (p.n0 - 1)) == 0) {
        int logn = 0;
        while ((1 << logn) < p.n0) ++logn;
        fft_line_pow2<real>(line, tw, p.n0, logn, a);
    } else {
        dft_line<real>(line, tw, p.n0, a);
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_rotate_batch(const MeasRep *__restrict__ mr,
                                                      const int *__restrict__ pre, int nrep, int d) {
    __shared__ cplx<real> tile[32][33];
    const int r = rep_of(pre, nrep, int(blockIdx.x));
    const MeasRep &m = mr[r];
    const PassDims p = pass_dims(m.g, d);
    const int gx = (p.n0 + 31) / 32, gy = (p.n1 + 31) / 32;
    const int lb = int(blockIdx.x) - pre[r];
    const int bz = lb / (gx * gy), rem = lb % (gx * gy);
    const void *in = (d & 1) ? m.ctmp : m.cbuf;
    void *out = (d & 1) ? m.cbuf : m.ctmp;
    rotate_block<real>(static_cast<const cplx<real> *>(in), static_cast<cplx<real> *>(out), p.n0, p.n1,
                       p.n2, rem % gx, rem / gx, bz, tile);
}

// the transformed spectrum lies in cbuf after an even number of passes, else in ctmp
template <typename real>
__global__ void __launch_bounds__(256) k_bin_batch(const MeasRep *__restrict__ mr,
                                                   const int *__restrict__ pre, int nrep) {
    extern __shared__ double wnd[];
    __shared__ double red[2][4];
    const int r = rep_of(pre, nrep, int(blockIdx.x));
    const MeasRep &m = mr[r];
    const void *spec = (m.g.D & 1) ? m.ctmp : m.cbuf;
    bin_row<real>(m.g, static_cast<const cplx<real> *>(spec), m.t, m.invN, int(blockIdx.x) - pre[r], wnd,
                  red);
}

template <typename real>
__global__ void __launch_bounds__(256) k_modes_batch(const MeasRep *__restrict__ mr,
                                                     const int *__restrict__ pre, int nrep) {
    const int r = rep_of(pre, nrep, int(blockIdx.x));
    const MeasRep &m = mr[r];
    const void *spec = (m.g.D & 1) ? m.ctmp : m.cbuf;
    record_modes_block<real>(m.g, static_cast<const cplx<real> *>(spec), m.modes_nm, m.modes, m.modes_n,
                             m.modes_cap);
}

__global__ void __launch_bounds__(64) k_series_batch(const MeasRep *__restrict__ mr, int nrep,
                                                     const uint64_t *__restrict__ step_base,
                                                     uint32_t step_off) {
    for (int r = threadIdx.x; r < nrep; r += 64) {
        const MeasRep &m = mr[r];
        if (m.t.mom != nullptr)
            series_finalize(m.t.mom, m.t.series, m.series_n, m.t.series_cap, 2 + m.t.n_rad,
                            step_base[0] + step_off);
    }
}

int measure_plan(const MeasRep *reps, int nrep, MeasPlan &P) {
    P.nrep = nrep;
    P.pre.assign(size_t(MK_COUNT) * (nrep + 1), 0);
    for (int k = 0; k < 3; ++k) P.shm_fft[k] = 0;
    P.shm_bin = 0;
    P.any_series = false;
    if (nrep < 1) return -1;
    const int D = reps[0].g.D;
    P.D = D;
    int64_t tot[MK_COUNT] = {};
    for (int r = 0; r < nrep; ++r) {
        const MeasRep &m = reps[r];
        const Geometry &g = m.g;
        if (g.D != D) return -1;
        int64_t n[MK_COUNT] = {};
        n[MK_DENSITY] = int64_t((g.nx + 255) / 256) * g.ny * g.nz;
        for (int d = 0; d < D; ++d) {
            const PassDims p = pass_dims(g, d);
            if (p.n0 > 8192) return -1;
            n[MK_FFT + d] = int64_t(p.n1) * p.n2;
            n[MK_ROT + d] = int64_t((p.n0 + 31) / 32) * ((p.n1 + 31) / 32) * p.n2;
            const size_t sh = P.esz * 2 * size_t(p.n0);
            if (sh > P.shm_fft[d]) P.shm_fft[d] = sh;
        }
        n[MK_BIN] = int64_t(g.ny) * g.nz;
        n[MK_MODES] = m.modes_cap > 0 ? 1 : 0;
        if (m.t.n_rad > 0) {
            const size_t sh = sizeof(double) * 2 * size_t(g.nx / 2 + 3);
            if (sh > P.shm_bin) P.shm_bin = sh;
        }
        if (m.t.mom != nullptr) P.any_series = true;
        for (int k = 0; k < MK_COUNT; ++k) {
            P.pre[size_t(k) * (nrep + 1) + r] = int(tot[k]);
            tot[k] += n[k];
            if (tot[k] > 0x7fffffff) return -1;
        }
    }
    for (int k = 0; k < MK_COUNT; ++k) P.pre[size_t(k) * (nrep + 1) + nrep] = int(tot[k]);
    if (P.shm_fft[0] > 160 * 1024 || P.shm_bin > 160 * 1024) return -1;
    return 0;
}

template <class L, typename real>
static hipError_t measure_impl(const MeasPlan &P, const MeasRep *mr, const int *pre, int par,
                               const uint64_t *step_base, uint32_t step_off, hipStream_t s) {
    const int nrep = P.nrep;
    auto total = [&](int k) { return unsigned(P.pre[size_t(k) * (nrep + 1) + nrep]); };
    auto pk = [&](int k) { return pre + size_t(k) * (nrep + 1); };
    hipLaunchKernelGGL((k_density_batch<L, real>), dim3(total(MK_DENSITY)), dim3(256), 0, s, mr,
                       pk(MK_DENSITY), nrep, par);
    for (int d = 0; d < L::D; ++d) {
        hipLaunchKernelGGL(k_fft_batch<real>, dim3(total(MK_FFT + d)), dim3(256), P.shm_fft[d], s, mr,
                           pk(MK_FFT + d), nrep, d);
        hipLaunchKernelGGL(k_rotate_batch<real>, dim3(total(MK_ROT + d)), dim3(256), 0, s, mr,
                           pk(MK_ROT + d), nrep, d);
    }
    hipLaunchKernelGGL(k_bin_batch<real>, dim3(total(MK_BIN)), dim3(256), P.shm_bin, s, mr, pk(MK_BIN),
                       nrep);
    if (total(MK_MODES) > 0)
        hipLaunchKernelGGL(k_modes_batch<real>, dim3(total(MK_MODES)), dim3(256), 0, s, mr, pk(MK_MODES),
                           nrep);
    if (P.any_series)
        hipLaunchKernelGGL(k_series_batch, dim3(1), dim3(64), 0, s, mr, nrep, step_base, step_off);
    return hipGetLastError();
}

hipError_t launch_measure(const MeasPlan &P, const MeasRep *dev_reps, const int *dev_pre, int precision,
                          int parity, const uint64_t *step_base, uint32_t step_off, hipStream_t s) {
    if (P.nrep < 1 || P.pre.size() != size_t(MK_COUNT) * (P.nrep + 1)) return hipErrorInvalidValue;
    if (P.D == 2)
        return precision == 0 ? measure_impl<D2Q9, float>(P, dev_reps, dev_pre, parity, step_base, step_off, s)
                              : measure_impl<D2Q9, double>(P, dev_reps, dev_pre, parity, step_base, step_off, s);
    return precision == 0 ? measure_impl<D3Q19, float>(P, dev_reps, dev_pre, parity, step_base, step_off, s)
                          : measure_impl<D3Q19, double>(P, dev_reps, dev_pre, parity, step_base, step_off, s);
}

// ---------------------------------------------------------------------------
// Plain device copy (16-byte lanes, grid-stride): the practical HBM
// read+write ceiling and the calibration for the memory-traffic counters.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy(const u32x4 *__restrict__ src,
                                              u32x4 *__restrict__ dst, int64_t n16) {
    // One 16-byte element per lane and a grid that covers the buffer once
    // (the loop runs only for buffers beyond 2^38 bytes).  Blocks are
    // dispatched in address order, so the lanes in flight at any moment touch
    // one compact address range; a grid-stride copy with fewer, longer-lived
    // blocks spreads them over the whole buffer and measured 10% slower.
    // Non-temporal loads and stores.
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n16; k += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t s) {
    if (bytes <= 0 || (bytes & 15)) return hipErrorInvalidValue;
    const int64_t n16 = bytes / 16;
    const int64_t want = (n16 + 255) / 256;
    const unsigned blocks = unsigned(want < (int64_t(1) << 30) ? want : (int64_t(1) << 30));
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, static_cast<const u32x4 *>(src),
                       static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Generator checks.
// ---------------------------------------------------------------------------
__global__ void k_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const U4 r = philox4x32_10(U4{ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3]},
                               key[2 * k], key[2 * k + 1]);
    out[4 * k] = r.x;
    out[4 * k + 1] = r.y;
    out[4 * k + 2] = r.z;
    out[4 * k + 3] = r.w;
}

hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                         hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(unsigned(nb)), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

template <class L, typename real>
__global__ void k_normals(uint64_t seed, uint32_t replica, const int64_t *node,
                          const int64_t *step, int64_t n, double *out) {
    constexpr int NN = L::NNORM;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    real z[NN];
    node_normals<L, real>(uint32_t(node[k]), uint32_t(step[k]), uint32_t(seed >> 32), z,
                          uint32_t(seed), replica);
    for (int q = 0; q < NN; ++q) out[k * NN + q] = double(z[q]);
}

hipError_t launch_normals(int D, int precision, uint64_t seed, uint32_t replica,
                          const int64_t *node, const int64_t *step, int64_t n, double *out,
                          hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (nb == 0) return hipSuccess;
    if (D == 2) {
        if (precision == 0)
            hipLaunchKernelGGL((k_normals<D2Q9, float>), dim3(unsigned(nb)), dim3(256), 0,
                               s, seed, replica, node, step, n, out);
        else
            hipLaunchKernelGGL((k_normals<D2Q9, double>), dim3(unsigned(nb)), dim3(256), 0,
                               s, seed, replica, node, step, n, out);
    } else {
        if (precision == 0)
            hipLaunchKernelGGL((k_normals<D3Q19, float>), dim3(unsigned(nb)), dim3(256), 0,
                               s, seed, replica, node, step, n, out);
        else
            hipLaunchKernelGGL((k_normals<D3Q19, double>), dim3(unsigned(nb)), dim3(256),
                               0, s, seed, replica, node, step, n, out);
    }
    return hipGetLastError();
}

}  // namespace fsc
