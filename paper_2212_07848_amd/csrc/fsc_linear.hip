// fsc_linear.hip -- exact structure factor of the linearised fluctuating step
// for any wave vector (the generalisation of Eq. 16 off the lattice axes).
//
// Around the homogeneous state n0 the step of Eq. 12, with the Shan-Chen
// force of Eq. 1 linearised (dF = G psi0 psi0' dn sum_a w_a e_a e^{ik.e_a}),
// acts on the Fourier amplitude of the populations as f_k <- A(k) f_k + noise,
// A = P C: C the moment-space collision with the linearised Guo source, P the
// streaming phases diag(e^{-i c_i.k}).  The noise covariance is
// Qn = P (sum over non-conserved rows a of amp_a^2 m_a m_a^T) P^H with
// m_a = M^{-1} e_a.  The stationary covariance X = sum_j A^j Qn (A^j)^H
// is summed by doubling (X <- X + A X A^H, A <- A A); S(k) = 1^T X 1.
// Doubling stays well posed where A has a unit-modulus eigenvalue the
// noise does not excite (k = pi on an axis at tau = 1).
//
// One 64-lane workgroup per wave vector; the three Q x Q complex matrices
// live in LDS (17 KB for D3Q19).  FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/fsc.h"
#include "fsc_device.h"

namespace fsc {
namespace {

struct cplx64 {
    double re, im;
};
__device__ __forceinline__ cplx64 cmul(cplx64 a, cplx64 b) {
    return cplx64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx64 cmulc(cplx64 a, cplx64 b) {  // a * conj(b)
    return cplx64{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

struct LinArgs {
    double n0, coupling;  // n0 and G psi0 psi0'
    double mu;            // kBT / c_s^2
    double lam[4];        // per class
    int doublings;
};

// C = A B (all Q x Q), lanes stride over the entries.
template <int Q>
__device__ void matmul(const cplx64 (&a)[Q][Q], const cplx64 (&b)[Q][Q], cplx64 (&c)[Q][Q]) {
    for (int e = threadIdx.x; e < Q * Q; e += 64) {
        const int i = e / Q, l = e % Q;
        cplx64 s{0.0, 0.0};
#pragma unroll
        for (int m = 0; m < Q; ++m) {
            const cplx64 p = cmul(a[i][m], b[m][l]);
            s.re += p.re;
            s.im += p.im;
        }
        c[i][l] = s;
    }
}

// C += A B^H
template <int Q>
__device__ void matmul_add_h(const cplx64 (&a)[Q][Q], const cplx64 (&b)[Q][Q], cplx64 (&c)[Q][Q]) {
    for (int e = threadIdx.x; e < Q * Q; e += 64) {
        const int i = e / Q, l = e % Q;
        cplx64 s = c[i][l];
#pragma unroll
        for (int m = 0; m < Q; ++m) {
            const cplx64 p = cmulc(a[i][m], b[l][m]);
            s.re += p.re;
            s.im += p.im;
        }
        c[i][l] = s;
    }
}

// A(k) and the noise covariance Qn(k) into A and X (T is scratch); ends
// with a barrier.
template <class L, class ST>
__device__ void build_operator(const LinArgs &la, const double (&k)[3], cplx64 (&A)[L::Q][L::Q],
                               cplx64 (&X)[L::Q][L::Q], cplx64 (&T)[L::Q][L::Q]) {
    constexpr int D = L::D, Q = L::Q;
    constexpr double CS2 = 1.0 / 3.0;
    const int lane = threadIdx.x;
    // dF per unit dn: coupling * sum over the full stencil of w e e^{ik.e}
    // = coupling * sum over the half set of 2 i w e sin(k.e)
    double gim[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < ST::NH; ++a) {
        const double kd = k[0] * ST::e(a, 0) + k[1] * ST::e(a, 1) + (D == 3 ? k[2] * ST::e(a, 2) : 0.0);
        const double s = 2.0 * ST::w(a) * sin(kd);
#pragma unroll
        for (int d = 0; d < D; ++d) gim[d] += s * ST::e(a, d);
    }
    cplx64 dF[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dF[d] = cplx64{0.0, la.coupling * gim[d]};
    // column j of A: a unit perturbation of population j through the
    // collision; the post-collision moments go through T (LDS)
    if (lane < Q) {
        const int j = lane;
        cplx64 du[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            du[d] = cplx64{(double(L::c(j, d)) + 0.5 * dF[d].re) / la.n0, 0.5 * dF[d].im / la.n0};
        // c_i . du and c_i . dF of every population, as the equilibrium and
        // source need them
#pragma unroll 1
        for (int a = 0; a < Q; ++a) {
            const double m = double(L::M(a, j));
            cplx64 meq{0.0, 0.0}, src{0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double Mw = double(L::M(a, i)) * L::w(i);
                double cur = 0.0, cui = 0.0, cfr = 0.0, cfi = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const double c = double(L::c(i, d));
                    cur += c * du[d].re;
                    cui += c * du[d].im;
                    cfr += c * dF[d].re;
                    cfi += c * dF[d].im;
                }
                meq.re += Mw * (1.0 + la.n0 * cur / CS2);
                meq.im += Mw * (la.n0 * cui / CS2);
                src.re += Mw * cfr / CS2;
                src.im += Mw * cfi / CS2;
            }
            const int cl = L::cls(a);  // select, not an indexed load (no scratch copy)
            const double lam = cl == 1 ? la.lam[1] : (cl == 2 ? la.lam[2] : (cl == 3 ? la.lam[3] : 1.0));
            T[a][j] = cplx64{m - lam * (m - meq.re) + (1.0 - 0.5 * lam) * src.re,
                             lam * meq.im + (1.0 - 0.5 * lam) * src.im};
        }
        // back-transform f_i = w_i sum_a M_ai ms_a / b_a, then the streaming phase
#pragma unroll 1
        for (int i = 0; i < Q; ++i) {
            cplx64 f{0.0, 0.0};
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const double cf = L::w(i) * double(L::M(a, i)) / moment_norm<L>(a);
                f.re += cf * T[a][j].re;
                f.im += cf * T[a][j].im;
            }
            double ph = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) ph -= double(L::c(i, d)) * k[d];
            A[i][j] = cmul(cplx64{cos(ph), sin(ph)}, f);
        }
    }
    // noise covariance P (sum_a amp_a^2 m_a m_a^T) P^H
    for (int e = lane; e < Q * Q; e += 64) {
        const int i = e / Q, l = e % Q;
        double s = 0.0;
#pragma unroll
        for (int a = D + 1; a < Q; ++a) {
            const double lam = la.lam[L::cls(a)];
            const double amp2 = la.mu * la.n0 * (1.0 - (1.0 - lam) * (1.0 - lam)) / moment_norm<L>(a);
            s += double(L::M(a, i)) * double(L::M(a, l)) * amp2;
        }
        s *= L::w(i) * L::w(l);
        double ph = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) ph += double(L::c(l, d) - L::c(i, d)) * k[d];
        X[i][l] = cplx64{s * cos(ph), s * sin(ph)};
    }
    __syncthreads();
}

// X <- sum_j A^j X (A^j)^H by doubling; A is overwritten.
template <int Q>
__device__ void doubling_sum(const LinArgs &la, cplx64 (&A)[Q][Q], cplx64 (&X)[Q][Q],
                             cplx64 (&T)[Q][Q], double (&red)[64]) {
    const int lane = threadIdx.x;
    for (int it = 0; it < la.doublings; ++it) {
        matmul<Q>(A, X, T);  // T = A X
        __syncthreads();
        matmul_add_h<Q>(T, A, X);  // X += A X A^H
        __syncthreads();
        matmul<Q>(A, A, T);  // T = A A
        __syncthreads();
        double amax = 0.0;
        for (int e = lane; e < Q * Q; e += 64) {
            const cplx64 v = T[e / Q][e % Q];
            A[e / Q][e % Q] = v;
            amax = fmax(amax, fabs(v.re) + fabs(v.im));
        }
        red[lane] = amax;
        __syncthreads();
        // the remaining terms are below 1e-40 of X once A^(2^it) has decayed
        bool done = true;
        for (int q = 0; q < 64; ++q) done = done && (red[q] < 1e-20);
        __syncthreads();
        if (done) break;
    }
}

template <class L, class ST>
__global__ void __launch_bounds__(64) k_linear_sk(LinArgs la, const double *__restrict__ kv,
                                                  int64_t nk, double *__restrict__ out) {
    constexpr int D = L::D, Q = L::Q;
    __shared__ cplx64 A[Q][Q], X[Q][Q], T[Q][Q];
    __shared__ double red[64];
    const int lane = threadIdx.x;
    for (int64_t kid = blockIdx.x; kid < nk; kid += gridDim.x) {
        const double k[3] = {kv[3 * kid], kv[3 * kid + 1], D == 3 ? kv[3 * kid + 2] : 0.0};
        build_operator<L, ST>(la, k, A, X, T);
        doubling_sum<Q>(la, A, X, T, red);
        double s = 0.0;
        for (int e = lane; e < Q * Q; e += 64) s += X[e / Q][e % Q].re;
        red[lane] = s;
        __syncthreads();
        if (lane == 0) {
            double t = 0.0;
            for (int q = 0; q < 64; ++q) t += red[q];
            out[kid] = t;
        }
        __syncthreads();
    }
}

// C(k, tau) = 1^T A^tau X 1 at ascending lags: v = X 1, then v <- A v.
template <class L, class ST>
__global__ void __launch_bounds__(64) k_linear_corr(LinArgs la, const double *__restrict__ kv,
                                                    int64_t nk, const int *__restrict__ lags,
                                                    int nlag, double *__restrict__ out) {
    constexpr int D = L::D, Q = L::Q;
    __shared__ cplx64 A[Q][Q], X[Q][Q], T[Q][Q], A0[Q][Q];
    __shared__ cplx64 v[Q], vn[Q];
    __shared__ double red[64];
    const int lane = threadIdx.x;
    for (int64_t kid = blockIdx.x; kid < nk; kid += gridDim.x) {
        const double k[3] = {kv[3 * kid], kv[3 * kid + 1], D == 3 ? kv[3 * kid + 2] : 0.0};
        build_operator<L, ST>(la, k, A, X, T);
        for (int e = lane; e < Q * Q; e += 64) A0[e / Q][e % Q] = A[e / Q][e % Q];
        __syncthreads();
        doubling_sum<Q>(la, A, X, T, red);
        if (lane < Q) {
            cplx64 t{0.0, 0.0};
            for (int m = 0; m < Q; ++m) {
                t.re += X[lane][m].re;
                t.im += X[lane][m].im;
            }
            v[lane] = t;
        }
        __syncthreads();
        int tau = 0;
        for (int q = 0; q < nlag; ++q) {
            while (tau < lags[q]) {
                if (lane < Q) {
                    cplx64 t{0.0, 0.0};
                    for (int m = 0; m < Q; ++m) {
                        const cplx64 p = cmul(A0[lane][m], v[m]);
                        t.re += p.re;
                        t.im += p.im;
                    }
                    vn[lane] = t;
                }
                __syncthreads();
                if (lane < Q) v[lane] = vn[lane];
                __syncthreads();
                ++tau;
            }
            if (lane == 0) {
                double re = 0.0, im = 0.0;
                for (int m = 0; m < Q; ++m) {
                    re += v[m].re;
                    im += v[m].im;
                }
                out[(kid * nlag + q) * 2] = re;
                out[(kid * nlag + q) * 2 + 1] = im;
            }
            __syncthreads();
        }
    }
}

template <class L, class ST>
hipError_t launch_linear(const LinArgs &la, const double *kv, int64_t nk, double *out, hipStream_t s) {
    const unsigned blocks = unsigned(nk < 65536 ? nk : 65536);
    hipLaunchKernelGGL((k_linear_sk<L, ST>), dim3(blocks), dim3(64), 0, s, la, kv, nk, out);
    return hipGetLastError();
}

template <class L, class ST>
hipError_t launch_corr(const LinArgs &la, const double *kv, int64_t nk, const int *lags, int nlag,
                       double *out, hipStream_t s) {
    const unsigned blocks = unsigned(nk < 65536 ? nk : 65536);
    hipLaunchKernelGGL((k_linear_corr<L, ST>), dim3(blocks), dim3(64), 0, s, la, kv, nk, lags, nlag, out);
    return hipGetLastError();
}

int resolve_linear(const fsc_params *p, LinArgs &la) {
    if (!p || (p->D != 2 && p->D != 3) || (p->stencil != FSC_E4 && p->stencil != FSC_E8) ||
        (p->D == 3 && p->stencil == FSC_E8) || !(p->rho0 > 0.0) || !(p->kBT >= 0.0))
        return FSC_E_INVAL;
    const double lams[3] = {p->lambda_bulk, p->lambda_shear, p->lambda_ghost};
    for (double l : lams)
        if (!(l > 0.0 && l < 2.0)) return FSC_E_INVAL;
    const double CS2 = 1.0 / 3.0;
    double G = p->G;
    if (std::isnan(G)) {
        if (!(p->T_hat > 0.0)) return FSC_E_INVAL;
        G = std::exp(2.0) * CS2 / p->T_hat;
    }
    const double psi0 = std::exp(-1.0 / p->rho0);
    la.n0 = p->rho0;
    la.coupling = G * psi0 * psi0 / (p->rho0 * p->rho0);
    la.mu = p->kBT / CS2;
    la.lam[0] = 1.0;
    la.lam[1] = p->lambda_bulk;
    la.lam[2] = p->lambda_shear;
    la.lam[3] = p->lambda_ghost;
    la.doublings = 48;
    return FSC_OK;
}

}  // namespace
}  // namespace fsc

using namespace fsc;

extern "C" {

int fsc_linear_sk(const fsc_params *p, const double *host_k, int64_t nk, double *host_s,
                  void *stream) {
    LinArgs la;
    if (!host_k || !host_s || nk < 0) return FSC_E_INVAL;
    int rc = resolve_linear(p, la);
    if (rc) return rc;
    if (nk == 0) return FSC_OK;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<double> k3(size_t(nk) * 3, 0.0);
    for (int64_t i = 0; i < nk; ++i)
        for (int d = 0; d < p->D; ++d) k3[3 * i + d] = host_k[p->D * i + d];
    double *dk = nullptr, *ds = nullptr;
    if (hipMalloc(&dk, sizeof(double) * 3 * nk) != hipSuccess ||
        hipMalloc(&ds, sizeof(double) * nk) != hipSuccess) {
        (void)hipGetLastError();
        if (dk) (void)hipFree(dk);
        return FSC_E_OOM;
    }
    hipError_t e = hipMemcpyAsync(dk, k3.data(), sizeof(double) * 3 * nk, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (p->D == 2 && p->stencil == FSC_E4) e = launch_linear<D2Q9, StencilE4_2D>(la, dk, nk, ds, st);
        else if (p->D == 2) e = launch_linear<D2Q9, StencilE8_2D>(la, dk, nk, ds, st);
        else e = launch_linear<D3Q19, StencilE4_3D>(la, dk, nk, ds, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(host_s, ds, sizeof(double) * nk, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dk);
    (void)hipFree(ds);
    return e == hipSuccess ? FSC_OK : FSC_E_HIP;
}

int fsc_linear_corr(const fsc_params *p, const double *host_k, int64_t nk, const int *host_lags,
                    int nlag, double *host_c, void *stream) {
    LinArgs la;
    if (!host_k || !host_lags || !host_c || nk < 0 || nlag < 0) return FSC_E_INVAL;
    int rc = resolve_linear(p, la);
    if (rc) return rc;
    for (int q = 0; q < nlag; ++q)
        if (host_lags[q] < 0 || (q > 0 && host_lags[q] < host_lags[q - 1])) return FSC_E_INVAL;
    if (nk == 0 || nlag == 0) return FSC_OK;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<double> k3(size_t(nk) * 3, 0.0);
    for (int64_t i = 0; i < nk; ++i)
        for (int d = 0; d < p->D; ++d) k3[3 * i + d] = host_k[p->D * i + d];
    double *dk = nullptr, *dc = nullptr;
    int *dl = nullptr;
    if (hipMalloc(&dk, sizeof(double) * 3 * nk) != hipSuccess ||
        hipMalloc(&dc, sizeof(double) * 2 * nk * nlag) != hipSuccess ||
        hipMalloc(&dl, sizeof(int) * nlag) != hipSuccess) {
        (void)hipGetLastError();
        if (dk) (void)hipFree(dk);
        if (dc) (void)hipFree(dc);
        return FSC_E_OOM;
    }
    hipError_t e = hipMemcpyAsync(dk, k3.data(), sizeof(double) * 3 * nk, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dl, host_lags, sizeof(int) * nlag, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (p->D == 2 && p->stencil == FSC_E4) e = launch_corr<D2Q9, StencilE4_2D>(la, dk, nk, dl, nlag, dc, st);
        else if (p->D == 2) e = launch_corr<D2Q9, StencilE8_2D>(la, dk, nk, dl, nlag, dc, st);
        else e = launch_corr<D3Q19, StencilE4_3D>(la, dk, nk, dl, nlag, dc, st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_c, dc, sizeof(double) * 2 * nk * nlag, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dk);
    (void)hipFree(dc);
    (void)hipFree(dl);
    return e == hipSuccess ? FSC_OK : FSC_E_HIP;
}

int fsc_linear_sk_radial(const fsc_params *p, double *host_shell_mean, int64_t *host_count,
                         int nbins, void *stream) {
    if (!p || !host_shell_mean || nbins < 1) return FSC_E_INVAL;
    const int D = p->D, n = p->nx;
    if (n < 2 || p->ny != n || (D == 3 && p->nz != n) || (D == 2 && p->nz != 1)) return FSC_E_INVAL;
    // wave vectors of the fundamental domain of the square / cubic group,
    // 0 <= m_z <= m_y <= m_x <= n/2, each with the number of lattice modes
    // it stands for (sign choices x distinct permutations)
    const int h = n / 2;
    auto signs = [&](int v) { return (v == 0 || (2 * v == n)) ? 1 : 2; };
    auto round_sqrt = [](int64_t m) {
        int64_t b = int64_t(std::sqrt(double(m)));
        while (b * b > m) --b;
        while ((b + 1) * (b + 1) <= m) ++b;
        if (m - b * b > b) ++b;
        return int(b);
    };
    std::vector<double> kv;
    std::vector<int64_t> mult;
    std::vector<int> bin;
    const double two_pi_n = 2.0 * M_PI / n;
    for (int a = 0; a <= h; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= (D == 3 ? b : 0); ++c) {
                const int64_t m2 = int64_t(a) * a + int64_t(b) * b + int64_t(c) * c;
                if (m2 == 0) continue;
                int64_t perms;
                if (D == 2) perms = (a == b) ? 1 : 2;
                else perms = (a == b && b == c) ? 1 : ((a == b || b == c) ? 3 : 6);
                const int64_t mu = perms * signs(a) * signs(b) * (D == 3 ? signs(c) : 1);
                kv.push_back(two_pi_n * a);
                kv.push_back(two_pi_n * b);
                if (D == 3) kv.push_back(two_pi_n * c);
                mult.push_back(mu);
                bin.push_back(round_sqrt(m2));
            }
    const int64_t nk = int64_t(mult.size());
    std::vector<double> S(static_cast<size_t>(nk));
    int rc = fsc_linear_sk(p, kv.data(), nk, S.data(), stream);
    if (rc) return rc;
    std::vector<double> sum(size_t(nbins), 0.0);
    std::vector<int64_t> cnt(size_t(nbins), 0);
    for (int64_t i = 0; i < nk; ++i) {
        if (bin[i] >= nbins) continue;
        sum[bin[i]] += double(mult[i]) * S[i];
        cnt[bin[i]] += mult[i];
    }
    for (int b = 0; b < nbins; ++b) {
        host_shell_mean[b] = cnt[b] ? sum[b] / double(cnt[b]) : 0.0;
        if (host_count) host_count[b] = cnt[b];
    }
    return FSC_OK;
}

}  // extern "C"
