// fsc_step_kernel.h -- the fused time step of the fluctuating Shan-Chen lattice
// Boltzmann equation (Eq. 12 of Lulli et al., arXiv:2212.07848) on gfx950.
//
// One launch advances every replica of an ensemble by one step.  A workgroup
// owns a TX x TY cross-section tile (TY = 1 in 2D) and marches along the
// slowest axis (y in 2D, z in 3D) over H planes:
//
//   for each plane s of the march:
//     pull-load f_i(x - c_i) of plane s + R (R = stencil radius) for the tile
//       and its R-wide cross-section ring, form n, and write
//       dpsi = psi(n) - psi(n0) = psi0 expm1(dn / (n0 n)) into an LDS ring
//       buffer of 2R + 2 planes;
//     barrier;
//     for plane s (populations kept in registers since they were loaded):
//       Shan-Chen force of Eq. (1) from the LDS dpsi stencil, summed as
//         antisymmetric pairs so that a uniform field gives exactly zero;
//       velocity u = (j + F/2)/n, moment-space collision with Guo forcing
//         and Philox/Box-Muller noise on the non-conserved moments;
//       back-transform and store f*_i(x) (pull streaming: the next step reads
//         f*_i(x - c_i)).
//
// Populations are stored as deviations df_i = f_i - w_i n0 (float or double),
// SoA [i][slow][..][x], so that small thermal fluctuations keep their
// precision and every load/store is a coalesced 64-lane access.  Densities and
// the pseudopotential never touch HBM: the halo is recomputed from pulled
// populations (extra reads hit L2), so the algorithmic traffic is one read
// and one write per population per node.
#pragma once

#include "fsc_internal.h"

namespace fsc {


template <class L, class ST, typename real, bool NOISE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY)
    k_step(const RepDesc *__restrict__ reps, const int *__restrict__ tile_begin, int nrep,
           int parity, const uint64_t *__restrict__ step_base, uint32_t step_off) {
    constexpr int D = L::D, Q = L::Q, R = ST::R;
    constexpr int S = 2 * R + 2;                  // LDS planes (one barrier per plane)
    constexpr int EXTX = TX + 2 * R;
    constexpr int RY = (D == 3) ? R : 0;
    constexpr int EXTY = (D == 3) ? TY + 2 * R : 1;
    constexpr int NN = L::NNORM;
    constexpr int NT = TX * TY;
    __shared__ real lds[S][EXTY][EXTX];

    // ---- which replica / tile -------------------------------------------
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_begin[mid] <= lb) lo = mid;
        else hi = mid - 1;
    }
    const RepDesc &d = reps[lo];
    const int nx = d.nx, ny = d.ny, ns = d.ns, plane = d.plane;
    const int64_t N = d.N;
    const int t = lb - d.tile_begin;
    const int tix = t % d.tiles_x;
    const int t2 = t / d.tiles_x;
    const int tiy = t2 % d.tiles_y;
    const int chunk = t2 / d.tiles_y;
    const int s_begin = chunk * d.H;
    const int s_end = min(s_begin + d.H, ns);
    const int x0 = tix * TX, y0 = tiy * TY;
    const int TXe = min(TX, nx - x0);
    const int TYe = (D == 3) ? min(TY, ny - y0) : 1;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const bool active = tx < TXe && ty < TYe;
    const int x = active ? x0 + tx : 0;
    const int y = (D == 3 && active) ? y0 + ty : 0;

    const real *src = static_cast<const real *>(d.buf[parity]);
    real *dst = static_cast<real *>(d.buf[parity ^ 1]);

    const real rho0 = real(d.rho0);
    const real psi0 = real(d.psi0);
    const real G = real(d.G);
    const real inv_rho0 = real(1.0 / d.rho0);

    // cross-section pull offsets of the main node, by (c_x, c_y)
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x + 1 == nx ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1;
    const int yp = y + 1 == ny ? 0 : y + 1;
    auto cross_off = [&](int cxv, int cyv, int xx, int xxm, int xxp, int yy, int yym, int yyp) {
        const int xs = cxv == 1 ? xxm : (cxv == -1 ? xxp : xx);
        if (D == 2) return xs;
        const int ys = cyv == 1 ? yym : (cyv == -1 ? yyp : yy);
        return xs + nx * ys;
    };
    auto plane_off = [&](int p, int cs) { return wrap_any(p - cs, ns) * plane; };
    // marching-axis velocity component and cross-section components
    auto cm = [](int i) { return L::c(i, D - 1); };
    auto c0 = [](int i) { return L::c(i, 0); };
    auto c1 = [](int i) { return D == 3 ? L::c(i, 1) : 0; };

    auto slot = [](int p) { return (p + S) % S; };

    // pseudopotential deviation from a density deviation
    auto dpsi_of = [&](real dn) {
        if constexpr (sizeof(real) == 4) return psi0 * expm1f(dn * inv_rho0 / (rho0 + dn));
        else return psi0 * expm1(dn * inv_rho0 / (rho0 + dn));
    };

    // ring node k of the extended cross-section -> (ex, ey)
    const int ringW = TXe + 2 * R;
    const int nring = (D == 2) ? 2 * R : ringW * (TYe + 2 * R) - TXe * TYe;
    auto ring_pos = [&](int k, int &ex, int &ey) {
        if (D == 2) {
            ey = 0;
            ex = k < R ? k : TXe + k;
            return;
        }
        const int band = ringW * R;
        if (k < band) {
            ey = k / ringW;
            ex = k % ringW;
        } else if (k < 2 * band) {
            const int kk = k - band;
            ey = TYe + R + kk / ringW;
            ex = kk % ringW;
        } else {
            const int kk = k - 2 * band;
            ey = R + kk / (2 * R);
            const int c = kk % (2 * R);
            ex = c < R ? c : TXe + c;
        }
    };

    // computes plane p: main-node populations into fmain (if active) and the
    // dpsi of the whole extended cross-section into LDS
    auto do_plane = [&](int p, real (&fmain)[Q]) {
        const int po[3] = {plane_off(p, -1), plane_off(p, 0), plane_off(p, 1)};
        const int sl = slot(p);
        if (active) {
            real dn = real(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const real *pi = src + int64_t(i) * N;
                fmain[i] = pi[po[cm(i) + 1] + cross_off(c0(i), c1(i), x, xm, xp, y, ym, yp)];
                dn += fmain[i];
            }
            lds[sl][ty + RY][tx + R] = dpsi_of(dn);
        }
        for (int k = tid; k < nring; k += NT) {
            int ex, ey;
            ring_pos(k, ex, ey);
            const int xr = wrap_any(x0 - R + ex, nx);
            const int yr = (D == 3) ? wrap_any(y0 - RY + ey, ny) : 0;
            const int xrm = xr == 0 ? nx - 1 : xr - 1;
            const int xrp = xr + 1 == nx ? 0 : xr + 1;
            const int yrm = yr == 0 ? ny - 1 : yr - 1;
            const int yrp = yr + 1 == ny ? 0 : yr + 1;
            real dn = real(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const real *pi = src + int64_t(i) * N;
                dn += pi[po[cm(i) + 1] + cross_off(c0(i), c1(i), xr, xrm, xrp, yr, yrm, yrp)];
            }
            lds[sl][ey][ex] = dpsi_of(dn);
        }
    };

    const uint64_t step = step_base[0] + step_off;
    const uint32_t step32 = uint32_t(step);

    real fr[R + 1][Q];
#pragma unroll
    for (int k = -R; k < R; ++k) {
        real tmp[Q];
        do_plane(s_begin + k, tmp);
        if (k >= 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) fr[k][i] = tmp[i];
        }
    }

    for (int s = s_begin; s < s_end; ++s) {
        do_plane(s + R, fr[R]);
        __syncthreads();

        if (active) {
            int sl[2 * R + 1];
#pragma unroll
            for (int k = -R; k <= R; ++k) sl[k + R] = slot(s + k);

            // ---- Shan-Chen force, Eq. (1), as antisymmetric pairs ----------
            real g[3] = {real(0), real(0), real(0)};
#pragma unroll
            for (int a = 0; a < ST::NH; ++a) {
                const int ex = ST::e(a, 0);
                const int ey = D == 3 ? ST::e(a, 1) : 0;
                const int es = ST::e(a, D - 1);
                const real vp = lds[sl[R + es]][ty + RY + ey][tx + R + ex];
                const real vm = lds[sl[R - es]][ty + RY - ey][tx + R - ex];
                const real diff = vp - vm;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const int eq = ST::e(a, q);
                    if (eq != 0) g[q] += real(ST::w(a) * eq) * diff;
                }
            }
            const real pre = G * (psi0 + lds[sl[R]][ty + RY][tx + R]);
            real F[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) F[q] = pre * g[q];

            // ---- moments of the pulled populations -------------------------
            const real(&f)[Q] = fr[0];
            real dn = real(0);
            real j[3] = {real(0), real(0), real(0)};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                dn += f[i];
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    if (L::c(i, q) == 1) j[q] += f[i];
                    if (L::c(i, q) == -1) j[q] -= f[i];
                }
            }
            const real rho = rho0 + dn;
            const real inv_rho = real(1) / rho;
            real u[3] = {real(0), real(0), real(0)};
#pragma unroll
            for (int q = 0; q < D; ++q) u[q] = (j[q] + real(0.5) * F[q]) * inv_rho;

            real z[NN];
            real srho = real(0);
            if constexpr (NOISE) {
                const uint32_t node = uint32_t(x + nx * (y + (D == 3 ? ny * s : s)));
                node_normals<NN, real>(node, step32, d.seed_hi, d.key0, d.key1, z);
                srho = sqrt(rho);
            }

            // ---- collision in moment space ---------------------------------
            real ms[Q];
            ms[0] = dn;
#pragma unroll
            for (int q = 0; q < D; ++q) ms[1 + q] = j[q] + F[q];
#pragma unroll
            for (int a = D + 1; a < Q; ++a) {
                real m = real(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const int c = L::M(a, i);
                    if (c == 1) m += f[i];
                    else if (c == -1) m -= f[i];
                    else if (c != 0) m += real(c) * f[i];
                }
                const real lam = real(d.lam[a]);
                real out;
                if (L::cls(a) == 3) {
                    out = (real(1) - lam) * m;
                } else {
                    real uAu = real(0), uAF = real(0);
#pragma unroll
                    for (int p = 0; p < D; ++p)
#pragma unroll
                        for (int q = 0; q < D; ++q) {
                            const double A = L::A(a, p, q);
                            if (A != 0.0) {
                                uAu += real(A) * u[p] * u[q];
                                uAF += real(A) * u[p] * F[q];
                            }
                        }
                    const real meq = rho * uAu;
                    out = m - lam * (m - meq) + (real(1) - real(0.5) * lam) * (real(2) * uAF);
                }
                if constexpr (NOISE) out += real(d.amp[a]) * srho * z[a - D - 1];
                ms[a] = out;
            }

            // ---- back-transform and store ----------------------------------
            const int sp = s * plane + (D == 3 ? x + nx * y : x);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                real v = real(0);
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    const int c = L::M(a, i);
                    if (c != 0) v += real(back_coef<L>(i, a)) * ms[a];
                }
                dst[int64_t(i) * N + sp] = v;
            }
        }

#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int i = 0; i < Q; ++i) fr[k][i] = fr[k + 1][i];
    }
}

template <class L, class ST, typename real, bool NOISE, int TX, int TY>
inline hipError_t launch_one(const StepLaunch &P, hipStream_t s) {
    hipLaunchKernelGGL((k_step<L, ST, real, NOISE, TX, TY>), dim3(P.total_tiles), dim3(TX * TY),
                       0, s, P.reps, P.tile_begin, P.nrep, P.parity, P.step_base, P.step_off);
    return hipGetLastError();
}

template <class L, class ST, int TX, int TY>
inline hipError_t launch_prec(const StepLaunch &P, hipStream_t s) {
    if (P.precision == 0)
        return P.noise ? launch_one<L, ST, float, true, TX, TY>(P, s)
                       : launch_one<L, ST, float, false, TX, TY>(P, s);
    return P.noise ? launch_one<L, ST, double, true, TX, TY>(P, s)
                   : launch_one<L, ST, double, false, TX, TY>(P, s);
}

}  // namespace fsc
