// fsc_step_kernel.h -- the fused time step of the fluctuating Shan-Chen
// lattice Boltzmann equation (Eq. 12 of Lulli et al., arXiv:2212.07848) on
// gfx950.
//
// One launch advances every replica of an ensemble by one step.  A workgroup
// owns a TX x TY cross-section tile (TY = 1 in 2D) and marches along the
// slowest axis (y in 2D, z in 3D) over H planes:
//
//   for each plane s of the march (upwards in even chunks, downwards in odd):
//     wait for the pulled populations f_i(x - c_i) of plane s + R (R = stencil
//       radius, ahead in march direction; loads issued PF planes earlier, or
//       just now when PF = 0), form
//       n and write
//       dpsi = psi(n) - psi(n0) = psi0 expm1(dn / (n0 n)) for the tile and its
//       R-wide cross-section ring into an LDS ring buffer of 2R + 2 planes;
//     issue the loads of plane s + R + PF (software prefetch);
//     barrier;
//     for plane s (populations held in a register ring since they arrived):
//       Shan-Chen force of Eq. (1) from the LDS dpsi stencil, summed as
//         antisymmetric pairs so that a uniform field gives exactly zero;
//       u = (j + F/2)/n, moment-space collision with Guo forcing and
//         Philox/Box-Muller noise on the non-conserved moments;
//       back-transform and store f*_i(x) (pull streaming: the next step reads
//         f*_i(x - c_i)).
//
// Populations are stored as deviations df_i = f_i - w_i n0 (float or double),
// SoA [i][slow][..][x], so that small thermal fluctuations keep their
// precision and every access is a coalesced wave-wide transaction.  Densities
// and the pseudopotential never touch HBM: the halo is recomputed from pulled
// populations (the extra reads hit L2), so the algorithmic traffic is one
// read and one write per population per node.  Loads and stores use a
// wave-uniform 64-bit base (SGPR pair) plus a per-lane 32-bit byte offset that
// is constant along the march, so the addressing costs no vector ALU work.
#pragma once

#include "fsc_internal.h"

namespace fsc {

// Raw buffer accesses: a buffer resource (base, byte size) in SGPRs, a
// wave-uniform byte offset in an SGPR and a per-lane byte offset in a VGPR.
// Out-of-range lanes read 0 and drop writes.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int BUF_DWORD3 = 0x00020000;  // raw 32-bit buffer (gfx9 family)

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint64_t bytes) {
    const int n = bytes >= 0xffffffffull ? int(0xffffffff) : int(uint32_t(bytes));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, n, BUF_DWORD3);
}
#ifndef FSC_LOAD_POLICY
#define FSC_LOAD_POLICY 0
#endif
template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, FSC_LOAD_POLICY));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double,
                              __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, FSC_LOAD_POLICY));
}
// Cache policy of the population stores: 2 sets the non-temporal bit on
// gfx950 (the stored planes are not read again within the step; measured a
// few percent faster than the default policy, 0, for the single-step kernels
// and the two-step kernels with an edge wave).  The in-tile-halo two-step
// kernels store with the default policy, which measured 4-5% faster for them.
#ifndef FSC_STORE_POLICY
#define FSC_STORE_POLICY 2
#endif
template <int POL = FSC_STORE_POLICY>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, POL);
}
template <int POL = FSC_STORE_POLICY>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, POL);
}

// Fused multiply-add, written out wherever the step arithmetic uses one.  The
// step kernels are compiled with FP contraction off (-ffp-contract=off and the
// pragma below), so that no kernel rounds a product differently from another:
// left to itself the compiler fuses multiplies and adds differently in
// different kernels, and the tilings would then differ in the last bit.
#pragma clang fp contract(off)
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
// exp(x) - 1 in FP32 for the pseudopotential: for |x| < 1/2 the Taylor series
// through x^8 (truncation below 1.5e-8 relative, a quarter of an FP32 ulp),
// else the hardware exp2 minus one, where exp(x) is far enough from 1 that the
// subtraction loses at most a few ulp (about 2e-7 relative over the range at
// most).  Both branches are evaluated and one is selected, which is cheaper
// than the library's general expm1f with its special cases (the argument here
// is bounded above by 1 / n0 and NaN propagates).
__device__ __forceinline__ float fexpm1(float x) {
    float q = 1.0f / 40320.0f;
    q = fmadd(q, x, 1.0f / 5040.0f);
    q = fmadd(q, x, 1.0f / 720.0f);
    q = fmadd(q, x, 1.0f / 120.0f);
    q = fmadd(q, x, 1.0f / 24.0f);
    q = fmadd(q, x, 1.0f / 6.0f);
    q = fmadd(q, x, 0.5f);
    const float taylor = fmadd(x * x, q, x);
    const float viaexp = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.0f;
    return __builtin_fabsf(x) < 0.5f ? taylor : viaexp;
}
__device__ __forceinline__ double fexpm1(double x) { return expm1(x); }

// ---------------------------------------------------------------------------
// D2Q9 collision, written out on the weight-orthogonal basis
//   1, cx, cy, 3c^2-2, cx^2-cy^2, cxcy, (3c^2-4)cx, (3c^2-4)cy, 9c^4-15c^2+2
// (norms b = 1, 1/3, 1/3, 4, 4/9, 1/9, 2/3, 2/3, 16).  The equilibrium and
// Guo-source moments of the second-order rows are rho u.A.u and 2 u.A.F; the
// kinetic rows have none.  In: pulled deviations f (overwritten by the
// post-collision deviations), force F, noise normals z (6).
// ---------------------------------------------------------------------------
template <typename real, bool NOISE>
__device__ __forceinline__ void collide_d2q9(real (&f)[9], real rho0, const real F[3],
                                             const real (&lc)[4], const real (&ac)[4],
                                             const real (&z)[6]) {
    const real s13 = f[1] + f[3], d13 = f[1] - f[3];
    const real s24 = f[2] + f[4], d24 = f[2] - f[4];
    const real s57 = f[5] + f[7], d57 = f[5] - f[7];
    const real s68 = f[6] + f[8], d68 = f[6] - f[8];
    const real Ax = s13 + s24, Dg = s57 + s68;
    const real dn = f[0] + Ax + Dg;
    const real u1 = d57 - d68, u2 = d57 + d68;
    const real jx = d13 + u1, jy = d24 + u2;
    const real m3 = fmadd(real(-2), f[0], fmadd(real(4), Dg, Ax));
    const real m4 = s13 - s24;
    const real m5 = s57 - s68;
    const real m6 = fmadd(real(2), u1, -d13);
    const real m7 = fmadd(real(2), u2, -d24);
    const real m8 = fmadd(real(8), Dg, fmadd(real(-4), Ax, real(2) * f[0]));

    const real rho = rho0 + dn;
    const real ir = fast_rcp(rho);
    const real ux = fmadd(real(0.5), F[0], jx) * ir;
    const real uy = fmadd(real(0.5), F[1], jy) * ir;
    const real uyy = uy * uy, uxy = ux * uy;
    const real uFy = uy * F[1];

    // noise: row a of class c adds sqrt(b_a) amp_c sqrt(n) xi_a
    constexpr RowScale<D2Q9> sb{};
    const real sr = NOISE ? fsqrt(rho) : real(0);
    // second-moment row a: equilibrium rho q (q its quadratic form of u), Guo
    // source ks s (ks: the row's source constant times 1 - l/2, a per-class
    // constant formed outside the node loop)
    auto relax = [&](int a, real m, real q, real ks, real s, real zz) {
        const real l = lc[D2Q9::cls(a)];
        real o = fmadd(l, fmadd(rho, q, -m), m);
        o = fmadd(ks, s, o);
        if constexpr (NOISE) o = fmadd(real(sb.v[a]) * ac[D2Q9::cls(a)] * sr, zz, o);
        return o;
    };
    auto ghost = [&](int a, real m, real zz) {
        real o = (real(1) - lc[3]) * m;
        if constexpr (NOISE) o = fmadd(real(sb.v[a]) * ac[3] * sr, zz, o);
        return o;
    };
    const real k1 = fmadd(real(-0.5), lc[1], real(1)), k2 = fmadd(real(-0.5), lc[2], real(1));
    // post-collision moments o_a; n_a = o_a / b_a enters the back-transform
    // through the factors below (b_3..b_8 = 4, 4/9, 1/9, 2/3, 2/3, 16)
    const real o3 = relax(3, m3, real(3) * fmadd(ux, ux, uyy), real(6) * k1, fmadd(ux, F[0], uFy), z[0]);
    const real o4 = relax(4, m4, fmadd(ux, ux, -uyy), real(2) * k2, fmadd(ux, F[0], -uFy), z[1]);
    const real o5 = relax(5, m5, uxy, k2, fmadd(ux, F[1], uy * F[0]), z[2]);
    const real o6 = ghost(6, m6, z[3]);
    const real o7 = ghost(7, m7, z[4]);
    const real o8 = ghost(8, m8, z[5]);

    // back-transform f_i = w_i sum_a M_ai n_a, the weights folded in: with
    // t = j + F (the conserved momentum over b_1 = 1/3 is 3 t),
    // w_1 (3 t_x - 1.5 o_6) = t_x / 3 - o_6 / 6 and w_5 (3 t_x + 3 o_6) = (t_x + o_6) / 12
    const real n0 = dn;
    const real tx = jx + F[0], ty = jy + F[1];
    const real w0 = real(4.0 / 9.0), w1 = real(1.0 / 9.0), w5 = real(1.0 / 36.0);
    f[0] = w0 * fmadd(real(0.125), o8, fmadd(real(-0.5), o3, n0));
    const real ba = fmadd(real(-0.25), o8, fmadd(real(0.25), o3, n0));
    const real ap = fmadd(real(2.25), o4, ba), am = fmadd(real(-2.25), o4, ba);
    const real px = fmadd(real(-1.0 / 6.0), o6, tx * real(1.0 / 3.0));
    const real py = fmadd(real(-1.0 / 6.0), o7, ty * real(1.0 / 3.0));
    f[1] = fmadd(w1, ap, px);
    f[3] = fmadd(w1, ap, -px);
    f[2] = fmadd(w1, am, py);
    f[4] = fmadd(w1, am, -py);
    const real bd = fmadd(real(0.5), o8, n0 + o3);
    const real bp = fmadd(real(9), o5, bd), bm = fmadd(real(-9), o5, bd);
    const real X = tx + o6, Y = ty + o7;
    const real XpY = (X + Y) * real(1.0 / 12.0), XmY = (X - Y) * real(1.0 / 12.0);
    f[5] = fmadd(w5, bp, XpY);
    f[7] = fmadd(w5, bp, -XpY);
    f[6] = fmadd(w5, bm, -XmY);
    f[8] = fmadd(w5, bm, XmY);
}

// ---------------------------------------------------------------------------
// D3Q19 collision on the weight-orthogonal basis (rows as in fsc_device.h),
// written with the sums s and differences d of opposite populations: even
// rows see only sums, odd rows only differences, and the back-transform
// gives each opposite pair as w (E +- O) from its even and odd parts.
// ---------------------------------------------------------------------------
template <typename real, bool NOISE>
__device__ __forceinline__ void collide_d3q19(real (&f)[19], real rho0, const real F[3],
                                              const real (&lc)[4], const real (&ac)[4],
                                              const real (&z)[15]) {
    const real sx = f[1] + f[2], dx = f[1] - f[2];
    const real sy = f[3] + f[4], dy = f[3] - f[4];
    const real sz = f[5] + f[6], dz = f[5] - f[6];
    const real S1 = f[7] + f[8], D1 = f[7] - f[8];      // +-(1, 1, 0)
    const real S2 = f[9] + f[10], D2 = f[9] - f[10];    // +-(1,-1, 0)
    const real S3 = f[11] + f[12], D3 = f[11] - f[12];  // +-(1, 0, 1)
    const real S4 = f[13] + f[14], D4 = f[13] - f[14];  // +-(1, 0,-1)
    const real S5 = f[15] + f[16], D5 = f[15] - f[16];  // +-(0, 1, 1)
    const real S6 = f[17] + f[18], D6 = f[17] - f[18];  // +-(0, 1,-1)
    const real Sxy = S1 + S2, Sxz = S3 + S4, Syz = S5 + S6;
    const real Sd = Sxy + Sxz + Syz, Sa = sx + sy + sz;
    const real dn = f[0] + Sa + Sd;
    const real Dx4 = D1 + D2 + D3 + D4;
    const real Dy4 = D1 - D2 + D5 + D6;
    const real Dz4 = D3 - D4 + D5 - D6;
    const real jx = dx + Dx4, jy = dy + Dy4, jz = dz + Dz4;
    const real m4 = Sd - f[0];
    const real m5 = fmadd(real(-2), Syz, fmadd(real(2), sx, -sy) - sz + Sxy + Sxz);
    const real m6 = sy - sz + Sxy - Sxz;
    const real m7 = S1 - S2, m8 = S5 - S6, m9 = S3 - S4;
    const real m10 = fmadd(real(-2), dx, Dx4), m11 = fmadd(real(-2), dy, Dy4), m12 = fmadd(real(-2), dz, Dz4);
    const real m13 = D1 + D2 - D3 - D4;
    const real m14 = D2 - D1 + D5 + D6;
    const real m15 = D3 - D4 - D5 + D6;
    const real m16 = fmadd(real(-2), Sa, f[0]) + Sd;
    const real m17 = fmadd(real(-2), Syz, fmadd(real(-2), sx, sy + sz) + Sxy + Sxz);
    const real m18 = sz - sy + Sxy - Sxz;

    const real rho = rho0 + dn;
    const real ir = fast_rcp(rho);
    const real ux = fmadd(real(0.5), F[0], jx) * ir;
    const real uy = fmadd(real(0.5), F[1], jy) * ir;
    const real uz = fmadd(real(0.5), F[2], jz) * ir;
    const real uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const real uFx = ux * F[0], uFy = uy * F[1], uFz = uz * F[2];

    constexpr RowScale<D3Q19> sb{};
    real sa[4] = {real(0), real(0), real(0), real(0)};
    if constexpr (NOISE) {
        const real sr = fsqrt(rho);
        sa[1] = ac[1] * sr;
        sa[2] = ac[2] * sr;
        sa[3] = ac[3] * sr;
    }
    auto relax = [&](int a, real m, real meq, real src, real zz) {
        const real l = lc[D3Q19::cls(a)];
        real o = fmadd(l, meq - m, m);
        o = fmadd(fmadd(real(-0.5), l, real(1)), src, o);
        if constexpr (NOISE) o = fmadd(real(sb.v[a]) * sa[D3Q19::cls(a)], zz, o);
        return o;
    };
    auto ghost = [&](int a, real m, real zz) {
        real o = (real(1) - lc[3]) * m;
        if constexpr (NOISE) o = fmadd(real(sb.v[a]) * sa[3], zz, o);
        return o;
    };
    // conserved moments divided by b_a; the others as o_a, with n_a = o_a / b_a
    // entering the back-transform through the factors below (b_4..b_18 =
    // 2/3, 4/3, 4/9, 1/9 (3), 2/3 (3), 2/9 (3), 2, 4/3, 4/9)
    const real n0 = dn;
    const real n1 = (jx + F[0]) * real(3), n2 = (jy + F[1]) * real(3), n3 = (jz + F[2]) * real(3);
    const real o4 = relax(4, m4, rho * fmadd(ux, ux, fmadd(uy, uy, uzz)),
                          real(2) * fmadd(ux, F[0], fmadd(uy, F[1], uFz)), z[0]);
    const real o5 = relax(5, m5, rho * fmadd(real(2), uxx, -uyy - uzz),
                          real(2) * fmadd(real(2), uFx, -uFy - uFz), z[1]);
    const real o6 = relax(6, m6, rho * fmadd(uy, uy, -uzz), real(2) * fmadd(uy, F[1], -uFz), z[2]);
    const real o7 = relax(7, m7, rho * ux * uy, fmadd(ux, F[1], uy * F[0]), z[3]);
    const real o8 = relax(8, m8, rho * uy * uz, fmadd(uy, F[2], uz * F[1]), z[4]);
    const real o9 = relax(9, m9, rho * uz * ux, fmadd(uz, F[0], ux * F[2]), z[5]);
    const real o10 = ghost(10, m10, z[6]);
    const real o11 = ghost(11, m11, z[7]);
    const real o12 = ghost(12, m12, z[8]);
    const real o13 = ghost(13, m13, z[9]);
    const real o14 = ghost(14, m14, z[10]);
    const real o15 = ghost(15, m15, z[11]);
    const real o16 = ghost(16, m16, z[12]);
    const real o17 = ghost(17, m17, z[13]);
    const real o18 = ghost(18, m18, z[14]);

    // back-transform f_i = w_i sum_a M_ai n_a, pairwise
    const real w0 = real(1.0 / 3.0), w1 = real(1.0 / 18.0), w2 = real(1.0 / 36.0);
    f[0] = w0 * fmadd(real(0.5), o16, fmadd(real(-1.5), o4, n0));
    const real e0 = n0 - o16;
    const real p517 = o5 - o17, q517 = o5 + o17, p618 = o6 - o18, q618 = o6 + o18;
    const real Ex = fmadd(real(1.5), p517, e0), Ox = fmadd(real(-3), o10, n1);
    const real eyz = fmadd(real(-0.75), p517, e0);
    const real Ey = fmadd(real(2.25), p618, eyz), Oy = fmadd(real(-3), o11, n2);
    const real Ez = fmadd(real(-2.25), p618, eyz), Oz = fmadd(real(-3), o12, n3);
    f[1] = w1 * (Ex + Ox);
    f[2] = w1 * (Ex - Ox);
    f[3] = w1 * (Ey + Oy);
    f[4] = w1 * (Ey - Oy);
    f[5] = w1 * (Ez + Oz);
    f[6] = w1 * (Ez - Oz);
    const real ed = fmadd(real(0.5), o16, fmadd(real(1.5), o4, n0));
    const real e5 = fmadd(real(0.75), q517, ed);
    const real exy = fmadd(real(2.25), q618, e5);    // pairs 1, 2 (before the +-n7 term)
    const real exz = fmadd(real(-2.25), q618, e5);   // pairs 3, 4 (+-n9)
    const real eyz2 = fmadd(real(-1.5), q517, ed);   // pairs 5, 6 (+-n8)
    const real E1 = fmadd(real(9), o7, exy), E2 = fmadd(real(-9), o7, exy);
    const real E3 = fmadd(real(9), o9, exz), E4 = fmadd(real(-9), o9, exz);
    const real E5 = fmadd(real(9), o8, eyz2), E6 = fmadd(real(-9), o8, eyz2);
    const real ax = fmadd(real(1.5), o10, n1), ay = fmadd(real(1.5), o11, n2), az = fmadd(real(1.5), o12, n3);
    const real O1 = fmadd(real(4.5), o13 - o14, ax + ay);
    const real O2 = fmadd(real(4.5), o13 + o14, ax - ay);
    const real O3 = fmadd(real(4.5), o15 - o13, ax + az);
    const real O4 = fmadd(real(-4.5), o13 + o15, ax - az);
    const real O5 = fmadd(real(4.5), o14 - o15, ay + az);
    const real O6 = fmadd(real(4.5), o14 + o15, ay - az);
    f[7] = w2 * (E1 + O1);
    f[8] = w2 * (E1 - O1);
    f[9] = w2 * (E2 + O2);
    f[10] = w2 * (E2 - O2);
    f[11] = w2 * (E3 + O3);
    f[12] = w2 * (E3 - O3);
    f[13] = w2 * (E4 + O4);
    f[14] = w2 * (E4 - O4);
    f[15] = w2 * (E5 + O5);
    f[16] = w2 * (E5 - O5);
    f[17] = w2 * (E6 + O6);
    f[18] = w2 * (E6 - O6);
}

// ---------------------------------------------------------------------------
// The step kernel.
// ---------------------------------------------------------------------------
// WIDE: the population buffers reach 4 GiB, and each population is addressed
// through a buffer resource of its own (a separate instantiation, so that the
// common form keeps its registers).
template <class L, class ST, typename real, bool NOISE, int TX, int TY, int PF = 2, bool WIDE = false>
__global__ void __launch_bounds__(TX *TY)
    k_step(const RepDesc *__restrict__ reps, const int *__restrict__ tile_begin, int nrep,
           int parity, const uint64_t *__restrict__ step_base, uint32_t step_off) {
    constexpr int D = L::D, Q = L::Q, R = ST::R;
    constexpr int S = 2 * R + 2;                  // LDS planes (one barrier per plane)
    constexpr int NSLOT = R + 1 + PF;             // register ring of pulled planes
    constexpr int EXTX = TX + 2 * R;
    constexpr int RY = (D == 3) ? R : 0;
    constexpr int EXTY = (D == 3) ? TY + 2 * R : 1;
    constexpr int NN = L::NNORM;
    constexpr int NT = TX * TY;
    constexpr int MAXRING = (D == 2) ? 2 * R : (TX + 2 * R) * (TY + 2 * R) - TX * TY;
    static_assert(MAXRING <= NT, "one ring node per thread at most");
    constexpr uint32_t ES = sizeof(real);
    __shared__ real lds[S][EXTY][EXTX];
#ifdef FSC_LDS_POISON
    lds_poison(&lds[0][0][0], S * EXTY * EXTX);
    __syncthreads();
#endif

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
    const bool active = (tid % TX) < TXe && (tid / TX) < TYe;
    // Lanes past a ragged edge work on the last valid node of the tile: they
    // load, compute and store exactly what that node's own lane does (the
    // duplicate stores carry identical bytes), so the loads, the collision and
    // the stores need no branch; only their LDS writes are skipped.
    const int tx = min(tid % TX, TXe - 1), ty = min(tid / TX, TYe - 1);

    const uint64_t buf_bytes = uint64_t(Q) * uint64_t(d.N) * sizeof(real);
    const rsrc_t src = make_rsrc(d.buf[parity], buf_bytes);
    const rsrc_t dst = make_rsrc(d.buf[parity ^ 1], buf_bytes);
    // one population is below 4 GiB (checked on the host); a buffer of 4 GiB
    // or more is addressed with one resource per population, so that every
    // byte offset stays 32-bit
    const uint32_t pop_bytes = uint32_t(d.N) * ES;
    constexpr bool wide = WIDE;
    const uint64_t pop_bytes64 = uint64_t(d.N) * ES;
    auto pop_rsrc = [&](const void *base, int i) {
        return make_rsrc(static_cast<const char *>(base) + uint64_t(i) * pop_bytes64, pop_bytes64);
    };

    constexpr bool F32 = sizeof(real) == 4;
    const real rho0 = F32 ? real(d.rho0f) : real(d.rho0);
    const real psi0 = F32 ? real(d.psi0f) : real(d.psi0);
    const real G = F32 ? real(d.Gf) : real(d.G);
    const real inv_rho0 = F32 ? real(d.inv_rho0f) : real(1.0 / d.rho0);
    real lc[4], ac[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lc[k] = F32 ? real(d.lamcf[k]) : real(d.lamc[k]);
        // FP32: the normals come in units of BM_SCALE (see box_muller)
        ac[k] = F32 ? real(d.ampcf[k] * BM_SCALE) : real(d.ampc[k]);
    }

    // ---- per-lane pull offsets (bytes, within a plane), by (c_x, c_y) ------
    auto make_offsets = [&](int xx, int yy, uint32_t (&xo)[3][3]) {
        const int xm = xx == 0 ? nx - 1 : xx - 1, xp = xx + 1 == nx ? 0 : xx + 1;
        const int ym = yy == 0 ? ny - 1 : yy - 1, yp = yy + 1 == ny ? 0 : yy + 1;
        const int xs[3] = {xp, xx, xm};  // index c + 1 -> x - c
        const int ys[3] = {yp, yy, ym};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                xo[a][b] = uint32_t(D == 3 ? xs[b] + nx * ys[a] : xs[b]) * ES;
    };
    // main node
    const int x = x0 + tx;
    const int y = D == 3 ? y0 + ty : 0;
    uint32_t xo_m[3][3];
    make_offsets(x, y, xo_m);
    // ring node (extended cross-section, outside the tile), at most one per thread
    const int ringW = TXe + 2 * R;
    const int nring = (D == 2) ? 2 * R : ringW * (TYe + 2 * R) - TXe * TYe;
    const bool has_ring = tid < nring;
    int rex = 0, rey = 0;
    if (has_ring) {
        const int k = tid;
        if (D == 2) {
            rex = k < R ? k : TXe + k;
        } else {
            const int band = ringW * R;
            if (k < band) {
                rey = k / ringW;
                rex = k % ringW;
            } else if (k < 2 * band) {
                const int kk = k - band;
                rey = TYe + R + kk / ringW;
                rex = kk % ringW;
            } else {
                const int kk = k - 2 * band;
                rey = R + kk / (2 * R);
                const int c = kk % (2 * R);
                rex = c < R ? c : TXe + c;
            }
        }
    }
    uint32_t xo_r[3][3];
    make_offsets(has_ring ? wrap_any(x0 - R + rex, nx) : 0,
                 (D == 3 && has_ring) ? wrap_any(y0 - RY + rey, ny) : 0, xo_r);
    // Which lanes load the ring plane.  FP32: the lanes with a ring node.
    // FP64: every lane (the others load node (0, 0), an in-range offset, and
    // discard it), so that the ring registers are never written under a
    // partial execution mask -- the FP64 kernels run close to the register
    // limit, where the FP64 D3Q19 form with prefetch once gave wrong values
    // in lanes without a ring node.
    const bool ring_load = sizeof(real) == 8 || has_ring;

    const uint32_t pbytes = uint32_t(plane) * ES;
    auto cm = [](int i) { return L::c(i, D - 1); };
    auto c0 = [](int i) { return L::c(i, 0); };
    auto c1 = [](int i) { return D == 3 ? L::c(i, 1) : 0; };
    auto slot = [](int p) { return (p + S) % S; };

    // loads of plane p (pulled) for the lane offsets xo
    // plane index modulo ns; the planes touched lie within a few planes of
    // the chunk, so this costs a compare or two (a short loop only when the
    // lattice is thinner than the stencil and prefetch reach)
    auto wrap_plane = [ns](int v) {
        while (v < 0) v += ns;
        while (v >= ns) v -= ns;
        return v;
    };
    auto load_plane = [&](int p, const uint32_t (&xo)[3][3], real (&out)[Q]) {
        const int pc = wrap_plane(p);
        const int pp = pc + 1 == ns ? 0 : pc + 1, pm = pc == 0 ? ns - 1 : pc - 1;
        const uint32_t pb[3] = {uint32_t(pp) * pbytes, uint32_t(pc) * pbytes, uint32_t(pm) * pbytes};
        if constexpr (wide) {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                out[i] = bload<real>(pop_rsrc(d.buf[parity], i), xo[c1(i) + 1][c0(i) + 1], pb[cm(i) + 1]);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                out[i] = bload<real>(src, xo[c1(i) + 1][c0(i) + 1], uint32_t(i) * pop_bytes + pb[cm(i) + 1]);
        }
    };
    auto dpsi_of = [&](const real (&fv)[Q]) {
        real dn = real(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) dn += fv[i];
        return psi0 * fexpm1(dn * inv_rho0 * fast_rcp(rho0 + dn));
    };
    auto put_psi = [&](int p, const real (&fm)[Q], const real (&fr)[Q]) {
        const int sl = slot(p);
        if (active) lds[sl][ty + RY][tx + R] = dpsi_of(fm);
        if (has_ring) lds[sl][rey][rex] = dpsi_of(fr);
    };

    const uint64_t step = step_base[0] + step_off;
    const uint32_t step32 = uint32_t(step);

    // ---- march order ---------------------------------------------------------
    // Odd chunks march downwards, so two neighbouring chunks reach their shared
    // boundary planes at the same time (both at the start or both at the end of
    // their march) and the halo planes one of them re-reads are still in L2.
    const int dir = (chunk & 1) ? -1 : 1;
    const int len = s_end - s_begin;
    const int first = dir > 0 ? s_begin : s_end - 1;

    // ---- prologue: planes first - dir R .. first + dir (R - 1) ---------------
    real F[NSLOT][Q];
    // The ring plane is prefetched one plane ahead unless the main planes are
    // not prefetched either (PF = 0, the register-lean form).
    constexpr bool RING_PF = PF > 0;
    // Ring-plane registers.  Lanes without a ring node never load them; they
    // still get a defined value, so that no lane carries an undefined value
    // through the march loop.
    real RG[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) RG[i] = real(0);
#pragma unroll
    for (int k = -R; k < R; ++k) {
        real tm[Q];
        load_plane(first + dir * k, xo_m, tm);
        if (ring_load) load_plane(first + dir * k, xo_r, RG);
        put_psi(first + dir * k, tm, RG);
        if (k >= 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) F[k][i] = tm[i];
        }
    }
    // prefetch: ring plane first + dir R, main planes first + dir (R + q), q < PF
    if (RING_PF && ring_load) load_plane(first + dir * R, xo_r, RG);
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (q < len) load_plane(first + dir * (R + q), xo_m, F[R + q]);

    const uint32_t lane_store = uint32_t(D == 3 ? x + nx * y : x) * ES;

    for (int m0 = 0; m0 < len; m0 += NSLOT) {
#pragma unroll
        for (int j = 0; j < NSLOT; ++j) {
            const int m = m0 + j;
            if (m >= len) break;
            const int s = first + dir * m;
            // The noise of this plane depends on neither memory nor LDS: it is
            // generated first, so that it fills the wait for the prefetched
            // plane and the barrier (nothing is scheduled across a barrier).
            real z[NN];
            if constexpr (NOISE) {
                const uint32_t node = uint32_t(x + nx * (y + (D == 3 ? ny * s : s)));
                node_normals<L, real, !F32>(node, step32, d.seed_hi, z, d.key0, d.key1);
            } else {
#pragma unroll
                for (int k = 0; k < NN; ++k) z[k] = real(0);
            }
            // plane s + dir R has arrived: its dpsi goes to LDS
            // PF = 0: plane s + dir R is loaded here, right before its dpsi is needed
            if constexpr (PF == 0) load_plane(s + dir * R, xo_m, F[(j + R) % NSLOT]);
            if (!RING_PF && ring_load) load_plane(s + dir * R, xo_r, RG);
            put_psi(s + dir * R, F[(j + R) % NSLOT], RG);
            // prefetch: ring plane s + dir (R + 1), main plane s + dir (R + PF)
            if (RING_PF && ring_load && m + 1 < len) load_plane(s + dir * (R + 1), xo_r, RG);
            if (PF > 0 && m + PF < len) load_plane(s + dir * (R + PF), xo_m, F[(j + R + PF) % NSLOT]);
            __syncthreads();

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
                const real diff = lds[sl[R + es]][ty + RY + ey][tx + R + ex] -
                                  lds[sl[R - es]][ty + RY - ey][tx + R - ex];
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const int eq = ST::e(a, q);
                    if (eq != 0) g[q] = fmadd(real(ST::w(a) * eq), diff, g[q]);
                }
            }
            const real pre = G * (psi0 + lds[sl[R]][ty + RY][tx + R]);
            const real Fv[3] = {pre * g[0], pre * g[1], pre * g[2]};

            real(&fv)[Q] = F[j % NSLOT];
            if constexpr (D == 2) collide_d2q9<real, NOISE>(fv, rho0, Fv, lc, ac, z);
            else collide_d3q19<real, NOISE>(fv, rho0, Fv, lc, ac, z);

            const uint32_t so = uint32_t(s) * pbytes + lane_store;
            if constexpr (wide) {
#pragma unroll
                for (int i = 0; i < Q; ++i) bstore(pop_rsrc(d.buf[parity ^ 1], i), so, 0u, fv[i]);
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) bstore(dst, so, uint32_t(i) * pop_bytes, fv[i]);
            }
        }
    }
}

template <class L, class ST, typename real, bool NOISE, int TX, int TY, int PF>
inline hipError_t launch_one(const StepLaunch &P, hipStream_t s) {
    if (P.wide)
        hipLaunchKernelGGL((k_step<L, ST, real, NOISE, TX, TY, PF, true>), dim3(P.total_tiles),
                           dim3(TX * TY), 0, s, P.reps, P.tile_begin, P.nrep, P.parity, P.step_base,
                           P.step_off);
    else
        hipLaunchKernelGGL((k_step<L, ST, real, NOISE, TX, TY, PF, false>), dim3(P.total_tiles),
                           dim3(TX * TY), 0, s, P.reps, P.tile_begin, P.nrep, P.parity, P.step_base,
                           P.step_off);
    return hipGetLastError();
}

}  // namespace fsc
