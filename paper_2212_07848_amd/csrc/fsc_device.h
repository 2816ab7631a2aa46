// fsc_device.h -- lattice tables, moment basis, counter-based generator and
// small device helpers shared by the library's kernels (gfx950, wave64).
//
// Everything is constexpr so that the per-node collision, written as loops
// over populations and moments, folds into straight-line code with the
// integer moment coefficients as immediates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsc {

// ---------------------------------------------------------------------------
// Lattices (c_s^2 = 1/3).  Population order is the ABI order of include/fsc.h.
// ---------------------------------------------------------------------------
struct D2Q9 {
    static constexpr int D = 2, Q = 9;
    static constexpr int NNORM = 6;  // non-conserved moments that receive noise
    __host__ __device__ static constexpr int c(int i, int d) {
        constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return d == 0 ? cx[i] : (d == 1 ? cy[i] : 0);
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    // Moment rows, orthogonal under the weights w_i:
    //   1, cx, cy, 3c^2-2, cx^2-cy^2, cx cy, (3c^2-4)cx, (3c^2-4)cy, 9c^4-15c^2+2
    __host__ __device__ static constexpr int M(int a, int i) {
        int x = c(i, 0), y = c(i, 1), q = x * x + y * y;
        switch (a) {
        case 0: return 1;
        case 1: return x;
        case 2: return y;
        case 3: return 3 * q - 2;
        case 4: return x * x - y * y;
        case 5: return x * y;
        case 6: return (3 * q - 4) * x;
        case 7: return (3 * q - 4) * y;
        default: return 9 * q * q - 15 * q + 2;
        }
    }
    // class: 0 conserved, 1 bulk, 2 shear, 3 ghost
    __host__ __device__ static constexpr int cls(int a) {
        return a <= 2 ? 0 : (a == 3 ? 1 : (a <= 5 ? 2 : 3));
    }
    // Second-moment rows a = 3..5 are u^T A u quadratic forms: A(a, p, q).
    __host__ __device__ static constexpr double A(int a, int p, int q) {
        if (a == 3) return p == q ? 3.0 : 0.0;
        if (a == 4) return p == q ? (p == 0 ? 1.0 : -1.0) : 0.0;
        if (a == 5) return p != q ? 0.5 : 0.0;
        return 0.0;
    }
};

struct D3Q19 {
    static constexpr int D = 3, Q = 19;
    static constexpr int NNORM = 15;
    __host__ __device__ static constexpr int c(int i, int d) {
        constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return d == 0 ? cx[i] : (d == 1 ? cy[i] : cz[i]);
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    // Rows orthogonal under w_i: 1, c, c^2-1, 3cx^2-c^2, cy^2-cz^2, cxcy, cycz,
    // czcx, (3c^2-5)c, cx(cy^2-cz^2) and cyclic, 3c^4-6c^2+1,
    // (2c^2-3)(3cx^2-c^2), (2c^2-3)(cy^2-cz^2).
    __host__ __device__ static constexpr int M(int a, int i) {
        int x = c(i, 0), y = c(i, 1), z = c(i, 2), q = x * x + y * y + z * z;
        switch (a) {
        case 0: return 1;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return q - 1;
        case 5: return 3 * x * x - q;
        case 6: return y * y - z * z;
        case 7: return x * y;
        case 8: return y * z;
        case 9: return z * x;
        case 10: return (3 * q - 5) * x;
        case 11: return (3 * q - 5) * y;
        case 12: return (3 * q - 5) * z;
        case 13: return x * (y * y - z * z);
        case 14: return y * (z * z - x * x);
        case 15: return z * (x * x - y * y);
        case 16: return 3 * q * q - 6 * q + 1;
        case 17: return (2 * q - 3) * (3 * x * x - q);
        default: return (2 * q - 3) * (y * y - z * z);
        }
    }
    __host__ __device__ static constexpr int cls(int a) {
        return a <= 3 ? 0 : (a == 4 ? 1 : (a <= 9 ? 2 : 3));
    }
    __host__ __device__ static constexpr double A(int a, int p, int q) {
        switch (a) {
        case 4: return p == q ? 1.0 : 0.0;
        case 5: return p == q ? (p == 0 ? 2.0 : -1.0) : 0.0;
        case 6: return p == q ? (p == 0 ? 0.0 : (p == 1 ? 1.0 : -1.0)) : 0.0;
        case 7: return ((p == 0 && q == 1) || (p == 1 && q == 0)) ? 0.5 : 0.0;
        case 8: return ((p == 1 && q == 2) || (p == 2 && q == 1)) ? 0.5 : 0.0;
        case 9: return ((p == 2 && q == 0) || (p == 0 && q == 2)) ? 0.5 : 0.0;
        default: return 0.0;
        }
    }
};

// b_a = sum_i w_i M_ai^2 and the back-transform K(i, a) = w_i M_ai / b_a.
template <class L>
__host__ __device__ constexpr double moment_norm(int a) {
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += L::w(i) * double(L::M(a, i)) * double(L::M(a, i));
    return s;
}

// sqrt(b_a), by Newton's iteration at compile time: the noise of row a is
// sqrt(b_a) times a per-class amplitude.
__host__ __device__ constexpr double const_sqrt(double x) {
    double r = x > 1.0 ? x : 1.0;
    for (int k = 0; k < 64; ++k) r = 0.5 * (r + x / r);
    return r;
}
template <class L>
struct RowScale {
    double v[19];
    __host__ __device__ constexpr RowScale() : v{} {
        for (int a = 0; a < L::Q; ++a) v[a] = const_sqrt(moment_norm<L>(a));
    }
};

// ---------------------------------------------------------------------------
// Interaction stencils of Eq. (1), as half sets (one of each +-e pair).
// Weights are normalised to sum_a w e_x^2 = 1 over the full set.
// ---------------------------------------------------------------------------
struct StencilE4_2D {
    static constexpr int R = 1, NH = 4;
    __host__ __device__ static constexpr int e(int a, int d) {
        constexpr int ex[4] = {1, 0, 1, -1};
        constexpr int ey[4] = {0, 1, 1, 1};
        return d == 0 ? ex[a] : (d == 1 ? ey[a] : 0);
    }
    __host__ __device__ static constexpr double w(int a) { return a < 2 ? 1.0 / 3.0 : 1.0 / 12.0; }
};

struct StencilE8_2D {
    static constexpr int R = 2, NH = 12;
    __host__ __device__ static constexpr int e(int a, int d) {
        // |e|^2 = 1: (1,0) (0,1); 2: (1,1) (-1,1); 4: (2,0) (0,2);
        // 5: (2,1) (1,2) (-1,2) (-2,1); 8: (2,2) (-2,2)
        constexpr int ex[12] = {1, 0, 1, -1, 2, 0, 2, 1, -1, -2, 2, -2};
        constexpr int ey[12] = {0, 1, 1, 1, 0, 2, 1, 2, 2, 1, 2, 2};
        return d == 0 ? ex[a] : (d == 1 ? ey[a] : 0);
    }
    __host__ __device__ static constexpr double w(int a) {
        return a < 2 ? 4.0 / 21.0
                     : (a < 4 ? 4.0 / 45.0
                              : (a < 6 ? 1.0 / 60.0 : (a < 10 ? 2.0 / 315.0 : 1.0 / 5040.0)));
    }
};

struct StencilE4_3D {
    static constexpr int R = 1, NH = 9;
    __host__ __device__ static constexpr int e(int a, int d) {
        // |e|^2 = 1: x, y, z; 2: (1,1,0) (1,-1,0) (1,0,1) (1,0,-1) (0,1,1) (0,1,-1)
        constexpr int ex[9] = {1, 0, 0, 1, 1, 1, 1, 0, 0};
        constexpr int ey[9] = {0, 1, 0, 1, -1, 0, 0, 1, 1};
        constexpr int ez[9] = {0, 0, 1, 0, 0, 1, -1, 1, -1};
        return d == 0 ? ex[a] : (d == 1 ? ey[a] : ez[a]);
    }
    __host__ __device__ static constexpr double w(int a) { return a < 3 ? 1.0 / 6.0 : 1.0 / 12.0; }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The 32x32->64 products
// are single v_mad_u64_u32 operations; the key schedule is wave-uniform.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

// a ^ b ^ c as one gfx950 three-input bit operation (truth table 0x96: the
// parity of the three inputs) instead of two XORs
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = uint64_t(MA) * c.x;
        const uint64_t pb = uint64_t(MB) * c.z;
        U4 n;
        if (r < 2) {
            // the first two rounds see wave-uniform counter words (step, block,
            // seed), whose XORs the scalar unit takes
            n.x = uint32_t(pb >> 32) ^ c.y ^ k0;
            n.z = uint32_t(pa >> 32) ^ c.w ^ k1;
        } else {
            n.x = xor3(uint32_t(pb >> 32), c.y, k0);
            n.z = xor3(uint32_t(pa >> 32), c.w, k1);
        }
        n.y = uint32_t(pb);
        n.w = uint32_t(pa);
        c = n;
        k0 += WA;
        k1 += WB;
    }
    return c;
}

// The 20 round keys of Philox4x32-10 (k0 of round r at rk[2r], k1 at rk[2r+1])
// formed once, held in vector registers: an identity DPP move makes the
// compiler keep them per lane, where the round XORs read them directly, instead
// of forming them anew with scalar adds for every draw (there are too many to
// keep in scalar registers beside the rest of a step kernel).
struct PhiloxKeys {
    uint32_t rk[20];
};
__device__ __forceinline__ PhiloxKeys philox_keys(uint32_t k0, uint32_t k1) {
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
    PhiloxKeys K;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        K.rk[2 * r] = uint32_t(__builtin_amdgcn_mov_dpp(int(k0), 0xE4, 0xF, 0xF, false));
        K.rk[2 * r + 1] = uint32_t(__builtin_amdgcn_mov_dpp(int(k1), 0xE4, 0xF, 0xF, false));
        k0 += WA;
        k1 += WB;
    }
    return K;
}
__device__ inline U4 philox4x32_10(U4 c, const PhiloxKeys &K) {
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = uint64_t(MA) * c.x;
        const uint64_t pb = uint64_t(MB) * c.z;
        U4 n;
        n.x = xor3(uint32_t(pb >> 32), c.y, K.rk[2 * r]);
        n.y = uint32_t(pb);
        n.z = xor3(uint32_t(pa >> 32), c.w, K.rk[2 * r + 1]);
        n.w = uint32_t(pa);
        c = n;
    }
    return c;
}

// Noise normals of one node.  The paper fixes only that the thermal noise is
// Gaussian and uncorrelated in space and time; the bit layout below is this
// library's definition (the oracle implements the same one):
//   words w_0, w_1, ... = Philox4x32-10 outputs of blocks 0, 1, ... with
//     counter (node, step, block, seed >> 32), key (seed & 0xffffffff, replica);
//   pair k takes a radius uniform u_a = (floor(w_k / 2^9) + 1/2) 2^-23 and an
//     angle uniform u_b = (h_k + 1/2) 2^-16 from a 16-bit field h_k:
//       D2Q9  (3 pairs, 1 block):  h_0 = w_3 >> 16, h_1 = w_3 & 0xffff,
//                                  h_2 = (w_0 & 0xff) << 8 | (w_1 & 0xff)
//       D3Q19 (8 pairs, 3 blocks): h_k = 16-bit half k of w_8 .. w_11
//                                  (high half first)
//   (z_2k, z_2k+1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b); normal k goes
//   to the k-th non-conserved moment.  Both uniforms are exact in float.
// UNIT = false (the FP32 step kernels): the normals come divided by
// sqrt(2 ln 2), so that the radius is sqrt(-log2 u_a), one multiply fewer per
// pair; those kernels fold BM_SCALE into their noise amplitudes.
constexpr float BM_SCALE = 1.17741002251547469f;  // sqrt(2 ln 2)

template <bool UNIT = true>
__device__ __forceinline__ void box_muller(float ua, float ub, float &z0, float &z1) {
#ifdef FSC_ACCURATE_BOX_MULLER
    const float rad = UNIT ? sqrtf(-2.0f * logf(ua)) : sqrtf(-log2f(ua));
    float s, c;
    sincospif(2.0f * ub, &s, &c);
#else
    // hardware log2, sqrt and sin/cos (argument in revolutions)
    const float l2 = __builtin_amdgcn_logf(ua);
    const float rad = __builtin_amdgcn_sqrtf(UNIT ? -1.3862943611198906f * l2 : -l2);
    const float s = __builtin_amdgcn_sinf(ub), c = __builtin_amdgcn_cosf(ub);
#endif
    z0 = rad * c;
    z1 = rad * s;
}
template <bool UNIT = true>
__device__ __forceinline__ void box_muller(double ua, double ub, double &z0, double &z1) {
    static_assert(UNIT, "FP64 normals are always unit");
    const double rad = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

template <class L, typename real, bool UNIT = true, typename... Key>
__device__ __forceinline__ void node_normals(uint32_t node, uint32_t step, uint32_t seed_hi,
                                             real (&z)[L::NNORM], const Key &...key) {
    constexpr int NN = L::NNORM;
    constexpr int P = (NN + 1) / 2;
    constexpr int NB = L::D == 2 ? 1 : 3;
    uint32_t w[4 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const U4 r = philox4x32_10(U4{node, step, uint32_t(b), seed_hi}, key...);
        w[4 * b] = r.x;
        w[4 * b + 1] = r.y;
        w[4 * b + 2] = r.z;
        w[4 * b + 3] = r.w;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        uint32_t h;
        if (L::D == 2)
            h = k == 0 ? (w[3] >> 16) : (k == 1 ? (w[3] & 0xffffu) : (((w[0] & 0xffu) << 8) | (w[1] & 0xffu)));
        else
            h = (k & 1) ? (w[8 + k / 2] & 0xffffu) : (w[8 + k / 2] >> 16);
        real ua, ub;
        if constexpr (sizeof(real) == 4) {
            // the same values from the bits, each an exact subtraction: the float
            // 1 + m 2^-23 (m = w_k >> 9 as its mantissa) minus 1 - 2^-24, and
            // 1 + (2h + 1) 2^-17 minus 1
            const uint32_t fa = __builtin_amdgcn_alignbit(0x7Fu, w[k], 9u);
            ua = __builtin_bit_cast(float, fa) - (1.0f - 5.9604644775390625e-08f);
            ub = __builtin_bit_cast(float, (h << 7) | 0x3F800040u) - 1.0f;
        } else {
            ua = real((w[k] >> 8) | 1u) * real(5.9604644775390625e-08);  // (2m+1) 2^-24
            ub = real(2u * h + 1u) * real(7.62939453125e-06);             // (2h+1) 2^-17
        }
        real z0, z1;
        box_muller<UNIT>(ua, ub, z0, z1);
        z[2 * k] = z0;
        if (2 * k + 1 < NN) z[2 * k + 1] = z1;
    }
}

// ---------------------------------------------------------------------------
// Per-replica description, resident in device memory and read by the kernels
// with wave-uniform (scalar) loads.
// ---------------------------------------------------------------------------
struct RepDesc {
    void *buf[2];            // population buffers; state at step t is in buf[t & 1]
    int64_t N;               // nodes
    int32_t nx, ny, nz;      // sides
    int32_t ns;              // extent of the marching axis (ny in 2D, nz in 3D)
    int32_t plane;           // nodes per plane orthogonal to the marching axis
    int32_t tiles_x, tiles_y;  // cross-section tiles (tiles_y = 1 in 2D)
    int32_t nchunk, H;       // chunks along the marching axis and their length
    int32_t tile_begin;      // first global tile index of this replica
    int32_t noise;           // kBT > 0
    int32_t pad0;
    double G, rho0, psi0;
    // Per moment class c (1 bulk, 2 shear, 3 ghost; 0 = conserved, unused):
    // relaxation rate lam_c and noise amplitude sqrt(kBT/c_s^2 (1 - (1-lam_c)^2));
    // row a of class c gets noise sqrt(b_a) amp_c sqrt(n) xi_a.
    double lamc[4], ampc[4];
    // float copies for the FP32 kernels (wave-uniform, kept in scalar registers)
    float Gf, rho0f, psi0f, inv_rho0f;
    float lamcf[4], ampcf[4];
    uint32_t key0, key1, seed_hi, pad1;
};

// Block index -> logical tile index so that each XCD (blocks are dealt to the
// 8 XCDs round-robin) receives one contiguous range of tiles, which keeps
// neighbouring tiles' halo reads inside one L2.
__device__ inline int xcd_remap(int b, int B) {
    const int q = B >> 3, r = B & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__host__ __device__ inline int wrap_any(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}


// Debug builds with FSC_LDS_POISON fill a kernel's LDS with NaN before use
// (then a barrier): a read of a slot that the launch has not written yet
// carries the NaN into the results, where the parity and bit-identity tests
// see it.  Off in normal builds.
template <typename T>
__device__ __forceinline__ void lds_poison(T *p, int n) {
#ifdef FSC_LDS_POISON
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = T(__builtin_nanf(""));
#else
    (void)p;
    (void)n;
#endif
}

}  // namespace fsc
