// fsc_step2_kernel.h -- two fused time steps of the fluctuating Shan-Chen
// lattice Boltzmann equation (Eq. 12 of Lulli et al., arXiv:2212.07848) per
// pass over HBM, for D2Q9 (temporal blocking).
//
// The single-step kernel reads and writes every population once per step.
// Here a workgroup computes step t -> t+1 ("level 1") on its tile widened by
// R + 1 columns and rows, keeps f(t+1) in LDS, and immediately computes
// t+1 -> t+2 ("level 2") on the tile itself, so that each step costs half the
// HBM traffic.  The per-node arithmetic is the single-step kernel's (same
// functions, same order), so two steps here equal two single steps bit for
// bit, and the noise keeps its counter (node, step) keys.
//
// Workgroup: TX tile lanes plus one extra wave.  Every thread owns one
// level-1 node at column offset x1 from the tile origin x0:
//   tile lanes           x1 = lane (lanes past a ragged edge duplicate the last
//                        valid column and write nothing to LDS; a wave wholly
//                        past it does no work at all)
//   extra wave, e < 2R+2 the level-1 edge columns -R-1..-1 and TXe..TXe+R
//   extra wave, e < 4R+2 psi-only columns -2R-1..-R-2 and TXe+R+1..TXe+2R
// and at most one level-2 node: tile lanes x2 = x1 (collide and store), extra
// wave e < 2R the psi(t+1)-only columns -R..-1 and TXe..TXe+R-1.  When the
// tile spans a whole periodic row (one tile across) the extra wave idles and
// the tile lanes near either end also write their LDS values at the periodic
// image columns, so the halo reads stay plain offsets.
//
// In-tile halos (template HIN): the workgroup has TX + 4R + 2 lanes and lane l
// owns column l - (2R + 1), so the halo columns sit in the same waves as the
// tile's own; every stage keeps the lanes whose column lies in its range
// (psi(t) [-2R-1, TXe+2R], level 1 [-R-1, TXe+R], psi(t+1) [-R, TXe+R-1],
// level 2 [0, TXe-1]).  The edge wave's mostly idle lanes disappear: per
// output column a launch issues about a tenth fewer wave instructions.  A
// whole row takes the same mapping, its halo columns wrapped periodically, so
// no mirrored writes are needed.
//
// March of a chunk of H output rows o_0..o_{H-1} (direction alternating by
// chunk as in the single-step kernel): level 1 runs over the rows
// l_k = o_{k-R-1}, k = 0..H+2R+1, with the pulled rows of f(t) in a register
// ring of R+1 rows and psi(t) in an LDS ring of 2R+2 rows (A); f(t+1) goes to
// an LDS ring (B).  Two schedules (template BARS):
//   one barrier per iteration j, B of 4 rows:
//     before the barrier: loads of level-1 row l_{j+R}; the noise of both
//       levels; level 2 pulls f(t+1) of row l_{j-3} from B (rows written at
//       least two iterations ago) into a register ring of R+1 rows and writes
//       its psi(t+1) into an LDS ring of 2R+2 rows (C); psi(t) of l_{j+R} -> A;
//     after the barrier: level-1 force and collision of row l_j -> B; level-2
//       force and collision of row l_{j-3-R} -> HBM;
//   two barriers per iteration, B of 3 rows (less LDS, so more workgroups
//     per CU): loads, noise, psi(t) -> A | barrier | level 1 of row l_j -> B |
//     barrier | level-2 collision of row l_{j-2-R}, then the pull and
//     psi(t+1) of row l_{j-1}.
// The ring sizes make sure that no slot is rewritten while a slower wave may
// still read it (B and C are the smallest that do).
#pragma once

#include "fsc_step_kernel.h"

namespace fsc {

// Threads of a workgroup: TX tile lanes and the edge wave, or (HIN) the tile's
// TX output columns with their 2R + 1 halo columns on either side.
template <class ST, int TX, bool HIN>
constexpr int step2_lanes() {
    return HIN ? TX + 4 * ST::R + 2 : TX + 64;
}

template <class ST, typename real, bool NOISE, int TX, int BARS, bool HIN = false>
__global__ void __launch_bounds__((step2_lanes<ST, TX, HIN>()))
    k_step2(const RepDesc *__restrict__ reps, const int *__restrict__ tile_begin, int nrep,
            int parity, const uint64_t *__restrict__ step_base, uint32_t step_off) {
    using L = D2Q9;
    constexpr int Q = 9, R = ST::R, NN = L::NNORM;
    constexpr int NR = R + 1;                       // register rings (rows)
    // psi rings of 2R + 2 rows, rounded up to a power of two in the in-tile
    // halo form with one barrier (its LDS still allows three workgroups per
    // CU), so that ring slots wrap with a mask
    constexpr int SPSI = (HIN && BARS == 1) ? ((2 * R + 2) <= 4 ? 4 : 8) : 2 * R + 2;
    constexpr int SA = SPSI, SB = BARS == 1 ? 4 : 3, SC = SPSI;
    constexpr int OA = 2 * R + 1, OB = R + 1, OC = R;  // column of offset 0
    constexpr int WA = TX + 4 * R + 2, WB = TX + 2 * R + 2, WC = TX + 2 * R;
    constexpr uint32_t ES = sizeof(real);
    __shared__ real A[SA][WA];
    __shared__ real B[SB][Q][WB];
    __shared__ real Cs[SC][WC];
#ifdef FSC_LDS_POISON
    lds_poison(&A[0][0], SA * WA);
    lds_poison(&B[0][0][0], SB * Q * WB);
    lds_poison(&Cs[0][0], SC * WC);
    __syncthreads();
#endif

    // ---- which replica / tile (as in the single-step kernel) ----------------
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_begin[mid] <= lb) lo = mid;
        else hi = mid - 1;
    }
    const RepDesc &d = reps[lo];
    const int nx = d.nx, ns = d.ny;
    const int t = lb - d.tile_begin;
    const int tix = t % d.tiles_x;
    const int chunk = t / d.tiles_x;
    const int s_begin = chunk * d.H;
    const int s_end = min(s_begin + d.H, ns);
    const int H = s_end - s_begin;
    const int x0 = tix * TX;
    const int TXe = min(TX, nx - x0);
    // TXe == nx: the tile holds whole periodic rows (mirrored LDS writes; the
    // in-tile-halo form instead wraps its halo columns, which fit its lanes)
    const bool full = !HIN && d.tiles_x == 1;

    const int tid = threadIdx.x;
    // HIN: lane tid owns column tid - (2R + 1), whole rows included
    const bool shifted = HIN;
    const bool ewave = !HIN && tid >= TX;
    const int e = tid - TX;
    const bool eidle = ewave && full;  // wave-uniform
    // A wave wholly past the columns the tile needs (a tile narrower than TX)
    // has no node of its own: it only takes part in the barriers.
    const bool tidle = !ewave && (shifted ? (tid & ~63) >= TXe + 4 * R + 2 : (tid & ~63) >= TXe);
    const bool idle = eidle || tidle;

    // level-1 node: column offset x1, collides (c1), writes to A (wa) and B (wb)
    int x1 = 0;
    bool c1 = !ewave && !tidle, wa = false, wb = false;
    // level-2 node: column offset x2, forms psi(t+1) (p2), writes to C (wc);
    // collides and stores to HBM (st2)
    int x2 = 0;
    bool p2 = !ewave && !tidle, wc = false, st2 = !ewave && !tidle;
    if (shifted) {
        // the tile's columns and both halos in one range of lanes; lanes past
        // its end duplicate the last column and write nothing
        const int c = tid - (2 * R + 1);
        x1 = min(c, TXe + 2 * R);
        wa = c < TXe + 2 * R + 1;
        c1 = wb = c >= -R - 1 && c < TXe + R + 1;
        x2 = x1;
        p2 = wc = c >= -R && c < TXe + R;
        st2 = c >= 0 && c < TXe;
    } else if (!ewave) {
        x1 = min(tid, TXe - 1);
        wa = wb = tid < TXe;
        x2 = x1;
        wc = tid < TXe;
    } else if (!full && e < 2 * R + 2) {
        x1 = e < R + 1 ? -R - 1 + e : TXe + (e - R - 1);
        c1 = wa = wb = true;
    } else if (!full && e < 4 * R + 2) {
        const int k = e - 2 * R - 2;
        x1 = k < R ? -2 * R - 1 + k : TXe + R + 1 + (k - R);
        wa = true;
    }
    if (ewave && !full && e < 2 * R) {
        x2 = e < R ? -R + e : TXe + (e - R);
        p2 = wc = true;
    }
    // periodic images of tile columns near the row ends (whole-row tiles only)
    const bool mir = full && !ewave && tid < TXe;
    const int ia_lo = (mir && x1 >= nx - (2 * R + 1)) ? x1 - nx + OA : -1;
    const int ia_hi = (mir && x1 <= 2 * R) ? x1 + nx + OA : -1;
    const int ib_lo = (mir && x1 >= nx - (R + 1)) ? x1 - nx + OB : -1;
    const int ib_hi = (mir && x1 <= R) ? x1 + nx + OB : -1;
    const int ic_lo = (mir && x2 >= nx - R) ? x2 - nx + OC : -1;
    const int ic_hi = (mir && x2 <= R - 1) ? x2 + nx + OC : -1;

    const uint64_t buf_bytes = uint64_t(Q) * uint64_t(d.N) * sizeof(real);
    const rsrc_t src = make_rsrc(d.buf[parity], buf_bytes);
    const rsrc_t dst = make_rsrc(d.buf[parity ^ 1], buf_bytes);
    const uint32_t pop_bytes = uint32_t(d.N) * ES;
    const uint32_t pbytes = uint32_t(nx) * ES;

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

    // ---- pull offsets of the level-1 node (bytes within a row) ---------------
    const int gx1 = wrap_any(x0 + x1, nx);
    const int gx2 = wrap_any(x0 + x2, nx);
    uint32_t xo[3];  // index c_x + 1 -> column x - c_x
    xo[0] = uint32_t(gx1 + 1 == nx ? 0 : gx1 + 1) * ES;
    xo[1] = uint32_t(gx1) * ES;
    xo[2] = uint32_t(gx1 == 0 ? nx - 1 : gx1 - 1) * ES;
    auto wrap_row = [ns](int v) {
        while (v < 0) v += ns;
        while (v >= ns) v -= ns;
        return v;
    };
    auto load_wrapped = [&](int pc, real (&out)[Q]) {  // lattice row pc in [0, ns)
        const int pp = pc + 1 == ns ? 0 : pc + 1, pm = pc == 0 ? ns - 1 : pc - 1;
        const uint32_t pb[3] = {uint32_t(pp) * pbytes, uint32_t(pc) * pbytes, uint32_t(pm) * pbytes};
#pragma unroll
        for (int i = 0; i < Q; ++i)
            out[i] = bload<real>(src, xo[L::c(i, 0) + 1], uint32_t(i) * pop_bytes + pb[L::c(i, 1) + 1]);
    };
    auto load_row = [&](int row, real (&out)[Q]) { load_wrapped(wrap_row(row), out); };
    auto dpsi_of = [&](const real (&fv)[Q]) {
        real dn = real(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) dn += fv[i];
        return psi0 * fexpm1(dn * inv_rho0 * fast_rcp(rho0 + dn));
    };

    const uint64_t step = step_base[0] + step_off;
    const uint32_t step1 = uint32_t(step), step2 = uint32_t(step + 1);
    // Philox round keys held per lane (20 VGPRs) where LDS already limits the
    // workgroups per CU (the one-barrier in-tile-halo form); elsewhere the
    // registers would cost occupancy, and the keys are formed per draw
    constexpr bool VKEYS = HIN && BARS == 1;
    const PhiloxKeys PK = VKEYS ? philox_keys(d.key0, d.key1) : PhiloxKeys{};
    auto normals = [&](uint32_t node, uint32_t st, real (&z)[NN]) {
        if constexpr (VKEYS) node_normals<L, real, !F32>(node, st, d.seed_hi, z, PK);
        else node_normals<L, real, !F32>(node, st, d.seed_hi, z, d.key0, d.key1);
    };

    // ---- march order ----------------------------------------------------------
    const int dir = (chunk & 1) ? -1 : 1;
    const int first = dir > 0 ? s_begin : s_end - 1;       // o_0
    auto lrow = [&](int k) { return first + dir * (k - R - 1); };  // lattice row of l_k
    const int H1 = H + 2 * R + 2;                          // level-1 rows

    // ring slot t of a ring of n rows, for t within one ring length of [0, n)
    auto wrapc = [](int t, int n) {
        if ((n & (n - 1)) == 0) return t & (n - 1);  // power of two (n is a constant)
        return t < 0 ? t + n : (t >= n ? t - n : t);
    };
    auto put_slot = [&](int sl, real v) {  // psi(t) of the row in slot sl of A
        if (wa) A[sl][x1 + OA] = v;
        if (ia_lo >= 0) A[sl][ia_lo] = v;
        if (ia_hi >= 0) A[sl][ia_hi] = v;
    };
    auto put_a = [&](int k, real v) { put_slot((k + SA) % SA, v); };  // psi(t) of l_k

    // ---- prologue: psi(t) of l_{-R} .. l_{R-1}; pulled rows l_0 .. l_{R-1} ----
    real F[NR][Q];
    real G2[NR][Q];
#pragma unroll
    for (int k = -R; k < R; ++k) {
        real tm[Q];
        if (!idle) load_row(lrow(k), tm);
        else
#pragma unroll
            for (int i = 0; i < Q; ++i) tm[i] = real(0);
        put_a(k, idle ? real(0) : dpsi_of(tm));
        if (k >= 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) F[k][i] = tm[i];
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) G2[k][i] = real(0);

    const uint32_t lane_store = uint32_t(x0 + x2) * ES;  // tile lanes only store

    // ---- the three pieces of an iteration ---------------------------------------
    // level 2: pull f(t+1) of l_k from B into the register ring, psi(t+1) -> C
    // (kb, kc: the slots of l_k in B and C)
    auto psi_stage = [&](int kb, int kc, int gs) {
        const int sb[3] = {wrapc(kb + dir, SB), kb, wrapc(kb - dir, SB)};  // c_y + 1 -> row - c_y
        real(&g2)[Q] = G2[gs];
#pragma unroll
        for (int i = 0; i < Q; ++i) g2[i] = B[sb[L::c(i, 1) + 1]][i][x2 - L::c(i, 0) + OB];
        const real v = dpsi_of(g2);
        const int sl = kc;
        if (wc) Cs[sl][x2 + OC] = v;
        if (ic_lo >= 0) Cs[sl][ic_lo] = v;
        if (ic_hi >= 0) Cs[sl][ic_hi] = v;
    };
    // level 1: force and collision of l_j (pulled populations in F[fs]) -> B
    // (ja, jb: the slots of l_j in A and B)
    auto level1 = [&](int ja, int jb, int fs, const real (&z)[NN]) {
        real g[3] = {real(0), real(0), real(0)};
#pragma unroll
        for (int a = 0; a < ST::NH; ++a) {
            const int ex = ST::e(a, 0), es = dir * ST::e(a, 1);
            const real diff = A[wrapc(ja + es, SA)][x1 + ex + OA] - A[wrapc(ja - es, SA)][x1 - ex + OA];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int eq = ST::e(a, q);
                if (eq != 0) g[q] = fmadd(real(ST::w(a) * eq), diff, g[q]);
            }
        }
        const real pre = G * (psi0 + A[ja][x1 + OA]);
        const real Fv[3] = {pre * g[0], pre * g[1], pre * g[2]};
        real(&fv)[Q] = F[fs];
        collide_d2q9<real, NOISE>(fv, rho0, Fv, lc, ac, z);
        const int sl = jb;
        if (wb) {
#pragma unroll
            for (int i = 0; i < Q; ++i) B[sl][i][x1 + OB] = fv[i];
        }
        if (ib_lo >= 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) B[sl][i][ib_lo] = fv[i];
        }
        if (ib_hi >= 0) {
#pragma unroll
            for (int i = 0; i < Q; ++i) B[sl][i][ib_hi] = fv[i];
        }
    };
    // level 2: force and collision of l_k (pulled populations in G2[gs]) -> HBM
    // (kc: the slot of l_k in C; krow: its lattice row)
    auto level2 = [&](int kc, int gs, int krow, const real (&z)[NN]) {
        real g[3] = {real(0), real(0), real(0)};
#pragma unroll
        for (int a = 0; a < ST::NH; ++a) {
            const int ex = ST::e(a, 0), es = dir * ST::e(a, 1);
            const real diff = Cs[wrapc(kc + es, SC)][x2 + ex + OC] - Cs[wrapc(kc - es, SC)][x2 - ex + OC];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int eq = ST::e(a, q);
                if (eq != 0) g[q] = fmadd(real(ST::w(a) * eq), diff, g[q]);
            }
        }
        const real pre = G * (psi0 + Cs[kc][x2 + OC]);
        const real Fv[3] = {pre * g[0], pre * g[1], pre * g[2]};
        real(&fv)[Q] = G2[gs];
        collide_d2q9<real, NOISE>(fv, rho0, Fv, lc, ac, z);
        const uint32_t so = uint32_t(krow) * pbytes + lane_store;
#pragma unroll
        for (int i = 0; i < Q; ++i) bstore<HIN ? 0 : FSC_STORE_POLICY>(dst, so, uint32_t(i) * pop_bytes, fv[i]);
    };

    // Level 2 trails level 1.  Its pull (and psi(t+1)) of iteration j is row
    // kp = j - LAG: with one barrier per iteration it can only read B rows
    // written two iterations ago (LAG = 3), with two barriers also the row
    // written before the second barrier (LAG = 1).  Its collision is row
    // km = kp - LAG2, whose psi(t+1) stencil reaches km + R: with one barrier
    // that row is written before the barrier of the same iteration
    // (LAG2 = R); with two barriers it was written one iteration earlier
    // (LAG2 = R + 1, so the collision can run before this iteration's pull).
    constexpr int LAG = BARS == 1 ? 3 : 1;
    constexpr int LAG2 = BARS == 1 ? R : R + 1;
    const int J = H + R + LAG + LAG2 + 1;  // iterations: the last one collides km = H + R
    // wrapped lattice rows of l_{j+R} (loads), l_j (level 1) and l_km (level
    // 2), advanced by one row per iteration instead of wrapped anew
    auto next_row = [&](int r) {
        r += dir;
        return r >= ns ? r - ns : (r < 0 ? r + ns : r);
    };
    int row_ld = wrap_row(lrow(R)), row_1 = wrap_row(lrow(0)), row_2 = wrap_row(lrow(-LAG - LAG2));
    // ring slots, advanced likewise: l_j in A and B, l_kp in B and C, l_km in C
    auto slot0 = [](int k, int n) { return (k % n + n) % n; };
    int sa_j = 0, sb_j = 0, sb_p = slot0(-LAG, SB), sc_p = slot0(-LAG, SC),
        sc_m = slot0(-LAG - LAG2, SC);
    for (int j0 = 0; j0 < J; j0 += NR) {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int j = j0 + u;
            if (j >= J) break;
            const int kp = j - LAG;       // psi(t+1) row of this iteration
            const int km = kp - LAG2;     // level-2 output row of this iteration
            const bool lev1 = j < H1;
            const bool psi2 = kp >= 1 && kp <= H1 - 2;
            const bool lev2 = km >= R + 1 && km <= H1 - 2 - R;
            // register-ring slots (constants once the loop over u is unrolled)
            const int fs_new = (u + R) % NR;                     // row l_{j+R}
            const int gs_new = ((u - LAG) % NR + NR) % NR;       // row l_kp
            const int gs_use = ((u - LAG - LAG2) % NR + NR) % NR;  // row l_km

            // loads of level-1 row l_{j+R} (consumed by its psi below and by
            // its collision R iterations later)
            if (lev1 && !idle) load_wrapped(row_ld, F[fs_new]);
            // noise of both levels (independent of memory and LDS)
            real z1[NN], z2[NN];
            if constexpr (NOISE) {
                if (lev1 && !idle) normals(uint32_t(gx1 + nx * row_1), step1, z1);
                if (lev2 && st2) normals(uint32_t(gx2 + nx * row_2), step2, z2);
            }
            if constexpr (!NOISE) {
#pragma unroll
                for (int k = 0; k < NN; ++k) z1[k] = z2[k] = real(0);
            }
            if constexpr (BARS == 1) {
                // B rows kp - 1 .. kp + 1 were written at least two iterations ago
                if (psi2 && p2) psi_stage(sb_p, sc_p, gs_new);
                if (lev1) put_slot(wrapc(sa_j + R, SA), idle ? real(0) : dpsi_of(F[fs_new]));
                __syncthreads();
                if (lev1 && c1) level1(sa_j, sb_j, u, z1);
                if (lev2 && st2) level2(sc_m, gs_use, row_2, z2);
            } else {
                if (lev1) put_slot(wrapc(sa_j + R, SA), idle ? real(0) : dpsi_of(F[fs_new]));
                __syncthreads();
                if (lev1 && c1) level1(sa_j, sb_j, u, z1);
                __syncthreads();
                // the collision frees the ring slot that the pull then refills
                // (gs_use == gs_new, as kp - km = R + 1)
                if (lev2 && st2) level2(sc_m, gs_use, row_2, z2);
                if (psi2 && p2) psi_stage(sb_p, sc_p, gs_new);
            }
            row_ld = next_row(row_ld);
            row_1 = next_row(row_1);
            row_2 = next_row(row_2);
            sa_j = wrapc(sa_j + 1, SA);
            sb_j = wrapc(sb_j + 1, SB);
            sb_p = wrapc(sb_p + 1, SB);
            sc_p = wrapc(sc_p + 1, SC);
            sc_m = wrapc(sc_m + 1, SC);
        }
    }
}

template <class ST, typename real, bool NOISE, int TX, int BARS, bool HIN = false>
inline hipError_t launch_two(const StepLaunch &P, hipStream_t s) {
    hipLaunchKernelGGL((k_step2<ST, real, NOISE, TX, BARS, HIN>), dim3(P.total_tiles),
                       dim3(step2_lanes<ST, TX, HIN>()), 0, s, P.reps, P.tile_begin, P.nrep, P.parity,
                       P.step_base, P.step_off);
    return hipGetLastError();
}

}  // namespace fsc
