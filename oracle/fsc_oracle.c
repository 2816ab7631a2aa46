/*
 * fsc_oracle.c -- plain FP64 CPU oracle for the fluctuating Shan-Chen lattice
 * Boltzmann step (D2Q9 / D3Q19) of Lulli et al., "Metastable and Unstable
 * Dynamics in multi-phase lattice Boltzmann" (arXiv:2212.07848).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or generator with the GPU library; both are written from the
 * paper and from the published definition of Philox4x32-10.
 *
 * The state is the full population field f_i(x, t) right after streaming,
 * stored as f[i][z][y][x] (x fastest), in double precision.  One step follows
 * the fluctuating lattice Boltzmann equation, Eq. (12) of the paper:
 *
 *   f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i + F_i + eta_i
 *
 * evaluated in the order of the paper's description:
 *   1. n = sum_i f_i, j = sum_i f_i c_i
 *   2. psi = exp(-1/n)                                (pseudopotential choice)
 *   3. F(x) = G psi(x) sum_a w(|e_a|^2) psi(x + e_a) e_a           (Eq. 1)
 *   4. u = (j + F/2)/n, Guo forcing (cited by the paper for F_i)
 *   5. collision in moment space with a basis orthogonal under the lattice
 *      weights, so that the noise covariance is diagonal in moment space and
 *      zero on the conserved moments (text after Eq. 16)
 *   6. back-transform and periodic streaming.
 * Readings of points the paper leaves open are listed at each step.
 * Nothing here is blocked, fused or reordered for speed; the node loops carry
 * an OpenMP pragma only so that large baselines finish in bounded time.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 19
#define ORC_MAXF 24

/* ------------------------------------------------------------------------ */
/* Lattices.  Velocity order is the population order of the state arrays.   */
/* D2Q9: rest, 4 axis, 4 diagonal.  D3Q19: rest, 6 axis, 12 face diagonals. */
/* Weights are the standard ones with c_s^2 = 1/3.                          */
/* ------------------------------------------------------------------------ */
static const int d2q9_c[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int d3q19_c[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double CS2 = 1.0 / 3.0; /* isothermal T = c_s^2 */

static int lattice_q(int D) { return D == 2 ? 9 : (D == 3 ? 19 : -1); }

static void lattice_c(int D, int i, int c[3]) {
    const int *v = (D == 2) ? d2q9_c[i] : d3q19_c[i];
    c[0] = v[0]; c[1] = v[1]; c[2] = v[2];
}

static double lattice_w(int D, int i) {
    int c[3];
    lattice_c(D, i, c);
    int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (D == 2) return c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

int orc_lattice(int D, int *Q, int *c, double *w) {
    int q = lattice_q(D);
    if (q < 0) return -1;
    *Q = q;
    for (int i = 0; i < q; ++i) {
        lattice_c(D, i, c + 3 * i);
        w[i] = lattice_w(D, i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Interaction stencils of Eq. (1).  The weights w(|e|^2) are normalised so */
/* that sum_a w e_ax^2 = 1, which makes the bulk pressure p = nT - G psi^2/2 */
/* of Eq. (2); the paper cites the isotropic sets without printing them.    */
/*   E4 (2D): |e|^2 = 1, 2                      -> 1/3, 1/12                */
/*   E8 (2D): |e|^2 = 1, 2, 4, 5, 8 (5x5 block) -> 4/21, 4/45, 1/60,        */
/*                                                 2/315, 1/5040            */
/*   E4 (3D): |e|^2 = 1, 2 (18 neighbours)      -> 1/6, 1/12                */
/* ------------------------------------------------------------------------ */
static double stencil_weight(int D, int stencil, int e2) {
    if (D == 2 && stencil == 4) {
        if (e2 == 1) return 1.0 / 3.0;
        if (e2 == 2) return 1.0 / 12.0;
        return 0.0;
    }
    if (D == 2 && stencil == 8) {
        switch (e2) {
        case 1: return 4.0 / 21.0;
        case 2: return 4.0 / 45.0;
        case 4: return 1.0 / 60.0;
        case 5: return 2.0 / 315.0;
        case 8: return 1.0 / 5040.0;
        default: return 0.0;
        }
    }
    if (D == 3 && stencil == 4) {
        if (e2 == 1) return 1.0 / 6.0;
        if (e2 == 2) return 1.0 / 12.0;
        return 0.0;
    }
    return -1.0;
}

/* Enumerates every offset of the stencil (both signs), returns the count. */
int orc_stencil(int D, int stencil, int *nf, int *e, double *w) {
    if (stencil_weight(D, stencil, 1) < 0.0) return -1;
    int r = (stencil == 8) ? 2 : 1;
    int zr = (D == 3) ? r : 0;
    int n = 0;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                int e2 = dx * dx + dy * dy + dz * dz;
                if (e2 == 0) continue;
                double ww = stencil_weight(D, stencil, e2);
                if (ww == 0.0) continue;
                e[3 * n + 0] = dx; e[3 * n + 1] = dy; e[3 * n + 2] = dz;
                w[n] = ww;
                ++n;
            }
    *nf = n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Moment basis.  The paper asks for a noise covariance that is diagonal in */
/* the space of the noise moments N_a = sum_i m_ai eta_i, with zero         */
/* variance on the conserved moments a = 0..D.  That holds for a basis that */
/* is orthogonal under the weighted product <g,h> = sum_i w_i g_i h_i.      */
/* It is built here by weighted Gram-Schmidt (no normalisation) from the    */
/* listed polynomials of the velocity components, in the listed order.      */
/* ------------------------------------------------------------------------ */
static double seed_poly(int D, int a, const int c[3]) {
    double x = c[0], y = c[1], z = c[2];
    double c2 = x * x + y * y + z * z;
    if (D == 2) {
        switch (a) {
        case 0: return 1.0;
        case 1: return x;
        case 2: return y;
        case 3: return c2;
        case 4: return x * x - y * y;
        case 5: return x * y;
        case 6: return c2 * x;
        case 7: return c2 * y;
        case 8: return c2 * c2;
        }
    } else {
        switch (a) {
        case 0: return 1.0;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return c2;
        case 5: return 3.0 * x * x - c2;
        case 6: return y * y - z * z;
        case 7: return x * y;
        case 8: return y * z;
        case 9: return z * x;
        case 10: return c2 * x;
        case 11: return c2 * y;
        case 12: return c2 * z;
        case 13: return x * (y * y - z * z);
        case 14: return y * (z * z - x * x);
        case 15: return z * (x * x - y * y);
        case 16: return c2 * c2;
        case 17: return c2 * (3.0 * x * x - c2);
        case 18: return c2 * (y * y - z * z);
        }
    }
    return 0.0;
}

/* Moment class of row a: 0 conserved, 1 bulk, 2 shear, 3 ghost (kinetic). */
static int moment_class(int D, int a) {
    if (a <= D) return 0;
    if (D == 2) return a == 3 ? 1 : (a <= 5 ? 2 : 3);
    return a == 4 ? 1 : (a <= 9 ? 2 : 3);
}

int orc_basis(int D, double *M, double *b, int *cls) {
    int Q = lattice_q(D);
    if (Q < 0) return -1;
    double w[ORC_MAXQ];
    for (int i = 0; i < Q; ++i) w[i] = lattice_w(D, i);
    for (int a = 0; a < Q; ++a) {
        for (int i = 0; i < Q; ++i) {
            int c[3];
            lattice_c(D, i, c);
            M[a * Q + i] = seed_poly(D, a, c);
        }
        for (int p = 0; p < a; ++p) {
            double num = 0.0, den = 0.0;
            for (int i = 0; i < Q; ++i) {
                num += w[i] * M[a * Q + i] * M[p * Q + i];
                den += w[i] * M[p * Q + i] * M[p * Q + i];
            }
            for (int i = 0; i < Q; ++i) M[a * Q + i] -= (num / den) * M[p * Q + i];
        }
    }
    for (int a = 0; a < Q; ++a) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += w[i] * M[a * Q + i] * M[a * Q + i];
        b[a] = s;
        cls[a] = moment_class(D, a);
    }
    return 0;
}

/* Plain Gauss-Jordan inverse with partial pivoting (n <= ORC_MAXQ). */
static int invert(int n, const double *A, double *Ainv) {
    double T[ORC_MAXQ][2 * ORC_MAXQ];
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < 2 * n; ++k)
            T[r][k] = (k < n) ? A[r * n + k] : (k - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(T[r][col]) > fabs(T[piv][col])) piv = r;
        if (T[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int k = 0; k < 2 * n; ++k) {
                double t = T[col][k]; T[col][k] = T[piv][k]; T[piv][k] = t;
            }
        double d = T[col][col];
        for (int k = 0; k < 2 * n; ++k) T[col][k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double m = T[r][col];
            if (m == 0.0) continue;
            for (int k = 0; k < 2 * n; ++k) T[r][k] -= m * T[col][k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < n; ++k) Ainv[r * n + k] = T[r][n + k];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror and   */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds  */
/* of two 32x32->64 multiplications, with a Weyl key schedule.               */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Thermal-noise normals.  The paper fixes only that the noise is Gaussian  */
/* and uncorrelated in space and time; the generator is the library's own  */
/* choice and is stated exactly so that two independent implementations can */
/* agree on it:                                                             */
/*   words w_0, w_1, ... : Philox4x32-10 outputs of blocks 0, 1, ..., with   */
/*     key (seed low 32 bits, replica),                                     */
/*     counter (node, step low 32 bits, block, seed high 32 bits);          */
/*   pair k uses the radius uniform u_a = (floor(w_k / 2^9) + 1/2) / 2^23    */
/*     and the angle uniform u_b = (h_k + 1/2) / 2^16 of a 16-bit field h_k: */
/*     D2Q9 (3 pairs, block 0):  h_0 = high half of w_3, h_1 = low half of   */
/*       w_3, h_2 = (low byte of w_0) * 256 + (low byte of w_1);             */
/*     D3Q19 (8 pairs, blocks 0-2): h_k = the k-th 16-bit half of w_8..w_11, */
/*       high half first;                                                   */
/*   (z_2k, z_2k+1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b);           */
/* normal m goes to the m-th non-conserved moment (a = D+1+m).              */
/* ------------------------------------------------------------------------ */
void orc_normals(int D, int64_t node, int64_t step, uint64_t seed, uint32_t replica, double *xi) {
    int Q = lattice_q(D);
    int nn = Q - D - 1;
    int npairs = (nn + 1) / 2;
    int nblocks = (D == 2) ? 1 : 3;
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), replica};
    uint32_t w[12];
    for (int blk = 0; blk < nblocks; ++blk) {
        uint32_t ctr[4] = {(uint32_t)node, (uint32_t)step, (uint32_t)blk, (uint32_t)(seed >> 32)};
        orc_philox4x32_10(ctr, key, w + 4 * blk);
    }
    int k = 0;
    for (int p = 0; p < npairs; ++p) {
        uint32_t h;
        if (D == 2) {
            if (p == 0) h = w[3] >> 16;
            else if (p == 1) h = w[3] & 0xffffu;
            else h = ((w[0] & 0xffu) << 8) | (w[1] & 0xffu);
        } else {
            uint32_t word = w[8 + p / 2];
            h = (p % 2 == 0) ? (word >> 16) : (word & 0xffffu);
        }
        double ua = ((double)(w[p] >> 9) + 0.5) / 8388608.0;
        double ub = ((double)h + 0.5) / 65536.0;
        double rad = sqrt(-2.0 * log(ua));
        double ang = 2.0 * M_PI * ub;
        xi[k++] = rad * cos(ang);
        if (k < nn) xi[k++] = rad * sin(ang);
    }
}

/* ------------------------------------------------------------------------ */
/* Field helpers.                                                           */
/* ------------------------------------------------------------------------ */
static int64_t wrap(int64_t v, int64_t n) {
    int64_t r = v % n;
    return r < 0 ? r + n : r;
}

static int64_t node_index(int64_t x, int64_t y, int64_t z, int nx, int ny) {
    return x + (int64_t)nx * (y + (int64_t)ny * z);
}

int orc_density(const double *f, int D, int nx, int ny, int nz, double *n) {
    int Q = lattice_q(D);
    if (Q < 0) return -1;
    int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        double acc = 0.0;
        for (int i = 0; i < Q; ++i) acc += f[(int64_t)i * N + s];
        n[s] = acc;
    }
    return 0;
}

/* Eq. (1): F(x) = G psi(x) sum_a w(|e_a|^2) psi(x + e_a) e_a, periodic. */
int orc_force_from_psi(const double *psi, int D, int nx, int ny, int nz, int stencil,
                       double G, double *F) {
    int nf;
    int e[3 * ORC_MAXF];
    double we[ORC_MAXF];
    if (orc_stencil(D, stencil, &nf, e, we) != 0) return -1;
    int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t s = node_index(x, y, z, nx, ny);
                double acc[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < nf; ++a) {
                    int64_t t = node_index(wrap(x + e[3 * a], nx), wrap(y + e[3 * a + 1], ny),
                                           wrap(z + e[3 * a + 2], nz), nx, ny);
                    for (int d = 0; d < 3; ++d) acc[d] += we[a] * psi[t] * e[3 * a + d];
                }
                for (int d = 0; d < D; ++d) F[(int64_t)d * N + s] = G * psi[s] * acc[d];
            }
    return 0;
}

/* Per-node covariance factor of the noise populations: eta = B xi, with    */
/* B (Q x (Q-D-1)) = M^{-1} restricted to the non-conserved moments, times  */
/* the moment amplitudes sqrt(mu n b_a (1 - (1 - lam_a)^2)), mu = kBT/c_s^2. */
/* The paper fixes the variance only up to "proportional to k_B theta"; the */
/* constant is read from the ideal-gas limit of the exact S(k), Eq. (16):   */
/* S = n0 kBT / T at G = 0.                                                 */
static void moment_rates(int D, double lb, double ls, double lg, double *lam) {
    int Q = lattice_q(D);
    for (int a = 0; a < Q; ++a) {
        int k = moment_class(D, a);
        lam[a] = (k == 0) ? 1.0 : (k == 1 ? lb : (k == 2 ? ls : lg));
    }
}

int orc_noise_matrix(int D, double n, double kBT, double lb, double ls, double lg, double *B) {
    int Q = lattice_q(D);
    if (Q < 0) return -1;
    double M[ORC_MAXQ * ORC_MAXQ], Mi[ORC_MAXQ * ORC_MAXQ], b[ORC_MAXQ], lam[ORC_MAXQ];
    int cls[ORC_MAXQ];
    orc_basis(D, M, b, cls);
    if (invert(Q, M, Mi) != 0) return -2;
    moment_rates(D, lb, ls, lg, lam);
    double mu = kBT / CS2;
    int nn = Q - D - 1;
    for (int i = 0; i < Q; ++i)
        for (int k = 0; k < nn; ++k) {
            int a = D + 1 + k;
            double g = 1.0 - lam[a];
            double amp = sqrt(mu * n * b[a] * (1.0 - g * g));
            B[i * nn + k] = Mi[i * Q + a] * amp;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One or more steps of Eq. (12), in place on f (state at time t0 on entry,  */
/* t0 + nsteps on exit).                                                    */
/* ------------------------------------------------------------------------ */
int orc_step(double *f, int D, int nx, int ny, int nz, int stencil, double G,
             double lam_bulk, double lam_shear, double lam_ghost, double kBT,
             uint64_t seed, uint32_t replica, int64_t t0, int64_t nsteps) {
    int Q = lattice_q(D);
    if (Q < 0 || nx < 1 || ny < 1 || nz < 1 || (D == 2 && nz != 1)) return -1;
    if (stencil_weight(D, stencil, 1) < 0.0) return -1;
    int64_t N = (int64_t)nx * ny * nz;

    double M[ORC_MAXQ * ORC_MAXQ], Mi[ORC_MAXQ * ORC_MAXQ], b[ORC_MAXQ], lam[ORC_MAXQ];
    int cls[ORC_MAXQ];
    orc_basis(D, M, b, cls);
    if (invert(Q, M, Mi) != 0) return -2;
    moment_rates(D, lam_bulk, lam_shear, lam_ghost, lam);
    const double mu = kBT / CS2;
    const int nn = Q - D - 1;
    int cv[ORC_MAXQ][3];
    double wv[ORC_MAXQ];
    for (int i = 0; i < Q; ++i) {
        lattice_c(D, i, cv[i]);
        wv[i] = lattice_w(D, i);
    }

    double *n = (double *)malloc(sizeof(double) * N);
    double *psi = (double *)malloc(sizeof(double) * N);
    double *F = (double *)calloc((size_t)3 * N, sizeof(double));
    double *fs = (double *)malloc(sizeof(double) * Q * N);
    if (!n || !psi || !F || !fs) {
        free(n); free(psi); free(F); free(fs);
        return -3;
    }

    for (int64_t t = t0; t < t0 + nsteps; ++t) {
        /* 1-2. density and pseudopotential psi = exp(-1/n) */
        orc_density(f, D, nx, ny, nz, n);
        for (int64_t s = 0; s < N; ++s) psi[s] = exp(-1.0 / n[s]);
        /* 3. Shan-Chen force, Eq. (1) */
        orc_force_from_psi(psi, D, nx, ny, nz, stencil, G, F);

        /* 4-5. collision with Guo forcing and moment-space noise, per node */
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < N; ++s) {
            double fi[ORC_MAXQ], feq[ORC_MAXQ], Si[ORC_MAXQ];
            double m[ORC_MAXQ], meq[ORC_MAXQ], sm[ORC_MAXQ], ms[ORC_MAXQ], xi[ORC_MAXQ];
            double j[3] = {0.0, 0.0, 0.0}, Fv[3] = {0.0, 0.0, 0.0}, u[3];
            double rho = n[s];
            for (int i = 0; i < Q; ++i) {
                fi[i] = f[(int64_t)i * N + s];
                for (int d = 0; d < 3; ++d) j[d] += fi[i] * cv[i][d];
            }
            for (int d = 0; d < D; ++d) Fv[d] = F[(int64_t)d * N + s];
            for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * Fv[d]) / rho;
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            double uF = u[0] * Fv[0] + u[1] * Fv[1] + u[2] * Fv[2];
            for (int i = 0; i < Q; ++i) {
                double cu = cv[i][0] * u[0] + cv[i][1] * u[1] + cv[i][2] * u[2];
                double cF = cv[i][0] * Fv[0] + cv[i][1] * Fv[1] + cv[i][2] * Fv[2];
                /* second-order equilibrium */
                feq[i] = wv[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
                /* Guo source: w_i [ (c_i - u)/c_s^2 + (c_i.u) c_i / c_s^4 ] . F */
                Si[i] = wv[i] * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2));
            }
            for (int a = 0; a < Q; ++a) {
                m[a] = meq[a] = sm[a] = 0.0;
                for (int i = 0; i < Q; ++i) {
                    m[a] += M[a * Q + i] * fi[i];
                    meq[a] += M[a * Q + i] * feq[i];
                    sm[a] += M[a * Q + i] * Si[i];
                }
            }
            if (kBT > 0.0) orc_normals(D, s, t, seed, replica, xi);
            for (int a = 0; a < Q; ++a) {
                double Na = 0.0;
                if (a > D && kBT > 0.0) {
                    double g = 1.0 - lam[a];
                    Na = sqrt(mu * rho * b[a] * (1.0 - g * g)) * xi[a - D - 1];
                }
                ms[a] = m[a] - lam[a] * (m[a] - meq[a]) + (1.0 - 0.5 * lam[a]) * sm[a] + Na;
            }
            (void)nn;
            for (int i = 0; i < Q; ++i) {
                double acc = 0.0;
                for (int a = 0; a < Q; ++a) acc += Mi[i * Q + a] * ms[a];
                fs[(int64_t)i * N + s] = acc;
            }
        }

        /* 6. periodic streaming: f_i(x + c_i, t + 1) = f*_i(x, t) */
#pragma omp parallel for collapse(2) schedule(static)
        for (int i = 0; i < Q; ++i)
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        int64_t src = node_index(x, y, z, nx, ny);
                        int64_t dst = node_index(wrap(x + cv[i][0], nx), wrap(y + cv[i][1], ny),
                                                 wrap(z + cv[i][2], nz), nx, ny);
                        f[(int64_t)i * N + dst] = fs[(int64_t)i * N + src];
                    }
    }
    free(n); free(psi); free(F); free(fs);
    return 0;
}

/* Total mass sum_x n and momentum sum_x j of a state (the momentum of the  */
/* streamed state; sum_x F vanishes, so it is conserved as well).           */
int orc_conserved(const double *f, int D, int nx, int ny, int nz, double *mass, double *mom) {
    int Q = lattice_q(D);
    if (Q < 0) return -1;
    int64_t N = (int64_t)nx * ny * nz;
    double m = 0.0, p[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        int c[3];
        lattice_c(D, i, c);
        for (int64_t s = 0; s < N; ++s) {
            double v = f[(int64_t)i * N + s];
            m += v;
            for (int d = 0; d < 3; ++d) p[d] += v * c[d];
        }
    }
    *mass = m;
    for (int d = 0; d < D; ++d) mom[d] = p[d];
    return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops (timing of the oracle on one core). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
