/*
 * sanitize_main.c -- a small driver of the FP64 oracle (test infrastructure),
 * built with the host address and undefined-behaviour sanitizers by
 * tests/test_oracle_sanitizers.py: it runs every exported routine of
 * fsc_oracle.c on small 2D and 3D lattices, including the degenerate and
 * wrap-around sizes, and exits non-zero on a failed check.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_lattice(int D, int *Q, int *c, double *w);
int orc_stencil(int D, int stencil, int *nf, int *e, double *w);
int orc_basis(int D, double *M, double *b, int *cls);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals(int D, int64_t node, int64_t step, uint64_t seed, uint32_t replica, double *xi);
int orc_density(const double *f, int D, int nx, int ny, int nz, double *n);
int orc_force_from_psi(const double *psi, int D, int nx, int ny, int nz, int stencil, double G,
                       double *F);
int orc_noise_matrix(int D, double n, double kBT, double lb, double ls, double lg, double *B);
int orc_step(double *f, int D, int nx, int ny, int nz, int stencil, double G, double lam_bulk,
             double lam_shear, double lam_ghost, double kBT, uint64_t seed, uint32_t replica,
             int64_t t0, int64_t nsteps);
int orc_conserved(const double *f, int D, int nx, int ny, int nz, double *mass, double *mom);

static int run_case(int D, int nx, int ny, int nz, int stencil) {
    int Q, c[3 * 19];
    double w[19];
    if (orc_lattice(D, &Q, c, w) != 0) return 1;
    const int64_t N = (int64_t)nx * ny * nz;
    double *f = malloc(sizeof(double) * Q * N);
    double *n = malloc(sizeof(double) * N);
    double *F = malloc(sizeof(double) * 3 * N);
    if (!f || !n || !F) return 2;
    for (int i = 0; i < Q; ++i)
        for (int64_t s = 0; s < N; ++s) f[i * N + s] = w[i] * (0.8 + 0.01 * (double)((s * 7 + i) % 13));
    double m0, p0[3], m1, p1[3];
    orc_conserved(f, D, nx, ny, nz, &m0, p0);
    const double G = 2.9;
    if (orc_step(f, D, nx, ny, nz, stencil, G, 0.9, 1.2, 1.5, 1e-4, 7, 3, 11, 5) != 0) return 3;
    orc_conserved(f, D, nx, ny, nz, &m1, p1);
    if (fabs(m1 - m0) > 1e-12 * m0) return 4;
    if (orc_density(f, D, nx, ny, nz, n) != 0) return 5;
    for (int64_t s = 0; s < N; ++s) n[s] = exp(-1.0 / n[s]);
    if (orc_force_from_psi(n, D, nx, ny, nz, stencil, G, F) != 0) return 6;
    free(f);
    free(n);
    free(F);
    return 0;
}

int main(void) {
    int rc = 0;
    double M[19 * 19], b[19], B[19 * 15], xi[15], we[24];
    int cls[19], e[3 * 24], nf;
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    for (int D = 2; D <= 3; ++D) {
        rc |= orc_basis(D, M, b, cls);
        rc |= orc_noise_matrix(D, 0.7, 1e-3, 0.8, 1.2, 1.6, B);
        orc_normals(D, 12345, 678, 0x1234567890ull, 9, xi);
    }
    rc |= orc_stencil(2, 4, &nf, e, we) | orc_stencil(2, 8, &nf, e, we) | orc_stencil(3, 4, &nf, e, we);
    const int cases[][5] = {{2, 16, 12, 1, 4}, {2, 7, 5, 1, 8}, {2, 1, 1, 1, 4}, {2, 3, 2, 1, 8},
                            {3, 6, 5, 4, 4}, {3, 2, 3, 1, 4}, {3, 1, 1, 1, 4}};
    for (size_t k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k) {
        const int r = run_case(cases[k][0], cases[k][1], cases[k][2], cases[k][3], cases[k][4]);
        if (r) {
            fprintf(stderr, "case %zu failed (%d)\n", k, r);
            rc = 1;
        }
    }
    printf("oracle sanitizer driver: %s\n", rc ? "FAILED" : "ok");
    return rc ? 1 : 0;
}
