/*
 * Oracle: conventional, population-storing lattice Boltzmann
 * (test infrastructure only; see oracle.h).
 *
 * This is the "LB with populations" the paper compares against (Sec. IV):
 * the populations f_i are the stored state.  Per step, at every node:
 * moments by Eqs. 1-3, equilibrium by Eq. 5, BGK relaxation by Eq. 7, then
 * pull streaming f_i(x, t+1) = f'_i(x - c_i) with two population buffers.
 *
 * regularize = 1 replaces f_i by the reconstruction of its own moments
 * (Eq. 4, h = h^eq + h^neq, ghosts dropped) before relaxing: this is the
 * regularized scheme the paper cites for Eq. 6.  The population-free scheme
 * must coincide with it to rounding, which is what makes it a check of the
 * moment oracle through a code path that stores populations.
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* f = R(H) (Eq. 4) for every node: populations from a single-component
 * moment array. */
int ora_populations_from_moments(int q, long N, const double *H, double *f)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double rho, j[3], P[3][3], heq[ORA_QMAX], hneq[ORA_QMAX];
        ora_load_node(H, N, n, &rho, j, P);
        ora_hermite_parts(&L, rho, j, P, heq, hneq);
        for (int i = 0; i < q; ++i) f[(long)i * N + n] = heq[i] + hneq[i];
    }
    return 0;
}

/* H = P f (Eqs. 1-3) for every node. */
int ora_moments_from_populations(int q, long N, const double *f, double *H)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fn[ORA_QMAX], rho, j[3], P[3][3];
        for (int i = 0; i < q; ++i) fn[i] = f[(long)i * N + n];
        ora_project(&L, fn, &rho, j, P);
        ora_store_node(H, N, n, rho, j, P);
    }
    return 0;
}

static void population_step(const ora_lat *L, int nx, int ny, int nz, double omega, int regularize,
                            const double *fin, double *fout, double *fpost)
{
    long N = (long)nx * ny * nz;
    int q = L->q;

    /* Collide (Eq. 7) at every node. */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double fn[ORA_QMAX], rho, j[3], P[3][3], heq[ORA_QMAX], hneq[ORA_QMAX];
        for (int i = 0; i < q; ++i) fn[i] = fin[(long)i * N + n];
        ora_project(L, fn, &rho, j, P);
        ora_hermite_parts(L, rho, j, P, heq, hneq);
        for (int i = 0; i < q; ++i) {
            double fi = regularize ? heq[i] + hneq[i] : fn[i];
            fpost[(long)i * N + n] = (1.0 - omega) * fi + omega * heq[i];
        }
    }

    /* Pull streaming. */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                for (int i = 0; i < q; ++i) {
                    long src = ora_neighbour(nx, ny, nz, x, y, z, -L->c[i][0], -L->c[i][1], -L->c[i][2]);
                    fout[(long)i * N + n] = fpost[(long)i * N + src];
                }
            }
}

/* Advances the populations f (q fields, in place) by nsteps. */
int ora_population_run(int q, int nx, int ny, int nz, double tau, int regularize, int nsteps, double *f)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0 || nx < 1 || ny < 1 || nz < 1 || nsteps < 0) return -1;
    long N = (long)nx * ny * nz;
    double *tmp = malloc(sizeof(double) * q * N);
    double *fpost = malloc(sizeof(double) * q * N);
    if (!tmp || !fpost) {
        free(tmp);
        free(fpost);
        return -1;
    }
    for (int t = 0; t < nsteps; ++t) {
        population_step(&L, nx, ny, nz, 1.0 / tau, regularize, f, tmp, fpost);
        memcpy(f, tmp, sizeof(double) * q * N);
    }
    free(tmp);
    free(fpost);
    return 0;
}
