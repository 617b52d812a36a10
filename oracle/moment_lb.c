/*
 * Oracle: single-component lattice Boltzmann without populations
 * (test infrastructure only; see oracle.h).
 *
 * One time step, in the paper's order (Sec. II and Sec. III.A):
 *   1. at every node, reconstruct h_i from the stored hydro-fields H with the
 *      second-order operator of Eq. 4: equilibrium part Eq. 5 plus
 *      non-equilibrium part Eq. 6, ghost part g_i = 0;
 *   2. relax with the BGK rule of Eq. 7, h'_i = (1-omega) h_i + omega h_i^eq
 *      (Eq. 8 is the same expression written out);
 *   3. stream by pulling, h_i(x, t+1) = h'_i[H(x - c_i, t)] (Eq. 9, read as
 *      one assignment per direction: the sum printed on its right-hand side
 *      would not give a population);
 *   4. store the moments of the streamed set, Eqs. 1-3.
 * The stored state is therefore the post-streaming (pre-collision) set of
 * moments, which is what the fused approach of Sec. III.A stores.
 *
 * Readings of the paper used here:
 *   - "c_ia u_ia" in Eq. 4 is sum_a c_ia u_a / c_s^2 (second-order Hermite
 *     equilibrium);
 *   - P^eq, which the paper does not print, is the second moment of Eq. 5:
 *     P^eq_ab = rho c_s^2 delta_ab + rho u_a u_b;
 *   - the velocity is carried as the momentum density j = rho u.
 *
 * The post-collision populations are held in a temporary array of q*N
 * doubles: the oracle is a definition, not a memory-saving implementation.
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Eq. 5 (h_i^eq) and Eq. 6 (h_i^neq) at one node whose hydro-fields are
 * rho, j[3] and P[3][3]. */
void ora_hermite_parts(const ora_lat *L, double rho, const double j[3], double P[3][3],
                       double *heq, double *hneq)
{
    double u[3], Peq[3][3];
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Peq[a][b] = rho * ORA_CS2 * (a == b ? 1.0 : 0.0) + rho * u[a] * u[b];

    for (int i = 0; i < L->q; ++i) {
        double cu = 0.0;
        for (int a = 0; a < 3; ++a) cu += L->c[i][a] * u[a] / ORA_CS2;
        double Quu = 0.0, QdP = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                Quu += ora_Q(L, i, a, b) * u[a] * u[b];
                QdP += ora_Q(L, i, a, b) * (P[a][b] - Peq[a][b]);
            }
        heq[i] = L->w[i] * rho * (1.0 + cu + Quu);
        hneq[i] = L->w[i] * QdP;
    }
}

/* Hydro-fields of one node from the SoA arrays (single-component layout). */
void ora_load_node(const double *H, long N, long n, double *rho, double j[3], double P[3][3])
{
    double p6[6];
    *rho = H[0 * N + n];
    for (int a = 0; a < 3; ++a) j[a] = H[(1 + a) * N + n];
    for (int k = 0; k < 6; ++k) p6[k] = H[(4 + k) * N + n];
    ora_unpack_tensor(p6, P);
}

/* Eqs. 1-3: moments of a set of q populations. */
void ora_project(const ora_lat *L, const double *f, double *rho, double j[3], double P[3][3])
{
    *rho = 0.0;
    for (int a = 0; a < 3; ++a) {
        j[a] = 0.0;
        for (int b = 0; b < 3; ++b) P[a][b] = 0.0;
    }
    for (int i = 0; i < L->q; ++i) {
        *rho += f[i];
        for (int a = 0; a < 3; ++a) {
            j[a] += f[i] * L->c[i][a];
            for (int b = 0; b < 3; ++b) P[a][b] += f[i] * L->c[i][a] * L->c[i][b];
        }
    }
}

void ora_store_node(double *H, long N, long n, double rho, const double j[3], double P[3][3])
{
    H[0 * N + n] = rho;
    for (int a = 0; a < 3; ++a) H[(1 + a) * N + n] = j[a];
    H[4 * N + n] = P[0][0];
    H[5 * N + n] = P[1][1];
    H[6 * N + n] = P[2][2];
    H[7 * N + n] = P[0][1];
    H[8 * N + n] = P[0][2];
    H[9 * N + n] = P[1][2];
}

/* ---- exported single-node helpers (used by the identity tests) ---------- */

/* Eq. 4: h_i = h_i^eq + h_i^neq for one node; H holds the 10 hydro-fields. */
int ora_reconstruct(int q, const double *H, double *h)
{
    ora_lat L;
    double heq[ORA_QMAX], hneq[ORA_QMAX], P[3][3];
    if (ora_lattice_init(q, &L) != 0) return -1;
    ora_unpack_tensor(H + 4, P);
    ora_hermite_parts(&L, H[0], H + 1, P, heq, hneq);
    for (int i = 0; i < q; ++i) h[i] = heq[i] + hneq[i];
    return 0;
}

/* Eq. 7 applied to the reconstructed set of one node. */
int ora_collide_node(int q, double tau, const double *H, double *hpost)
{
    ora_lat L;
    double heq[ORA_QMAX], hneq[ORA_QMAX], P[3][3];
    double omega = 1.0 / tau;
    if (ora_lattice_init(q, &L) != 0) return -1;
    ora_unpack_tensor(H + 4, P);
    ora_hermite_parts(&L, H[0], H + 1, P, heq, hneq);
    for (int i = 0; i < q; ++i) {
        double h = heq[i] + hneq[i];
        hpost[i] = (1.0 - omega) * h + omega * heq[i];
    }
    return 0;
}

/* Eqs. 1-3 for one node. */
int ora_project_node(int q, const double *f, double *H)
{
    ora_lat L;
    double rho, j[3], P[3][3];
    if (ora_lattice_init(q, &L) != 0) return -1;
    ora_project(&L, f, &rho, j, P);
    H[0] = rho;
    for (int a = 0; a < 3; ++a) H[1 + a] = j[a];
    H[4] = P[0][0]; H[5] = P[1][1]; H[6] = P[2][2];
    H[7] = P[0][1]; H[8] = P[0][2]; H[9] = P[1][2];
    return 0;
}

/* ---- the time step ------------------------------------------------------- */

static void moment_step(const ora_lat *L, int nx, int ny, int nz, double omega,
                        const double *Hin, double *Hout, double *hpost)
{
    long N = (long)nx * ny * nz;
    int q = L->q;

    /* Reconstruct (Eq. 4) and collide (Eq. 7) at every node. */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double rho, j[3], P[3][3], heq[ORA_QMAX], hneq[ORA_QMAX];
        ora_load_node(Hin, N, n, &rho, j, P);
        ora_hermite_parts(L, rho, j, P, heq, hneq);
        for (int i = 0; i < q; ++i) {
            double h = heq[i] + hneq[i];
            hpost[(long)i * N + n] = (1.0 - omega) * h + omega * heq[i];
        }
    }

    /* Pull (Eq. 9) and take the moments of the streamed set (Eqs. 1-3). */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double f[ORA_QMAX], rho, j[3], P[3][3];
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                for (int i = 0; i < q; ++i) {
                    long src = ora_neighbour(nx, ny, nz, x, y, z, -L->c[i][0], -L->c[i][1], -L->c[i][2]);
                    f[i] = hpost[(long)i * N + src];
                }
                ora_project(L, f, &rho, j, P);
                ora_store_node(Hout, N, n, rho, j, P);
            }
}

/* Advances the single-component state H (10 fields, in place) by nsteps.
 * Returns 0, or -1 on a bad argument or allocation failure. */
int ora_moment_run(int q, int nx, int ny, int nz, double tau, int nsteps, double *H)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0 || nx < 1 || ny < 1 || nz < 1 || nsteps < 0) return -1;
    long N = (long)nx * ny * nz;
    double *tmp = malloc(sizeof(double) * 10 * N);
    double *hpost = malloc(sizeof(double) * q * N);
    if (!tmp || !hpost) {
        free(tmp);
        free(hpost);
        return -1;
    }
    for (int t = 0; t < nsteps; ++t) {
        moment_step(&L, nx, ny, nz, 1.0 / tau, H, tmp, hpost);
        memcpy(H, tmp, sizeof(double) * 10 * N);
    }
    free(tmp);
    free(hpost);
    return 0;
}
