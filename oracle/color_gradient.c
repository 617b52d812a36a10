/*
 * Oracle: two-component colour-gradient lattice Boltzmann, without and with
 * populations (test infrastructure only; see oracle.h).
 *
 * The paper carries two species on one flow field with the colour-gradient
 * model (Sec. III.A): per species only a density is stored (2 extra arrays),
 * the density gradient is evaluated on the post-streaming state before the
 * collision, and "perturbation" and "re-colouring" operators are applied to
 * the populations of Eq. 8.  The paper names the model but does not print
 * its operators; the readings used here are:
 *
 *   phase field     phi = (rho1 - rho2)/(rho1 + rho2)           (Sec. III.B)
 *   colour gradient G = (1/c_s^2) sum_i w_i c_i phi(y + c_i)   (isotropic)
 *   smoothed norm   D = sqrt(|G|^2 + EPS_G^2), EPS_G = 1e-3
 *   normal          n = G / D: the unit normal on every interface (|G| ~ 0.1-0.5
 *                   there, relative deviation EPS_G^2/(2|G|^2) < 1e-4), and a
 *                   smooth fade to zero where the gradient vanishes (at
 *                   saddle points of phi between two interfaces the unit
 *                   normal is undefined, so no direction is preferred)
 *   perturbation    Df_i = (A/2) [w_i (c_i.G)^2 - B_i |G|^2] / D, B_0 = w_0 - 2/3,
 *                   B_i = w_i otherwise (three-dimensional operator of Liu,
 *                   Valocchi and Kang, written with G instead of |G| n); it
 *                   carries no mass and no momentum, and its second moment is
 *                   DP_ab = (A/9) (G_a G_b - |G|^2 delta_ab) / D, smooth in G;
 *                   surface tension sigma = 2 A tau / 9
 *   recolouring     f^k_i = (rho^k/rho) f'_i
 *                           + s_k beta (rho1 rho2/rho) w_i (c_i.n)/|c_i|,
 *                   s_1 = +1, s_2 = -1, zero for the rest velocity
 *                   (Latva-Kokko and Rothman form with f^eq(rho, u=0) = w_i rho)
 *   one relaxation time for the mixture (viscosity ratio one, Sec. IV)
 *
 *
 * Near-contact force (the LBNCI extension, Sec. III.B), optional: the paper
 * gives F_rep = -A_h[h(x)] n delta_I with delta_I proportional to grad phi,
 * but neither how h(x) is found nor the form of A_h nor how the force enters
 * the scheme.  Readings:
 *   delta_I = |G|/2 (integrates to one across an interface, phi going from
 *             -1 to 1), n = -G/|G| the outward normal of the species-1 phase,
 *             so F = (A_h/2) G: a repulsion pushing each interface back into
 *             its own drop;
 *   h(x)    : from node x, probe the nodes x + k c*, k = 1..h_max, along the
 *             lattice direction c* closest to n (largest c.n/|c|; exact ties
 *             go to the shorter |c|, then the larger c_x, c_y, c_z); a film
 *             is crossed when a probe with phi < 0 (or phi(x) < 0) is
 *             followed by one with phi > 0, and h is the k of that probe;
 *   A_h[h]  = A_h if a film is crossed within h_max probes, else 0;
 *   forcing : Guo's scheme on the mixture: the equilibrium takes
 *             u* = (j + F/2)/rho, and (1 - omega/2) S_i is added with
 *             S_i = w_i [(c_i - u*).F / c_s^2 + (c_i.u*)(c_i.F) / c_s^4];
 *             the stored momentum of the next step gains F.
 *   The paper prints no near-contact values, so these readings are parity
 *   unpinned as readings; what they compute is pinned (film distances and
 *   forces between flat slabs in closed form, the forced collision's moments,
 *   momentum gain equal to the total force).
 *
 * Without populations the perturbation enters through its second moment
 * only: the collided tensor is P' = P^eq + (1-omega)(P - P^eq) + DP and the
 * populations are the Eq. 4 reconstruction of it, so the operator's
 * fourth-order part is a ghost and is dropped with the others.  The stored
 * state is the post-streaming one, so the gradient is available before the
 * collision, as the paper requires.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define EPS_G 1e-3

/* Two-component SoA layout: rho1, rho2, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz. */
static void load_node2(const double *H, long N, long n, double *rho1, double *rho2, double j[3],
                       double P[3][3])
{
    double p6[6];
    *rho1 = H[0 * N + n];
    *rho2 = H[1 * N + n];
    for (int a = 0; a < 3; ++a) j[a] = H[(2 + a) * N + n];
    for (int k = 0; k < 6; ++k) p6[k] = H[(5 + k) * N + n];
    ora_unpack_tensor(p6, P);
}

static void store_node2(double *H, long N, long n, double rho1, double rho2, const double j[3],
                        double P[3][3])
{
    H[0 * N + n] = rho1;
    H[1 * N + n] = rho2;
    for (int a = 0; a < 3; ++a) H[(2 + a) * N + n] = j[a];
    H[5 * N + n] = P[0][0];
    H[6 * N + n] = P[1][1];
    H[7 * N + n] = P[2][2];
    H[8 * N + n] = P[0][1];
    H[9 * N + n] = P[0][2];
    H[10 * N + n] = P[1][2];
}

/* Colour gradient G at node (x,y,z) from the phase field, the smoothed norm
 * D = sqrt(|G|^2 + EPS_G^2), and the recolouring direction n = G / D. */
static void colour_gradient(const ora_lat *L, const double *phi, int nx, int ny, int nz, int x, int y,
                            int z, double G[3], double *D, double nrm[3])
{
    for (int a = 0; a < 3; ++a) G[a] = 0.0;
    for (int i = 0; i < L->q; ++i) {
        long nb = ora_neighbour(nx, ny, nz, x, y, z, L->c[i][0], L->c[i][1], L->c[i][2]);
        for (int a = 0; a < 3; ++a) G[a] += L->w[i] * L->c[i][a] * phi[nb] / ORA_CS2;
    }
    *D = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + EPS_G * EPS_G);
    for (int a = 0; a < 3; ++a) nrm[a] = G[a] / *D;
}

static double speed(const ora_lat *L, int i)
{
    return sqrt((double)(L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]));
}

/* Recolouring term beta (rho1 rho2/rho) w_i (c_i.n)/|c_i| (species 1 sign). */
static double recolour_term(const ora_lat *L, int i, double beta, double rho1, double rho2,
                            const double nrm[3])
{
    if (i == 0 || speed(L, i) == 0.0) return 0.0;
    double cn = L->c[i][0] * nrm[0] + L->c[i][1] * nrm[1] + L->c[i][2] * nrm[2];
    return beta * rho1 * rho2 / (rho1 + rho2) * L->w[i] * cn / speed(L, i);
}

/* ---- near-contact force ---------------------------------------------------- */

/* Does direction i come before direction k in the canonical order used to
 * break exact ties (shorter |c| first, then larger c_x, c_y, c_z)? */
static int canonical_before(const ora_lat *L, int i, int k)
{
    int si = L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2];
    int sk = L->c[k][0] * L->c[k][0] + L->c[k][1] * L->c[k][1] + L->c[k][2] * L->c[k][2];
    if (si != sk) return si < sk;
    for (int a = 0; a < 3; ++a)
        if (L->c[i][a] != L->c[k][a]) return L->c[i][a] > L->c[k][a];
    return 0;
}

/* Force field F (3 arrays of N) and the film distance h (N values, 0 where no
 * film is found) from the phase field; see the readings above. */
static void nc_force(const ora_lat *L, int nx, int ny, int nz, const double *phi, double Ah, int hmax,
                     double *F, int *hout)
{
    long N = (long)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double G[3], D, nrm[3];
                colour_gradient(L, phi, nx, ny, nz, x, y, z, G, &D, nrm);
                int h = 0;
                if (G[0] != 0.0 || G[1] != 0.0 || G[2] != 0.0) {
                    int best = -1;
                    double best_score = 0.0;
                    for (int i = 0; i < L->q; ++i) {
                        double sp = speed(L, i);
                        if (sp == 0.0) continue;
                        /* c.n/|c| with n = -G/|G|; the common 1/|G| is left out */
                        double score = -(L->c[i][0] * G[0] + L->c[i][1] * G[1] + L->c[i][2] * G[2]) / sp;
                        if (best < 0 || score > best_score ||
                            (score == best_score && canonical_before(L, i, best))) {
                            best = i;
                            best_score = score;
                        }
                    }
                    int seen = phi[n] < 0.0;
                    for (int k = 1; k <= hmax; ++k) {
                        long m = ora_neighbour(nx, ny, nz, x, y, z, k * L->c[best][0], k * L->c[best][1],
                                               k * L->c[best][2]);
                        if (phi[m] < 0.0) {
                            seen = 1;
                        } else if (phi[m] > 0.0 && seen) {
                            h = k;
                            break;
                        }
                    }
                }
                for (int a = 0; a < 3; ++a) F[a * N + n] = h ? 0.5 * Ah * G[a] : 0.0;
                if (hout) hout[n] = h;
            }
}

/* Guo's forcing term S_i for force F at velocity u (see the readings). */
static double guo_term(const ora_lat *L, int i, const double u[3], const double F[3])
{
    double cu = 0.0, cF = 0.0, uF = 0.0;
    for (int a = 0; a < 3; ++a) {
        cu += L->c[i][a] * u[a];
        cF += L->c[i][a] * F[a];
        uF += u[a] * F[a];
    }
    return L->w[i] * ((cF - uF) / ORA_CS2 + cu * cF / (ORA_CS2 * ORA_CS2));
}

/* Equilibrium part at the shifted momentum j + F/2 and the shifted velocity. */
static void forced_equilibrium(const ora_lat *L, double rho, const double j[3], double P[3][3],
                               const double F[3], double *heqs, double us[3])
{
    double js[3], tmp[ORA_QMAX];
    for (int a = 0; a < 3; ++a) {
        js[a] = j[a] + 0.5 * F[a];
        us[a] = js[a] / rho;
    }
    ora_hermite_parts(L, rho, js, P, heqs, tmp);
}

int ora_nc_force(int q, int nx, int ny, int nz, const double *phi, double Ah, int hmax, double *F, int *h)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0 || nx < 1 || ny < 1 || nz < 1 || hmax < 0) return -1;
    nc_force(&L, nx, ny, nz, phi, Ah, hmax, F, h);
    return 0;
}

/* Post-collision mixture populations of one node under a body force F:
 * BGK with Guo's forcing, without perturbation and recolouring (for tests of
 * the forcing alone).  P is row-major 3x3. */
int ora_forced_collide_node(int q, double tau, double rho, const double *j, const double *P9, const double *F,
                            double *fpost)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
    double P[3][3], jj[3], Fn[3], heq[ORA_QMAX], hneq[ORA_QMAX], heqs[ORA_QMAX], us[3];
    for (int a = 0; a < 3; ++a) {
        jj[a] = j[a];
        Fn[a] = F[a];
        for (int b = 0; b < 3; ++b) P[a][b] = P9[3 * a + b];
    }
    double omega = 1.0 / tau;
    ora_hermite_parts(&L, rho, jj, P, heq, hneq);
    forced_equilibrium(&L, rho, jj, P, Fn, heqs, us);
    for (int i = 0; i < q; ++i) {
        double hi = heq[i] + hneq[i];
        fpost[i] = hi - omega * (hi - heqs[i]) + (1.0 - 0.5 * omega) * guo_term(&L, i, us, Fn);
    }
    return 0;
}

/* ---- without populations ------------------------------------------------- */

static void cg_moment_step(const ora_lat *L, int nx, int ny, int nz, double omega, double A,
                           double beta, double Ah, int hmax, const double *Hin, double *Hout, double *phi,
                           double *f1post, double *f2post, double *F)
{
    long N = (long)nx * ny * nz;
    int q = L->q;

#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) phi[n] = (Hin[n] - Hin[N + n]) / (Hin[n] + Hin[N + n]);
    const int forced = Ah != 0.0;
    if (forced) nc_force(L, nx, ny, nz, phi, Ah, hmax, F, NULL);

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double rho1, rho2, j[3], P[3][3], G[3], D, nrm[3];
                double heq[ORA_QMAX], hneq[ORA_QMAX], DP[3][3];
                load_node2(Hin, N, n, &rho1, &rho2, j, P);
                double rho = rho1 + rho2;
                colour_gradient(L, phi, nx, ny, nz, x, y, z, G, &D, nrm);
                ora_hermite_parts(L, rho, j, P, heq, hneq);
                double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) DP[a][b] = A / 9.0 * (G[a] * G[b] - (a == b ? G2 : 0.0)) / D;
                double heqs[ORA_QMAX], us[3], Fn[3];
                if (forced) {
                    for (int a = 0; a < 3; ++a) Fn[a] = F[a * N + n];
                    forced_equilibrium(L, rho, j, P, Fn, heqs, us);
                }
                for (int i = 0; i < q; ++i) {
                    /* Eq. 7 (with Guo's forcing if forced), then the
                     * reconstructed perturbation w_i Q_i:DP. */
                    double hpost;
                    if (forced) {
                        double hi = heq[i] + hneq[i];
                        hpost = hi - omega * (hi - heqs[i]) + (1.0 - 0.5 * omega) * guo_term(L, i, us, Fn);
                    } else {
                        hpost = (1.0 - omega) * (heq[i] + hneq[i]) + omega * heq[i];
                    }
                    double QDP = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) QDP += ora_Q(L, i, a, b) * DP[a][b];
                    hpost += L->w[i] * QDP;
                    double rc = recolour_term(L, i, beta, rho1, rho2, nrm);
                    f1post[(long)i * N + n] = rho1 / rho * hpost + rc;
                    f2post[(long)i * N + n] = rho2 / rho * hpost - rc;
                }
            }

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double f[ORA_QMAX], rho1 = 0.0, rho2 = 0.0, rho, j[3], P[3][3];
                for (int i = 0; i < q; ++i) {
                    long src = ora_neighbour(nx, ny, nz, x, y, z, -L->c[i][0], -L->c[i][1], -L->c[i][2]);
                    double a1 = f1post[(long)i * N + src], a2 = f2post[(long)i * N + src];
                    rho1 += a1;
                    rho2 += a2;
                    f[i] = a1 + a2;
                }
                ora_project(L, f, &rho, j, P);
                store_node2(Hout, N, n, rho1, rho2, j, P);
            }
}

/* Advances the two-component state H (11 fields, in place) by nsteps. */
int ora_cg_moment_run(int q, int nx, int ny, int nz, double tau, double A, double beta, double Ah, int hmax,
                      int nsteps, double *H)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0 || nx < 1 || ny < 1 || nz < 1 || nsteps < 0 || hmax < 0) return -1;
    long N = (long)nx * ny * nz;
    double *tmp = malloc(sizeof(double) * 11 * N);
    double *phi = malloc(sizeof(double) * N);
    double *f1 = malloc(sizeof(double) * q * N);
    double *f2 = malloc(sizeof(double) * q * N);
    double *F = malloc(sizeof(double) * 3 * N);
    int rc = 0;
    if (!tmp || !phi || !f1 || !f2 || !F) {
        rc = -1;
    } else {
        for (int t = 0; t < nsteps; ++t) {
            cg_moment_step(&L, nx, ny, nz, 1.0 / tau, A, beta, Ah, hmax, H, tmp, phi, f1, f2, F);
            memcpy(H, tmp, sizeof(double) * 11 * N);
        }
    }
    free(tmp);
    free(phi);
    free(f1);
    free(f2);
    free(F);
    return rc;
}

/* ---- with populations ------------------------------------------------------ */

static void cg_population_step(const ora_lat *L, int nx, int ny, int nz, double omega, double A,
                               double beta, int regularize, double Ah, int hmax, const double *f1in,
                               const double *f2in, double *f1out, double *f2out, double *phi, double *f1post,
                               double *f2post, double *F)
{
    long N = (long)nx * ny * nz;
    int q = L->q;

#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double r1 = 0.0, r2 = 0.0;
        for (int i = 0; i < q; ++i) {
            r1 += f1in[(long)i * N + n];
            r2 += f2in[(long)i * N + n];
        }
        phi[n] = (r1 - r2) / (r1 + r2);
    }
    const int forced = Ah != 0.0;
    if (forced) nc_force(L, nx, ny, nz, phi, Ah, hmax, F, NULL);

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double f[ORA_QMAX], rho1 = 0.0, rho2 = 0.0, rho, j[3], P[3][3];
                double heq[ORA_QMAX], hneq[ORA_QMAX], Df[ORA_QMAX], G[3], D, nrm[3];
                for (int i = 0; i < q; ++i) {
                    rho1 += f1in[(long)i * N + n];
                    rho2 += f2in[(long)i * N + n];
                    f[i] = f1in[(long)i * N + n] + f2in[(long)i * N + n];
                }
                ora_project(L, f, &rho, j, P);
                ora_hermite_parts(L, rho, j, P, heq, hneq);
                colour_gradient(L, phi, nx, ny, nz, x, y, z, G, &D, nrm);

                /* Perturbation operator, written per population. */
                double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                for (int i = 0; i < q; ++i) {
                    double cG = L->c[i][0] * G[0] + L->c[i][1] * G[1] + L->c[i][2] * G[2];
                    double B = i == 0 ? L->w[0] - 2.0 / 3.0 : L->w[i];
                    Df[i] = A / 2.0 * (L->w[i] * cG * cG - B * G2) / D;
                }
                if (regularize) {
                    /* Keep only the Hermite (second-order) part of Df. */
                    double DP[3][3] = {{0}};
                    for (int i = 0; i < q; ++i)
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) DP[a][b] += Df[i] * L->c[i][a] * L->c[i][b];
                    for (int i = 0; i < q; ++i) {
                        double QDP = 0.0;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) QDP += ora_Q(L, i, a, b) * DP[a][b];
                        Df[i] = L->w[i] * QDP;
                    }
                }
                double heqs[ORA_QMAX], us[3], Fn[3];
                if (forced) {
                    for (int a = 0; a < 3; ++a) Fn[a] = F[a * N + n];
                    forced_equilibrium(L, rho, j, P, Fn, heqs, us);
                }
                for (int i = 0; i < q; ++i) {
                    double fi = regularize ? heq[i] + hneq[i] : f[i];
                    double fpost = forced ? fi - omega * (fi - heqs[i]) + (1.0 - 0.5 * omega) * guo_term(L, i, us, Fn) +
                                                Df[i]
                                          : (1.0 - omega) * fi + omega * heq[i] + Df[i];
                    double rc = recolour_term(L, i, beta, rho1, rho2, nrm);
                    f1post[(long)i * N + n] = rho1 / rho * fpost + rc;
                    f2post[(long)i * N + n] = rho2 / rho * fpost - rc;
                }
            }

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                for (int i = 0; i < q; ++i) {
                    long src = ora_neighbour(nx, ny, nz, x, y, z, -L->c[i][0], -L->c[i][1], -L->c[i][2]);
                    f1out[(long)i * N + n] = f1post[(long)i * N + src];
                    f2out[(long)i * N + n] = f2post[(long)i * N + src];
                }
            }
}

/* Advances the species populations f1, f2 (q fields each, in place). */
int ora_cg_population_run(int q, int nx, int ny, int nz, double tau, double A, double beta,
                          int regularize, double Ah, int hmax, int nsteps, double *f1, double *f2)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0 || nx < 1 || ny < 1 || nz < 1 || nsteps < 0 || hmax < 0) return -1;
    long N = (long)nx * ny * nz;
    double *t1 = malloc(sizeof(double) * q * N);
    double *t2 = malloc(sizeof(double) * q * N);
    double *p1 = malloc(sizeof(double) * q * N);
    double *p2 = malloc(sizeof(double) * q * N);
    double *phi = malloc(sizeof(double) * N);
    double *F = malloc(sizeof(double) * 3 * N);
    int rc = 0;
    if (!t1 || !t2 || !p1 || !p2 || !phi || !F) {
        rc = -1;
    } else {
        for (int t = 0; t < nsteps; ++t) {
            cg_population_step(&L, nx, ny, nz, 1.0 / tau, A, beta, regularize, Ah, hmax, f1, f2, t1, t2, phi,
                               p1, p2, F);
            memcpy(f1, t1, sizeof(double) * q * N);
            memcpy(f2, t2, sizeof(double) * q * N);
        }
    }
    free(t1);
    free(t2);
    free(p1);
    free(p2);
    free(phi);
    free(F);
    return rc;
}
