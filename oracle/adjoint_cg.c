/*
 * Oracle: discrete adjoint of one time step of the two-component
 * colour-gradient scheme without populations (test infrastructure only; see
 * oracle.h and color_gradient.c for the forward step and its readings).
 *
 * Forward, at every source node y (rho = rho1 + rho2, s_k = rho^k/rho):
 *   G(y)    = (1/c_s^2) sum_k w_k c_k phi(y + c_k),   phi = (rho1 - rho2)/rho
 *   h'_i(y) = BGK part of Eq. 8 at (rho, j, P) + w_i Q_i : DP(G),
 *             DP(G) = (A/9)(G G - |G|^2 I)/D,  D = sqrt(|G|^2 + eps^2)
 *   rc_i(y) = C w_i (c_i.n)/|c_i|,  C = beta rho1 rho2/rho,  n = G/D
 *   f1_i = s_1 h'_i + rc_i,  f2_i = s_2 h'_i - rc_i
 * and the node x = y + c_i receives f1_i in rho1, f2_i in rho2 and h'_i in
 * j and P.  For co-states lam(x, t+1) = (l1, l2, lj, lP) the transposed step
 * gathers, per direction,
 *   g1_i = l1(y + c_i),  g2_i = l2(y + c_i),  gm_i = c_i.lj + c_i c_i : lP at y + c_i,
 * sets  A_i = g1_i s_1 + g2_i s_2 + gm_i   (co-state of h'_i),
 *       B_i = g1_i - g2_i                  (co-state of rc_i),
 * and applies the chain rule through s_k, C, n, DP and the BGK part.  The
 * gradient G(y) couples to phi on the radius-1 stencil, so the co-state of
 * phi(z) = sum_k (1/c_s^2) w_k c_k . gG(z - c_k) is added through
 * d phi/d rho1 = 2 rho2/rho^2 and d phi/d rho2 = -2 rho1/rho^2.
 *
 * The tau-sensitivity is taken at fixed sigma (A = 9 sigma/(2 tau)):
 *   dL/dtau = -omega^2 sum_y Gamma_A : (j j/rho - S) - (1/tau) sum_y Gamma_A : DP,
 * Gamma_A = sum_i A_i w_i Q_i.  Every operator is smooth in G.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

#define EPS_G 1e-3

static const int PA[6] = {0, 1, 2, 0, 0, 1};
static const int PB[6] = {0, 1, 2, 1, 2, 2};

static double speed(const ora_lat *L, int i)
{
    return sqrt((double)(L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]));
}

/* Two-component SoA layout: rho1, rho2, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz. */
static void node2(const double *M, long N, long n, double *r1, double *r2, double j[3], double P[3][3])
{
    double p6[6];
    *r1 = M[n];
    *r2 = M[N + n];
    for (int a = 0; a < 3; ++a) j[a] = M[(2 + a) * N + n];
    for (int k = 0; k < 6; ++k) p6[k] = M[(5 + k) * N + n];
    ora_unpack_tensor(p6, P);
}

static void gradient(const ora_lat *L, const double *phi, int nx, int ny, int nz, int x, int y, int z, double G[3])
{
    for (int a = 0; a < 3; ++a) G[a] = 0.0;
    for (int k = 0; k < L->q; ++k) {
        long nb = ora_neighbour(nx, ny, nz, x, y, z, L->c[k][0], L->c[k][1], L->c[k][2]);
        for (int a = 0; a < 3; ++a) G[a] += L->w[k] * L->c[k][a] * phi[nb] / ORA_CS2;
    }
}

/* lam_out = J^T lam_next for the two-component step at state M (11 fields);
 * *dL_dtau (if not NULL) receives this step's dL/dtau at fixed sigma. */
int ora_cg_adjoint_step(int q, int nx, int ny, int nz, double tau, double A, double beta, const double *M,
                        const double *lam_next, double *lam_out, double *dL_dtau)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
    long N = (long)nx * ny * nz;
    double omega = 1.0 / tau;
    double *phi = malloc(sizeof(double) * N);
    double *gG = malloc(sizeof(double) * 3 * N);
    if (!phi || !gG) {
        free(phi);
        free(gG);
        return -1;
    }
    for (long n = 0; n < N; ++n) phi[n] = (M[n] - M[N + n]) / (M[n] + M[N + n]);

    double sum_omega = 0.0, sum_A = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : sum_omega, sum_A)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double r1, r2, j[3], P[3][3], G[3];
                node2(M, N, n, &r1, &r2, j, P);
                double rho = r1 + r2, s1 = r1 / rho, s2 = r2 / rho;
                gradient(&L, phi, nx, ny, nz, x, y, z, G);
                double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                double D = sqrt(G2 + EPS_G * EPS_G);
                double nv[3] = {G[0] / D, G[1] / D, G[2] / D};
                double C = beta * r1 * r2 / rho;
                double DP[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) DP[a][b] = A / 9.0 * (G[a] * G[b] - (a == b ? G2 : 0.0)) / D;

                double heq[ORA_QMAX], hneq[ORA_QMAX];
                ora_hermite_parts(&L, rho, j, P, heq, hneq);
                double Gam[3][3] = {{0}}, alpha = 0.0, bet[3] = {0, 0, 0}, V[3] = {0, 0, 0}, S1 = 0.0, S2 = 0.0;
                for (int i = 0; i < L.q; ++i) {
                    long dst = ora_neighbour(nx, ny, nz, x, y, z, L.c[i][0], L.c[i][1], L.c[i][2]);
                    double g1 = lam_next[dst], g2 = lam_next[N + dst], gm = 0.0;
                    for (int a = 0; a < 3; ++a) gm += L.c[i][a] * lam_next[(2 + a) * N + dst];
                    for (int k = 0; k < 6; ++k) gm += L.c[i][PA[k]] * L.c[i][PB[k]] * lam_next[(5 + k) * N + dst];
                    /* post-collision mixture population h'_i */
                    double QDP = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) QDP += ora_Q(&L, i, a, b) * DP[a][b];
                    double hp = (1.0 - omega) * (heq[i] + hneq[i]) + omega * heq[i] + L.w[i] * QDP;
                    double Ai = g1 * s1 + g2 * s2 + gm;
                    double Bi = g1 - g2;
                    S1 += g1 * hp;
                    S2 += g2 * hp;
                    alpha += Ai * L.w[i];
                    for (int a = 0; a < 3; ++a) bet[a] += Ai * L.w[i] * L.c[i][a];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Gam[a][b] += Ai * L.w[i] * ora_Q(&L, i, a, b);
                    if (i != 0 && speed(&L, i) > 0.0)
                        for (int a = 0; a < 3; ++a) V[a] += Bi * L.w[i] * L.c[i][a] / speed(&L, i);
                }

                /* BGK part (as in the one-component adjoint), with rho = rho1 + rho2. */
                double jGj = 0.0, Gj[3] = {0, 0, 0}, trG = Gam[0][0] + Gam[1][1] + Gam[2][2];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        Gj[a] += Gam[a][b] * j[b];
                        jGj += j[a] * Gam[a][b] * j[b];
                    }
                double l_rho = alpha - omega * jGj / (rho * rho) - (1.0 - omega) * ORA_CS2 * trG;
                double out[11];
                for (int a = 0; a < 3; ++a) out[2 + a] = 3.0 * bet[a] + 2.0 * omega * Gj[a] / rho;
                for (int k = 0; k < 6; ++k)
                    out[5 + k] = (1.0 - omega) * (k < 3 ? Gam[PA[k]][PB[k]] : 2.0 * Gam[PA[k]][PB[k]]);

                /* Through s_k = rho^k/rho and C = beta rho1 rho2/rho. */
                double Vn = V[0] * nv[0] + V[1] * nv[1] + V[2] * nv[2];
                double rho2 = rho * rho;
                out[0] = l_rho + S1 * (r2 / rho2) + S2 * (-r2 / rho2) + Vn * beta * r2 * r2 / rho2;
                out[1] = l_rho + S1 * (-r1 / rho2) + S2 * (r1 / rho2) + Vn * beta * r1 * r1 / rho2;
                for (int k = 0; k < 11; ++k) lam_out[k * N + n] = out[k];

                /* Co-state of G: perturbation (A/9)(GG - G^2 I)/D and normal G/D. */
                double g[3] = {0, 0, 0};
                {
                    double GGG = 0.0, GamG[3] = {0, 0, 0};
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            GamG[a] += Gam[a][b] * G[b];
                            GGG += G[a] * Gam[a][b] * G[b];
                        }
                    double num = GGG - G2 * trG; /* D * Gamma:DP * 9/A */
                    for (int a = 0; a < 3; ++a)
                        g[a] += A / 9.0 * ((2.0 * GamG[a] - 2.0 * trG * G[a]) / D - num * G[a] / (D * D * D));
                    double GV = G[0] * V[0] + G[1] * V[1] + G[2] * V[2];
                    for (int a = 0; a < 3; ++a) g[a] += C * (V[a] / D - G[a] * GV / (D * D * D));
                }
                for (int a = 0; a < 3; ++a) gG[a * N + n] = g[a];

                /* tau-sensitivity: omega part and A part (A proportional to 1/tau). */
                double S[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) S[a][b] = P[a][b] - (a == b ? rho * ORA_CS2 : 0.0);
                double eo = 0.0, ea = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        eo += Gam[a][b] * (j[a] * j[b] / rho - S[a][b]);
                        ea += Gam[a][b] * DP[a][b];
                    }
                sum_omega += eo;
                sum_A += ea;
            }

    /* phi(z) enters G(z - c_k) with weight (1/c_s^2) w_k c_k. */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double gphi = 0.0;
                for (int k = 0; k < L.q; ++k) {
                    long src = ora_neighbour(nx, ny, nz, x, y, z, -L.c[k][0], -L.c[k][1], -L.c[k][2]);
                    for (int a = 0; a < 3; ++a) gphi += L.w[k] * L.c[k][a] / ORA_CS2 * gG[a * N + src];
                }
                double r1 = M[n], r2 = M[N + n], rho = r1 + r2;
                lam_out[n] += gphi * 2.0 * r2 / (rho * rho);
                lam_out[N + n] += gphi * (-2.0 * r1 / (rho * rho));
            }

    if (dL_dtau) *dL_dtau = -omega * omega * sum_omega - sum_A / tau;
    free(phi);
    free(gG);
    return 0;
}
