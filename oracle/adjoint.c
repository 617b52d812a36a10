/*
 * Oracle: discrete adjoint of one time step of the single-component scheme
 * without populations (test infrastructure only; see oracle.h).
 *
 * The paper has no adjoint; this is the exact transpose of the Jacobian of
 * the oracle's own step (moment_lb.c), derived by hand.  With Eqs. 4-8 the
 * post-collision population rebuilt at a node with moments (rho, j, P) is
 *   h'_i = w_i [ rho + 3 c_i.j + omega Q_i:(j j/rho) + (1 - omega) Q_i:(P - rho c_s^2 I) ]
 * (Eq. 8 with P^eq = rho c_s^2 I + j j/rho), and the step stores
 *   M(x, t+1) = sum_i m_i h'_i(M(x - c_i, t)),  m_i = (1, c_i, c_i c_i)  (Eqs. 9, 1-3).
 * For a co-state lam(t+1) (one value per stored field) the transposed step is
 *   a_i(y)   = m_i . lam(y + c_i, t+1),
 *   lam(y,t) = sum_i a_i(y) d h'_i / d M(y, t),
 * with the partial derivatives written out below.  The sensitivity to the
 * relaxation frequency is sum_y sum_i a_i(y) d h'_i / d omega.
 *
 * Stored tensor components are P_xx, P_yy, P_zz, P_xy, P_xz, P_yz; an
 * off-diagonal stored value stands for both P_ab and P_ba.
 */
#include <stdlib.h>

#include "oracle.h"

static const int PA[6] = {0, 1, 2, 0, 0, 1};
static const int PB[6] = {0, 1, 2, 1, 2, 2};

/* d h'_i / d (rho, j_a, P_k) and d h'_i / d omega at one node. */
static void population_jacobian(const ora_lat *L, int i, double omega, double rho, const double j[3],
                                double P[3][3], double d[10], double *d_omega)
{
    double w = L->w[i];
    double Qjj = 0.0, QP = 0.0, QI = 0.0, Qj[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double Q = ora_Q(L, i, a, b);
            Qjj += Q * j[a] * j[b];
            QP += Q * P[a][b];
            QI += Q * (a == b ? 1.0 : 0.0);
            Qj[a] += Q * j[b];
        }
    /* rho */
    d[0] = w * (1.0 - omega * Qjj / (rho * rho) - (1.0 - omega) * ORA_CS2 * QI);
    /* j_a */
    for (int a = 0; a < 3; ++a) d[1 + a] = w * (3.0 * L->c[i][a] + omega * 2.0 * Qj[a] / rho);
    /* P_k */
    for (int k = 0; k < 6; ++k) {
        double Q = ora_Q(L, i, PA[k], PB[k]);
        d[4 + k] = w * (1.0 - omega) * (k < 3 ? Q : 2.0 * Q);
    }
    /* omega */
    *d_omega = w * (Qjj / rho - (QP - rho * ORA_CS2 * QI));
}

/* m_i . lam at one node: lam_rho + c_i . lam_j + sum_k (c_i c_i)_k lam_P_k. */
static double moment_row_dot(const ora_lat *L, int i, const double *lam, long N, long n)
{
    double s = lam[0 * N + n];
    for (int a = 0; a < 3; ++a) s += L->c[i][a] * lam[(1 + a) * N + n];
    for (int k = 0; k < 6; ++k) s += L->c[i][PA[k]] * L->c[i][PB[k]] * lam[(4 + k) * N + n];
    return s;
}

/* lam_out = (dM(t+1)/dM(t))^T lam_next for the state M = M(t) (10 fields);
 * *dL_domega (if not NULL) receives sum over nodes of a_i dh'_i/domega. */
int ora_moment_adjoint_step(int q, int nx, int ny, int nz, double tau, const double *M, const double *lam_next,
                            double *lam_out, double *dL_domega)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
    long N = (long)nx * ny * nz;
    double omega = 1.0 / tau;
    double total = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : total)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = (long)x + (long)nx * ((long)y + (long)ny * z);
                double rho, j[3], P[3][3], out[10] = {0}, dom = 0.0;
                ora_load_node(M, N, n, &rho, j, P);
                for (int i = 0; i < L.q; ++i) {
                    /* h'_i(y) streams to y + c_i. */
                    long dst = ora_neighbour(nx, ny, nz, x, y, z, L.c[i][0], L.c[i][1], L.c[i][2]);
                    double a = moment_row_dot(&L, i, lam_next, N, dst);
                    double d[10], d_om;
                    population_jacobian(&L, i, omega, rho, j, P, d, &d_om);
                    for (int k = 0; k < 10; ++k) out[k] += a * d[k];
                    dom += a * d_om;
                }
                for (int k = 0; k < 10; ++k) lam_out[k * N + n] = out[k];
                total += dom;
            }
    if (dL_domega) *dL_domega = total;
    return 0;
}
