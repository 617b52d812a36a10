/*
 * Oracle for the lattice Boltzmann scheme without populations.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision CPU
 * implementation written directly from the paper's equations.  It exists so
 * that the GPU library can be checked against something obviously correct.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * Notation follows Sec. II of the paper: populations f_i, discrete velocities
 * c_i with weights w_i, sound speed c_s^2 = 1/3, hydro-fields
 * H = [rho, rho*u_a, P_ab] (Eqs. 1-3), relaxation frequency omega = 1/tau.
 *
 * Array layout (every function): structure of arrays, one contiguous block
 * of N = nx*ny*nz doubles per field, node index n = x + nx*(y + ny*z),
 * fully periodic box.
 *   single component  H: rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz
 *   two components    H: rho1, rho2, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz
 *   populations       f: q blocks in this oracle's own velocity ordering
 * where j = rho*u is the momentum density.
 */
#ifndef LB_ORACLE_H
#define LB_ORACLE_H

#define ORA_QMAX 27
#define ORA_CS2 (1.0 / 3.0)

typedef struct {
    int q;
    int c[ORA_QMAX][3];
    double w[ORA_QMAX];
} ora_lat;

/* Returns 0 and fills *L for q = 19 or 27, -1 otherwise. */
int ora_lattice_init(int q, ora_lat *L);

/* Periodic neighbour of node (x,y,z) displaced by (dx,dy,dz). */
long ora_neighbour(int nx, int ny, int nz, int x, int y, int z, int dx, int dy, int dz);

/* Second-order Hermite tensor Q_iab = (c_ia c_ib - c_s^2 delta_ab)/(2 c_s^4). */
double ora_Q(const ora_lat *L, int i, int a, int b);

/* Unpacks the 6 stored pressure-tensor components into a symmetric 3x3. */
void ora_unpack_tensor(const double *p6, double P[3][3]);

/* Eq. 5 (h_i^eq) and Eq. 6 (h_i^neq) at one node with hydro-fields
 * rho, j = rho u and P. */
void ora_hermite_parts(const ora_lat *L, double rho, const double j[3], double P[3][3],
                       double *heq, double *hneq);

/* Eqs. 1-3: moments of one node's q populations. */
void ora_project(const ora_lat *L, const double *f, double *rho, double j[3], double P[3][3]);

/* Single-component SoA access: node n of the 10-field array H (N nodes). */
void ora_load_node(const double *H, long N, long n, double *rho, double j[3], double P[3][3]);
void ora_store_node(double *H, long N, long n, double rho, const double j[3], double P[3][3]);

#endif
