/*
 * Oracle lattice tables (test infrastructure only; see oracle.h).
 *
 * The paper uses the D3Q19 velocity set with c_s = 1/sqrt(3) (Sec. III.A and
 * the sound speed stated after Eq. 11) but prints no weights; the values
 * below are the textbook ones.  D3Q27 is the tensor-product lattice with the
 * same sound speed.  Ordering: rest, 6 faces, 12 edges, 8 corners (D3Q19 is
 * the first 19 entries).  Moments do not depend on the ordering.
 */
#include "oracle.h"

static const int VEL[27][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1},
};

int ora_lattice_init(int q, ora_lat *L)
{
    double w_rest, w_face, w_edge, w_corner;
    if (q == 19) {
        w_rest = 1.0 / 3.0; w_face = 1.0 / 18.0; w_edge = 1.0 / 36.0; w_corner = 0.0;
    } else if (q == 27) {
        w_rest = 8.0 / 27.0; w_face = 2.0 / 27.0; w_edge = 1.0 / 54.0; w_corner = 1.0 / 216.0;
    } else {
        return -1;
    }
    L->q = q;
    for (int i = 0; i < q; ++i) {
        int nonzero = 0;
        for (int a = 0; a < 3; ++a) {
            L->c[i][a] = VEL[i][a];
            nonzero += VEL[i][a] != 0;
        }
        L->w[i] = nonzero == 0 ? w_rest : nonzero == 1 ? w_face : nonzero == 2 ? w_edge : w_corner;
    }
    return 0;
}

long ora_neighbour(int nx, int ny, int nz, int x, int y, int z, int dx, int dy, int dz)
{
    int xx = ((x + dx) % nx + nx) % nx;
    int yy = ((y + dy) % ny + ny) % ny;
    int zz = ((z + dz) % nz + nz) % nz;
    return (long)xx + (long)nx * ((long)yy + (long)ny * zz);
}

double ora_Q(const ora_lat *L, int i, int a, int b)
{
    double delta = a == b ? 1.0 : 0.0;
    return ((double)L->c[i][a] * L->c[i][b] - ORA_CS2 * delta) / (2.0 * ORA_CS2 * ORA_CS2);
}

void ora_unpack_tensor(const double *p6, double P[3][3])
{
    /* stored order: xx, yy, zz, xy, xz, yz */
    P[0][0] = p6[0]; P[1][1] = p6[1]; P[2][2] = p6[2];
    P[0][1] = P[1][0] = p6[3];
    P[0][2] = P[2][0] = p6[4];
    P[1][2] = P[2][1] = p6[5];
}

/* Exported copy of the tables for the lattice-identity tests. */
int ora_lattice(int q, int *c, double *w)
{
    ora_lat L;
    if (ora_lattice_init(q, &L) != 0) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
    }
    return q;
}
