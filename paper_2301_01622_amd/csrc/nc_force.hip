// Near-contact force of the LBNCI extension (Sec. III.B) for the
// two-component schemes.
//
// The paper gives F_rep = -A_h[h(x)] n delta_I, with h(x) the distance
// between two close interfaces and delta_I proportional to grad phi, and
// leaves the rest to its references.  This library's reading:
//   * G = (1/c_s^2) sum_i w_i c_i phi(x + c_i), the colour gradient;
//     delta_I = |G|/2 and n = -G/|G| (outward from species 1), so the force
//     is F = (A_h/2) G: it pushes each interface back into its own drop;
//   * h(x): the nodes x + k c*, k = 1..h_max, are probed along the lattice
//     direction c* closest to n (largest c.n/|c|; exact ties go to the
//     shorter |c|, then the larger c_x, c_y, c_z); a film is crossed when a
//     probe with phi < 0 (or phi(x) < 0) is followed by one with phi > 0;
//   * A_h[h] = A_h when a film is crossed within h_max probes, else 0.
// The force of time t is computed from the phase field of the streamed
// state, one thread per node, into three arrays of N values (x fastest);
// the collision kernels add it with Guo's forcing.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "lattice.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

// Launch shape of the per-node kernels: 64 x 4 threads over x and y, one z
// plane per block row (no index division).
constexpr int kNX = 64, kNY = 4;

// Phase field phi = (rho1 - rho2)/rho = 2 rho1/rho - 1 of the moment state
// (stored fields dr = rho - 1 and rho1), public layout.
template <class R>
__global__ __launch_bounds__(kNX *kNY) void k_phi_of_moments(const R *__restrict__ state, MomentLayout lay, int nx,
                                                             int ny, R *__restrict__ phi)
{
    const int x = blockIdx.x * kNX + threadIdx.x, y = blockIdx.y * kNY + threadIdx.y, z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t so = lay.node(x, y, z);
    const R dr = state[so], r1 = state[kBlock + so];
    phi[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)] = fma_(R(2) * r1, reciprocal<R>(R(1) + dr), R(-1));
}

// One step of a probe walk: p in [0, n), |d| <= 1.
__device__ inline int step_wrap(int p, int d, int n)
{
    p += d;
    return p < 0 ? p + n : (p >= n ? p - n : p);
}

// Lattice direction c* closest to n = -G/|G|: largest score (c.n)/|c|,
// exact ties to the smaller |c|^2, then to the lexicographically larger
// (c_x, c_y, c_z).  Returned as the key 13 + 9 c_x + 3 c_y + c_z, which orders
// directions as (c_x, c_y, c_z) does.  Only the 7 (D3Q19: 6) candidates
// whose non-zero components all carry the signs of n are scored: in any
// other candidate, setting the offending component to zero leaves a rounded
// sum at least as large with a shorter c, which scores strictly higher
// whenever the sum is positive; the winner's score is positive (|G_i| > 0
// on some axis), so no other candidate reaches or ties it.  The sums are
// formed in the order x, y, z, as the full search over all directions does.
template <class R>
__device__ inline void take_better(R score, int key, R &best, int &bkey)
{
    if (score > best || (score == best && key > bkey)) {
        best = score;
        bkey = key;
    }
}

template <int Q, class R>
__device__ inline int closest_direction(R Gx, R Gy, R Gz)
{
    const R ax = Gx < R(0) ? -Gx : Gx, ay = Gy < R(0) ? -Gy : Gy, az = Gz < R(0) ? -Gz : Gz;
    const int kx = Gx > R(0) ? -9 : 9, ky = Gy > R(0) ? -3 : 3, kz = Gz > R(0) ? -1 : 1;
    R b1 = ax;
    int k1 = 13 + kx;
    take_better(ay, 13 + ky, b1, k1);
    take_better(az, 13 + kz, b1, k1);
    const R i2 = R(0.70710678118654752440);
    R b2 = (ax + ay) * i2;
    int k2 = 13 + kx + ky;
    take_better((ax + az) * i2, 13 + kx + kz, b2, k2);
    take_better((ay + az) * i2, 13 + ky + kz, b2, k2);
    int key = b2 > b1 ? k2 : k1;
    if (Q == 27) {
        const R b3 = ((ax + ay) + az) * R(0.57735026918962576451);
        if (b3 > (b2 > b1 ? b2 : b1)) key = 13 + kx + ky + kz;
    }
    return key;
}

template <int Q, class R>
__global__ __launch_bounds__(kNX *kNY) void k_nc_force(const R *__restrict__ phi, R *__restrict__ F, int nx, int ny,
                                                       int nz, int64_t N, R half_Ah, int hmax)
{
    using L = Lattice<Q>;
    const int x = blockIdx.x * kNX + threadIdx.x, y = blockIdx.y * kNY + threadIdx.y, z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t n = x + sy * y + sz * z;
    // Offsets of the neighbouring rows, columns and planes (periodic).
    const int64_t ox[3] = {(x == 0 ? nx - 1 : x - 1) - (int64_t)x, 0, (x == nx - 1 ? 0 : x + 1) - (int64_t)x};
    const int64_t oy[3] = {((y == 0 ? ny - 1 : y - 1) - (int64_t)y) * sy, 0, ((y == ny - 1 ? 0 : y + 1) - (int64_t)y) * sy};
    const int64_t oz[3] = {((z == 0 ? nz - 1 : z - 1) - (int64_t)z) * sz, 0, ((z == nz - 1 ? 0 : z + 1) - (int64_t)z) * sz};
    R Gx = R(0), Gy = R(0), Gz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
        if (cx == 0 && cy == 0 && cz == 0) continue;
        const R wp = R(3.0 * L::w(i)) * phi[n + ox[cx + 1] + oy[cy + 1] + oz[cz + 1]];
        if (cx) Gx = cx > 0 ? Gx + wp : Gx - wp;
        if (cy) Gy = cy > 0 ? Gy + wp : Gy - wp;
        if (cz) Gz = cz > 0 ? Gz + wp : Gz - wp;
    }
    int found = 0;
    if (Gx != R(0) || Gy != R(0) || Gz != R(0)) {
        const int key = closest_direction<Q>(Gx, Gy, Gz);
        const int dx = key / 9 - 1, dy = key / 3 % 3 - 1, dz = key % 3 - 1;
        // Probes x + k c*, k = 1..h_max, each coordinate stepped with its own
        // wrap, stopping at the first film; four loads are issued at a time.
        bool seen = phi[n] < R(0);
        int px = x, py = y, pz = z;
        for (int k0 = 1; k0 <= hmax && !found; k0 += 4) {
            R f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                px = step_wrap(px, dx, nx);
                py = step_wrap(py, dy, ny);
                pz = step_wrap(pz, dz, nz);
                f[k] = phi[px + sy * py + sz * pz];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k0 + k <= hmax && !found) {
                    if (f[k] < R(0)) seen = true;
                    else if (f[k] > R(0) && seen) found = 1;
                }
        }
    }
    F[n] = found ? half_Ah * Gx : R(0);
    F[N + n] = found ? half_Ah * Gy : R(0);
    F[2 * N + n] = found ? half_Ah * Gz : R(0);
}

template <class R>
hipError_t run(const lbm_ctx *c, const void *moments, const R *phi_in, R *phi_buf, R *F)
{
    const dim3 grid((c->nx + kNX - 1) / kNX, (c->ny + kNY - 1) / kNY, c->nz), block(kNX, kNY);
    if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidConfiguration;
    const R *phi = phi_in;
    if (!phi) {
        hipLaunchKernelGGL((k_phi_of_moments<R>), grid, block, 0, c->stream, static_cast<const R *>(moments), c->lay,
                           c->nx, c->ny, phi_buf);
        phi = phi_buf;
    }
    if (c->q == 19)
        hipLaunchKernelGGL((k_nc_force<19, R>), grid, block, 0, c->stream, phi, F, c->nx, c->ny, c->nz, c->N,
                           (R)(0.5 * c->nc_A), c->nc_hmax);
    else
        hipLaunchKernelGGL((k_nc_force<27, R>), grid, block, 0, c->stream, phi, F, c->nx, c->ny, c->nz, c->N,
                           (R)(0.5 * c->nc_A), c->nc_hmax);
    return hipGetLastError();
}

} // namespace

hipError_t launch_nc_force(const lbm_ctx *c, const void *moments, const void *phi)
{
    if (c->species != 2 || !c->scratch_nc) return hipErrorInvalidValue;
    if (c->storage == LBM_STORE_F64) {
        double *buf = static_cast<double *>(c->scratch_nc);
        return run<double>(c, moments, static_cast<const double *>(phi), buf + 3 * c->N, buf);
    }
    float *buf = static_cast<float *>(c->scratch_nc);
    return run<float>(c, moments, static_cast<const float *>(phi), buf + 3 * c->N, buf);
}

} // namespace lbm
