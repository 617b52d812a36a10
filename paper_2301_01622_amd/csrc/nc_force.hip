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
//
// A film is crossed only between a node with phi < 0 and one with phi > 0,
// both within h_max nodes of x along every axis.  The pass therefore first
// records, per block of 64 x 4 nodes of a plane and per 16-node group of its
// rows, whether any phi is positive and whether any is negative
// (k_phi_signs); a block whose neighbourhood of radius h_max holds no
// positive phi or no negative phi has F = 0 at every node, exactly as the
// per-node search would find, and skips the search.  Its force arrays are
// rewritten (with zeros) only if a previous pass left non-zero values there
// (a per-block flag), so the bulk of a droplet run costs a few byte loads
// per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "lattice.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

// Launch shape of the per-node kernels: 64 x 4 threads over x and y, one z
// plane per block row (no index division).
constexpr int kNX = kNcBlockX, kNY = kNcBlockY;

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

// Planes per block of the sign and force passes.  The force pass may split a
// block's planes over NZ layers of threads (plane k on layer k mod NZ), so
// that a thread walks kZB / NZ planes, each a chain of dependent loads: two
// layers where the grid has fewer than 16 blocks per CU (the paper's 128^3
// collision: 6.6 % faster per step; on 512 x 256 x 256, with 64 blocks per
// CU, two layers made the step 2 % slower).
constexpr int kZB = 8;
// Largest probe range (lbm_create refuses more).
constexpr int kHmaxMax = 32;

// Sign summary of the phase field: for the block (bx, by) of 64 x 4 nodes
// of plane z, bit k (k = 0..3) is set if a node of x-group k (16 nodes) has
// phi > 0, bit 4 + k if one has phi < 0.  A wave covers one block column of
// 64 x-nodes, each lane one x over the block's 4 rows (the signs of the rows
// are OR-ed in the lane, then one ballot per plane); the waves of a
// workgroup (blockDim.x / 64, at most 4) cover consecutive block columns, so
// that each row is read in pieces of up to 1 KiB, and ZB planes.
constexpr int kSignWavesMax = 4;
template <class R, int ZB>
__global__ __launch_bounds__(64 * kSignWavesMax) void k_phi_signs(const R *__restrict__ phi, int nx, int ny, int nz,
                                                                 uint8_t *__restrict__ sig)
{
    const int lane = threadIdx.x % 64;
    const int bx = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64, by = blockIdx.y;
    const int gx = (nx + kNX - 1) / kNX, gy = (ny + kNY - 1) / kNY;
    const int x = bx * kNX + lane, y0 = by * kNY;
    const int z0 = blockIdx.z * ZB, zn = min(ZB, nz - z0);
    const bool in = x < nx;
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
        bool pos = false, neg = false;
#pragma unroll
        for (int r = 0; r < kNY; ++r) {
            const R f = in && y0 + r < ny && k < zn
                            ? phi[(int64_t)x + (int64_t)nx * ((int64_t)(y0 + r) + (int64_t)ny * (z0 + k))]
                            : R(0);
            pos = pos || f > R(0);
            neg = neg || f < R(0);
        }
        const unsigned long long bp = __ballot(pos), bn = __ballot(neg);
        if (lane == 0 && bx < gx && k < zn) {
            unsigned int b = 0u;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if ((bp >> (16 * g)) & 0xffffull) b |= 1u << g;
                if ((bn >> (16 * g)) & 0xffffull) b |= 1u << (4 + g);
            }
            sig[bx + (int64_t)gx * (by + (int64_t)gy * (z0 + k))] = (uint8_t)b;
        }
    }
}

// Group indices (groups of width g over [0, n)) met by the coordinates
// lo, lo+1, ..., lo+len-1 taken modulo n: at most two runs.
struct GroupRuns {
    int a0, n0, a1, n1;
    __device__ int at(int i) const { return i < n0 ? a0 + i : a1 + (i - n0); }
    __device__ int count() const { return n0 + n1; }
};

__device__ inline GroupRuns group_runs(int lo, int len, int n, int g)
{
    GroupRuns r{0, 0, 0, 0};
    if (len >= n) {
        r.n0 = (n + g - 1) / g;
        return r;
    }
    int a = lo % n;
    if (a < 0) a += n;
    const int b = a + len - 1;
    r.a0 = a / g;
    if (b < n) {
        r.n0 = b / g - r.a0 + 1;
    } else {
        r.n0 = (n - 1) / g - r.a0 + 1;
        r.n1 = (b - n) / g + 1;
    }
    return r;
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

template <int Q, class R, int NZ>
__global__ __launch_bounds__(kNX *kNY *NZ) void k_nc_force(const R *__restrict__ phi, R *__restrict__ F, int nx, int ny,
                                                       int nz, int64_t N, R half_Ah, int hmax,
                                                       const uint8_t *__restrict__ sig, uint8_t *__restrict__ dirty)
{
    using L = Lattice<Q>;
    const int x = blockIdx.x * kNX + threadIdx.x, y = blockIdx.y * kNY + threadIdx.y;
    const int tid = threadIdx.x + kNX * threadIdx.y + kNX * kNY * threadIdx.z;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;  // first thread of its layer
    const int z0 = blockIdx.z * kZB, zn = min(kZB, nz - z0);
    const int gx = (nx + kNX - 1) / kNX, gy = (ny + kNY - 1) / kNY;
    auto blk_of = [&](int z) { return blockIdx.x + (int64_t)gx * (blockIdx.y + (int64_t)gy * z); };
    // Signs of the window of planes z0 - hmax .. z0 + zn - 1 + hmax (wrapped)
    // over the x-groups and block rows within hmax of this block, and the
    // dirty flags of the block's planes, read before any is rewritten.
    const int W = zn + 2 * hmax;
    __shared__ unsigned int s_bits[kZB + 2 * kHmaxMax];
    __shared__ uint8_t s_dirty[kZB];
    if (tid < W) s_bits[tid] = 0u;
    if (tid < zn) s_dirty[tid] = dirty[blk_of(z0 + tid)];
    __syncthreads();
    {
        const GroupRuns gxr = group_runs(blockIdx.x * kNX - hmax, kNX + 2 * hmax, nx, 16);
        const GroupRuns gyr = group_runs(blockIdx.y * kNY - hmax, kNY + 2 * hmax, ny, kNY);
        const int cx = gxr.count(), pairs = cx * gyr.count(), total = pairs * W;
        for (int t = tid; t < total; t += kNX * kNY * NZ) {
            const int w = t / pairs, r = t - w * pairs;
            const int G = gxr.at(r % cx), by = gyr.at(r / cx);
            int zw = (z0 - hmax + w) % nz;
            if (zw < 0) zw += nz;
            const unsigned v = sig[G / 4 + (int64_t)gx * (by + (int64_t)gy * zw)];
            const unsigned b = ((v >> (G % 4)) & 1u) | (((v >> (4 + G % 4)) & 1u) << 1);
            if (b) atomicOr(&s_bits[w], b);
        }
    }
    __syncthreads();
    const bool in = x < nx && y < ny;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    for (int k = threadIdx.z; k < zn; k += NZ) {
        const int z = z0 + k;
        // Is there a phi > 0 and a phi < 0 within hmax of the block's plane z?
        unsigned int b = 0u;
        for (int w = k; w <= k + 2 * hmax; ++w) b |= s_bits[w];
        if (b != 3u) {
            // No film can be crossed from any node of this plane: F = 0.
            if (s_dirty[k]) {
                if (in) {
                    const int64_t n = x + sy * y + sz * z;
                    F[n] = R(0);
                    F[N + n] = R(0);
                    F[2 * N + n] = R(0);
                }
                if (lead) dirty[blk_of(z)] = 0;
            }
            continue;
        }
        if (lead && !s_dirty[k]) dirty[blk_of(z)] = 1;
        if (!in) continue;
        const int64_t n = x + sy * y + sz * z;
        // Offsets of the neighbouring rows, columns and planes (periodic).
        const int64_t ox[3] = {(x == 0 ? nx - 1 : x - 1) - (int64_t)x, 0, (x == nx - 1 ? 0 : x + 1) - (int64_t)x};
        const int64_t oy[3] = {((y == 0 ? ny - 1 : y - 1) - (int64_t)y) * sy, 0,
                               ((y == ny - 1 ? 0 : y + 1) - (int64_t)y) * sy};
        const int64_t oz[3] = {((z == 0 ? nz - 1 : z - 1) - (int64_t)z) * sz, 0,
                               ((z == nz - 1 ? 0 : z + 1) - (int64_t)z) * sz};
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
            // Probes x + k c*, k = 1..h_max, each coordinate stepped with its
            // own wrap, stopping at the first film; four loads at a time.
            bool seen = phi[n] < R(0);
            int px = x, py = y, pz = z;
            for (int k0 = 1; k0 <= hmax && !found; k0 += 4) {
                R f[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    px = step_wrap(px, dx, nx);
                    py = step_wrap(py, dy, ny);
                    pz = step_wrap(pz, dz, nz);
                    f[kk] = phi[px + sy * py + sz * pz];
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    if (k0 + kk <= hmax && !found) {
                        if (f[kk] < R(0)) seen = true;
                        else if (f[kk] > R(0) && seen) found = 1;
                    }
            }
        }
        F[n] = found ? half_Ah * Gx : R(0);
        F[N + n] = found ? half_Ah * Gy : R(0);
        F[2 * N + n] = found ? half_Ah * Gz : R(0);
    }
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
    uint8_t *sig = nc_block_flags(c), *dirty = sig + nc_blocks(c);
    const dim3 zgrid(grid.x, grid.y, (c->nz + kZB - 1) / kZB);
    if (c->nc_hmax > kHmaxMax) return hipErrorInvalidValue;
    const bool few = (int64_t)zgrid.x * zgrid.y * zgrid.z < 16 * 256;
    // The sign pass: up to 4 block columns per workgroup; on small grids two
    // planes per workgroup instead of kZB, so that the grid still fills the
    // chip.
    const unsigned sw = std::min<unsigned>(kSignWavesMax, grid.x);
    const dim3 sgrid((grid.x + sw - 1) / sw, grid.y, few ? (c->nz + 1) / 2 : zgrid.z);
    if (few)
        hipLaunchKernelGGL((k_phi_signs<R, 2>), sgrid, dim3(64 * sw), 0, c->stream, phi, c->nx, c->ny, c->nz, sig);
    else
        hipLaunchKernelGGL((k_phi_signs<R, kZB>), sgrid, dim3(64 * sw), 0, c->stream, phi, c->nx, c->ny, c->nz, sig);
    const dim3 block3(kNX, kNY, few ? 2 : 1);
    auto force = [&](auto q, auto nzc) {
        hipLaunchKernelGGL((k_nc_force<decltype(q)::value, R, decltype(nzc)::value>), zgrid, block3, 0, c->stream,
                           phi, F, c->nx, c->ny, c->nz, c->N, (R)(0.5 * c->nc_A), c->nc_hmax, sig, dirty);
    };
    using Q19 = std::integral_constant<int, 19>;
    using Q27 = std::integral_constant<int, 27>;
    using Z1 = std::integral_constant<int, 1>;
    using Z2 = std::integral_constant<int, 2>;
    if (c->q == 19) few ? force(Q19(), Z2()) : force(Q19(), Z1());
    else few ? force(Q27(), Z2()) : force(Q27(), Z1());
    return hipGetLastError();
}

} // namespace

int64_t nc_blocks(const lbm_ctx *c)
{
    return (int64_t)((c->nx + kNX - 1) / kNX) * ((c->ny + kNY - 1) / kNY) * c->nz;
}

size_t nc_scratch_bytes(const lbm_ctx *c)
{
    // F (3 N reals), the moment scheme's phase field (N reals), then the
    // sign summary and the dirty flag of every block (one byte each).
    const size_t reals = (size_t)c->N * (c->scheme == LBM_SCHEME_MOMENT ? 4 : 3);
    return c->elem * reals + 2 * (size_t)nc_blocks(c);
}

uint8_t *nc_block_flags(const lbm_ctx *c)
{
    const size_t reals = (size_t)c->N * (c->scheme == LBM_SCHEME_MOMENT ? 4 : 3);
    return static_cast<uint8_t *>(c->scratch_nc) + c->elem * reals;
}

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
