// The two-component step as the paper's split schedule (Sec. III.A), for
// comparison with the fused step: separate passes for the phase field, the
// collision and the streaming, each over the whole box.
//
//   1. phase pass      phi = (rho1 - rho2)/rho of every node (N reals);
//   2. collision pass  per node: the colour gradient G from phi of its
//                      neighbours, the BGK collision with the perturbation
//                      (and Guo's forcing of the near-contact force), written
//                      back in place (S', and j + F under a force), and the
//                      interface normal n = G/D (3 N reals);
//   3. streaming pass  k_cg_tile on the post-collision moments: rebuild the
//                      populations, recolour with the stored n, pull, sum.
//
// Every node computes what the fused step computes, in the same order and
// precision (shared arithmetic in cg_math.hpp), so the results are equal bit
// for bit; the passes move 49 stored values per node (52 with the force)
// against 22 for the fused step.
#include <hip/hip_runtime.h>

#include "cg_math.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

constexpr int kSX = 64, kSY = 4;

// Phase field of the stored two-species state (fields dr, rho1), public layout.
template <class R>
__global__ __launch_bounds__(kSX *kSY) void k_cg_phase(const R *__restrict__ state, MomentLayout lay, int nx, int ny,
                                                        R *__restrict__ phi)
{
    const int x = blockIdx.x * kSX + threadIdx.x, y = blockIdx.y * kSY + threadIdx.y, z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t so = lay.node(x, y, z);
    phi[(int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z)] = phase_field<R>(state[so], state[kBlock + so]);
}

// Collision pass, in place on the stored state; writes the normal.
template <int Q, class R, bool FORCE>
__global__ __launch_bounds__(kSX *kSY) void k_cg_collide(R *__restrict__ state, MomentLayout lay, int nx, int ny,
                                                         int nz, const R *__restrict__ phi, const R *__restrict__ F,
                                                         R *__restrict__ nrm, R omega, R A9)
{
    const int x = blockIdx.x * kSX + threadIdx.x, y = blockIdx.y * kSY + threadIdx.y, z = blockIdx.z;
    if (x >= nx || y >= ny) return;
    const int64_t sy = nx, sz = (int64_t)nx * ny, N = sz * nz;
    const int64_t n = x + sy * y + sz * z;
    const int64_t so = lay.node(x, y, z);
    R v[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) v[k] = state[k * kBlock + so];
    // Offsets of the neighbouring columns, rows and planes (periodic).
    const int64_t ox[3] = {(x == 0 ? nx - 1 : x - 1) - (int64_t)x, 0, (x == nx - 1 ? 0 : x + 1) - (int64_t)x};
    const int64_t oy[3] = {((y == 0 ? ny - 1 : y - 1) - (int64_t)y) * sy, 0, ((y == ny - 1 ? 0 : y + 1) - (int64_t)y) * sy};
    const int64_t oz[3] = {((z == 0 ? nz - 1 : z - 1) - (int64_t)z) * sz, 0, ((z == nz - 1 ? 0 : z + 1) - (int64_t)z) * sz};
    R G[3];
    colour_gradient<Q, R>([&](int cx, int cy, int cz) { return phi[n + ox[cx + 1] + oy[cy + 1] + oz[cz + 1]]; }, G);
    R fx = R(0), fy = R(0), fz = R(0);
    if (FORCE) {
        fx = F[n];
        fy = F[N + n];
        fz = F[2 * N + n];
    }
    const CgCollided<R> o = cg_collide<R, FORCE>(v, G, omega, A9, fx, fy, fz);
    if (FORCE) {
        state[2 * kBlock + so] = o.c.jx;
        state[3 * kBlock + so] = o.c.jy;
        state[4 * kBlock + so] = o.c.jz;
    }
    state[5 * kBlock + so] = o.c.sxx;
    state[6 * kBlock + so] = o.c.syy;
    state[7 * kBlock + so] = o.c.szz;
    state[8 * kBlock + so] = o.c.sxy;
    state[9 * kBlock + so] = o.c.sxz;
    state[10 * kBlock + so] = o.c.syz;
    nrm[n] = o.nx;
    nrm[N + n] = o.ny;
    nrm[2 * N + n] = o.nz;
}

template <class R>
hipError_t run(const lbm_ctx *c, void *in, void *out)
{
    const dim3 grid((c->nx + kSX - 1) / kSX, (c->ny + kSY - 1) / kSY, c->nz), block(kSX, kSY);
    if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidConfiguration;
    R *st = static_cast<R *>(in);
    R *phi = static_cast<R *>(c->scratch_split), *nrm = phi + c->N;
    hipLaunchKernelGGL((k_cg_phase<R>), grid, block, 0, c->stream, st, c->lay, c->nx, c->ny, phi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const R om = (R)c->omega, A9 = (R)(c->A / 9.0);
    if (c->nc_A != 0.0) {
        if ((e = launch_nc_force(c, nullptr, phi)) != hipSuccess) return e;
        const R *F = static_cast<const R *>(c->scratch_nc);
        if (c->q == 19)
            hipLaunchKernelGGL((k_cg_collide<19, R, true>), grid, block, 0, c->stream, st, c->lay, c->nx, c->ny, c->nz,
                               phi, F, nrm, om, A9);
        else
            hipLaunchKernelGGL((k_cg_collide<27, R, true>), grid, block, 0, c->stream, st, c->lay, c->nx, c->ny, c->nz,
                               phi, F, nrm, om, A9);
    } else if (c->q == 19) {
        hipLaunchKernelGGL((k_cg_collide<19, R, false>), grid, block, 0, c->stream, st, c->lay, c->nx, c->ny, c->nz,
                           phi, nullptr, nrm, om, A9);
    } else {
        hipLaunchKernelGGL((k_cg_collide<27, R, false>), grid, block, 0, c->stream, st, c->lay, c->nx, c->ny, c->nz,
                           phi, nullptr, nrm, om, A9);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_cg_step(c, in, out, false, nrm);
}

} // namespace

hipError_t launch_cg_split_step(const lbm_ctx *c, void *in, void *out)
{
    if (c->species != 2 || !c->scratch_split) return hipErrorInvalidValue;
    if (c->storage == LBM_STORE_F64) return run<double>(c, in, out);
    if (c->storage == LBM_STORE_F32) return run<float>(c, in, out);
    return hipErrorInvalidValue;
}

} // namespace lbm
