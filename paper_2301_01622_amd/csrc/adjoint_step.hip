// Discrete adjoint of the one-species moment-only step.
//
// Forward (Eqs. 4-9, 1-3): M(x, t+1) = sum_i m_i h'_i(M(x - c_i, t)), with
// m_i = (1, c_i, c_i c_i) and the reconstructed post-collision population
//   h'_i(M) = w_i [rho + 3 c_i.j + Q_i : S'],  S' = (1 - omega)(P - rho c_s^2 I) + omega j j/rho,
//   Q_i : X = 4.5 c_i c_i : X - 1.5 tr X.
// Transposed step for a co-state lam(t+1) in the public layout
// (rho, j, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz):
//   a_i(y) = m_i . lam(y + c_i)            (gathered from the downstream node)
//   alpha = sum_i w_i a_i,  beta = sum_i w_i c_i a_i,
//   Gamma = sum_i w_i a_i Q_i = 4.5 sum_i w_i a_i c_i c_i - 1.5 alpha I,
//   lam_rho = alpha - (1 - omega) tr Gamma / 3 - omega j.Gamma.j / rho^2,
//   lam_j   = 3 beta + 2 omega Gamma j / rho,
//   lam_P   = (1 - omega) Gamma   (off-diagonal stored components: twice),
// and the relaxation-frequency sensitivity sum_y Gamma : (j j/rho - S).
//
// The kernel has the structure of the forward one: a tile marches along z,
// every node of the tile plus halo publishes w_i a_i-ready values
// b_i = w_i m_i . lam(z) to LDS, and each interior node gathers b_i from
// y + c_i (the reverse of the forward pull) into three plane accumulators.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "adjoint_math.hpp"
#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

// LSTORED: co-states in the stored (blocked) layout of the state instead of
// the public one.
template <int Q, class S, int TX, int TY, bool LSTORED>
__global__ __launch_bounds__(TX *TY) void k_adjoint_tile(const S *__restrict__ state,
                                                         const typename Store<S>::real *__restrict__ lam_in,
                                                         typename Store<S>::real *__restrict__ lam_out, TileGrid g,
                                                         typename Store<S>::real omega,
                                                         typename Store<S>::real inv_s_pi,
                                                         double *__restrict__ partials)
{
    using R = typename Store<S>::real;
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int RING = HN - NT;
    static_assert(RING <= NT, "halo ring must fit one pass");
    __shared__ R lds[kLdsSlots<Q> * HN];
    __shared__ double red[NT];

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = (int64_t)g.nx * g.ny;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < g.nx) && (y0 + ly < g.ny);
    const int h0 = (ly + 1) * HX + (lx + 1);

    const bool has_ring = tid < RING;
    int hr;
    {
        const int m = tid;
        int hx, hy;
        if (m < HX) { hx = m; hy = 0; }
        else if (m < 2 * HX) { hx = m - HX; hy = HY - 1; }
        else if (m < 2 * HX + TY) { hx = 0; hy = 1 + (m - 2 * HX); }
        else { hx = HX - 1; hy = 1 + (m - 2 * HX - TY); }
        hr = hy * HX + hx;
    }
    // Co-state offsets (field stride LF, plane stride LP) in the chosen layout.
    const int64_t LF = LSTORED ? (int64_t)kBlock : g.N;
    const int64_t LP = LSTORED ? g.lay.plane : plane;
    auto xy_of = [&](int h) -> int64_t {
        const int x = wrap_coord(x0 - 1 + h % HX, g.nx), y = wrap_coord(y0 - 1 + h / HX, g.ny);
        return LSTORED ? g.lay.xy(x, y) : (int64_t)x + (int64_t)g.nx * y;
    };
    const int64_t own_xy = xy_of(h0);
    const int64_t ring_xy = has_ring ? xy_of(hr) : 0;

    MomentAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();
    double dom = 0.0;

    R la[10], lb[10], ra[10], rb[10];
    auto fetch = [&](int p, R *own, R *ring) {
        const int zs = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
#pragma unroll
        for (int k = 0; k < 10; ++k) own[k] = lam_in[k * LF + own_xy + (int64_t)zs * LP];
        if (has_ring) {
#pragma unroll
            for (int k = 0; k < 10; ++k) ring[k] = lam_in[k * LF + ring_xy + (int64_t)zs * LP];
        }
    };

    auto publish = [&](const R *l, int h, R *own4) {
        Layer<R> L0, L1, L2;
        adjoint_layer<Q, -1, R>(l, L0);
        adjoint_layer<Q, 0, R>(l, L1);
        adjoint_layer<Q, 1, R>(l, L2);
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            if (lds_slot<Q>(-1, sl) >= 0) lds[lds_slot<Q>(-1, sl) * HN + h] = L0.v[sl];
            if (lds_slot<Q>(0, sl) >= 0) lds[lds_slot<Q>(0, sl) * HN + h] = L1.v[sl];
            if (lds_slot<Q>(1, sl) >= 0) lds[lds_slot<Q>(1, sl) * HN + h] = L2.v[sl];
        }
        if (own4) {
            own4[0] = L0.v[4];
            own4[1] = L1.v[4];
            own4[2] = L2.v[4];
        }
    };

    // Gathers layer CZ from y + c (the node the forward step streamed to);
    // source plane p feeds destination plane p - CZ.
    auto gather_layer = [&](auto czc, R own) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> f;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            if (sl == 4) f.v[sl] = own;
            else if (lds_slot<Q>(CZ, sl) >= 0) f.v[sl] = lds[lds_slot<Q>(CZ, sl) * HN + h0 + cy * HX + cx];
        }
        accumulate_layer<Q, CZ, R>(acc[1 - CZ], f);
    };

    auto finish = [&](int d) {
        const int64_t so = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)d * g.lay.plane;  // stored
        const int64_t o = LSTORED ? so : (int64_t)(x0 + lx) + (int64_t)g.nx * (y0 + ly) + (int64_t)d * plane;
        S v[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) v[k] = state[k * kBlock + so];
        R lam[10];
        dom += adjoint_node<S>(acc[0], v, omega, inv_s_pi, lam);
#pragma unroll
        for (int k = 0; k < 10; ++k) lam_out[k * LF + o] = lam[k];
    };

    auto plane_step = [&](int p, R *own, R *ring) {
        R own4[3];
        publish(own, h0, own4);
        if (has_ring) publish(ring, hr, nullptr);
        __syncthreads();
        if (p + 2 <= z_end) fetch(p + 2, own, ring);
        gather_layer(std::integral_constant<int, -1>(), own4[0]);
        gather_layer(std::integral_constant<int, 0>(), own4[1]);
        gather_layer(std::integral_constant<int, 1>(), own4[2]);
        __syncthreads();
        const int d = p - 1;
        if (d >= z0 && active) finish(d);
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    };

    fetch(z0 - 1, la, ra);
    fetch(z0, lb, rb);
    for (int p = z0 - 1; p <= z_end; p += 2) {
        plane_step(p, la, ra);
        if (p + 1 <= z_end) plane_step(p + 1, lb, rb);
    }

    // Fixed-order block sum of the relaxation-frequency sensitivity.
    red[tid] = dom;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partials[blockIdx.x] = red[0];
}

// Adds scale * sum(partials[0..n)) to *accum, in a fixed order.
__global__ __launch_bounds__(256) void k_add_partials(const double *__restrict__ partials, int n, double scale,
                                                      double *__restrict__ accum)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partials[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *accum += scale * sh[0];
}

template <int Q, class S, int TX, int TY, int WG_PER_CU>
hipError_t run(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out, double *partials,
               int max_partials, double *dtau_accum, bool stored)
{
    using R = typename Store<S>::real;
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.lay = c->lay;
    g.tiles_x = (c->nx + TX - 1) / TX;
    g.tiles_y = (c->ny + TY - 1) / TY;
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y, 256 * WG_PER_CU);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > max_partials) return hipErrorInvalidConfiguration;
    if (stored)
        hipLaunchKernelGGL((k_adjoint_tile<Q, S, TX, TY, true>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                           static_cast<const S *>(state), static_cast<const R *>(lam_in), static_cast<R *>(lam_out), g,
                           (R)c->omega, (R)(1.0 / c->s_pi), partials);
    else
        hipLaunchKernelGGL((k_adjoint_tile<Q, S, TX, TY, false>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                           static_cast<const S *>(state), static_cast<const R *>(lam_in), static_cast<R *>(lam_out), g,
                           (R)c->omega, (R)(1.0 / c->s_pi), partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dtau_accum) return e;
    // dL/dtau = dL/domega * domega/dtau = -omega^2 dL/domega
    hipLaunchKernelGGL(k_add_partials, dim3(1), dim3(256), 0, c->stream, partials, (int)blocks,
                       -c->omega * c->omega, dtau_accum);
    return hipGetLastError();
}

template <int Q>
hipError_t dispatch(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out, double *partials,
                    int max_partials, double *dtau, bool st)
{
    switch (c->storage) {
    case LBM_STORE_F64: return run<Q, double, 32, 8, 1>(c, state, lam_in, lam_out, partials, max_partials, dtau, st);
    case LBM_STORE_F32: return run<Q, float, 32, 16, 1>(c, state, lam_in, lam_out, partials, max_partials, dtau, st);
    case LBM_STORE_F16: return run<Q, f16, 32, 16, 1>(c, state, lam_in, lam_out, partials, max_partials, dtau, st);
    case LBM_STORE_BF16: return run<Q, bf16, 32, 16, 1>(c, state, lam_in, lam_out, partials, max_partials, dtau, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_adjoint_step(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out,
                               double *dtau_accum, bool stored)
{
    if (c->species != 1 || c->scheme != LBM_SCHEME_MOMENT) return hipErrorNotSupported;
    return c->q == 19 ? dispatch<19>(c, state, lam_in, lam_out, c->partials, kReduceBlocks * 5, dtau_accum, stored)
                      : dispatch<27>(c, state, lam_in, lam_out, c->partials, kReduceBlocks * 5, dtau_accum, stored);
}

} // namespace lbm
