// Two discrete-adjoint steps per launch (one species, co-states in the
// stored layout), the reverse counterpart of the two-step forward sweep.
//
// One adjoint step maps the co-state lam(t+1) to lam(t) = J(M(t))^T lam(t+1)
// (the transposed step written out in adjoint_step.hip): every node y
// publishes b_i = w_i m_i . lam(y), each node x gathers b_i from x + c_i
// into three plane accumulators, and a node-local map with the forward
// state M(t)(x) turns the finished accumulator into lam(t)(x).  Here a
// workgroup carries its tile through two such steps while it marches along
// z, so co-state and state cross HBM once per two steps:
//
//   * R0 = interior + two-node ring publishes b from lam(t+1) of plane p to
//     LDS buffer P0;
//   * R1 = interior + one-node ring gathers from P0, finishes plane p-1 of
//     lam(t) with the state M(t) and publishes b from it to buffer P1;
//   * the interior gathers from P1 and finishes plane p-2 of lam(t-1) with
//     the state M(t-1), which is stored.
//
// Each node runs the single adjoint step's own arithmetic, so lam(t-1)
// equals two single adjoint steps bit for bit; the relaxation-frequency
// sensitivity of both steps is summed per workgroup in a fixed order (equal
// to the two single-step sums up to FP64 rounding of the grouping).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "adjoint_math.hpp"
#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

template <int IX, int IY>
constexpr int kAdjSweepThreads = ((IX + 4) * (IY + 4) + 63) / 64 * 64;

// Buffer addressing of one z-plane (as in the forward sweep): descriptor in
// scalar registers, 32-bit node offset, field offset as an immediate.  The
// plane is below 2 GiB wherever the two-step passes are enabled.
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc2(const T *p, int64_t plane)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), (short)0, (int)(plane * (int64_t)sizeof(T)),
                                             0x00020000);
}
template <class T>
__device__ __forceinline__ T load_field2(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int k)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, k * kBlock * 4, 0));
    else if constexpr (sizeof(T) == 2)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rs, vo, k * kBlock * 2, 0));
}

// Position (x, y) of the m-th node of the one-node-wide ring of a W x H
// rectangle: top row, bottom row, left column, right column.
__device__ __forceinline__ void ring_pos2(int m, int W, int H, int &x, int &y)
{
    if (m < W) { x = m; y = 0; }
    else if (m < 2 * W) { x = m - W; y = H - 1; }
    else if (m < 2 * W + H - 2) { x = 0; y = 1 + (m - 2 * W); }
    else { x = W - 1; y = 1 + (m - 2 * W - (H - 2)); }
}

template <int Q, class S, int IX, int IY>
__global__ __launch_bounds__((kAdjSweepThreads<IX, IY>)) void k_adjoint_sweep2(
    const S *__restrict__ state_t1, const S *__restrict__ state_t0, const typename Store<S>::real *__restrict__ lam_in,
    typename Store<S>::real *__restrict__ lam_out, TileGrid g, typename Store<S>::real omega,
    typename Store<S>::real inv_s_pi, double *__restrict__ partials)
{
    using R = typename Store<S>::real;
    constexpr int HX0 = IX + 4, HY0 = IY + 4, N0 = HX0 * HY0;
    constexpr int HX1 = IX + 2, HY1 = IY + 2, N1 = HX1 * HY1;
    constexpr int NI = IX * IY;
    constexpr int NT = kAdjSweepThreads<IX, IY>;
    constexpr int NS = kLdsSlots<Q>;
    __shared__ R p0[NS * N0];
    __shared__ R p1[NS * N1];
    __shared__ double red[NT];

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * IX, y0 = ty * IY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = g.lay.plane;

    // Thread t holds one node in all its roles: interior nodes first (row by
    // row), then the one-node ring, then the outer ring.
    const int tid = threadIdx.x;
    const bool r0 = tid < N0, r1 = tid < N1, ri = tid < NI;
    int hx, hy;  // position in the R0 frame
    if (ri) { hx = tid % IX + 2; hy = tid / IX + 2; }
    else if (r1) { ring_pos2(tid - NI, HX1, HY1, hx, hy); hx += 1; hy += 1; }
    else { ring_pos2(r0 ? tid - N1 : 0, HX0, HY0, hx, hy); }
    const int h0 = hy * HX0 + hx;
    const int h1 = (hy - 1) * HX1 + (hx - 1);
    const int ix = tid % IX, iy = tid / IX;
    const bool active = ri && (x0 + ix < g.nx) && (y0 + iy < g.ny);
    const int64_t node_xy = r0 ? g.lay.xy(wrap_coord(x0 - 2 + hx, g.nx), wrap_coord(y0 - 2 + hy, g.ny)) : 0;

    MomentAcc<R> a1[3], a2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a1[k].zero();
        a2[k].zero();
    }
    double dom = 0.0;

    auto wrapz = [&](int p) { return p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p); };

    R la[10];  // lam(t+1) of the source plane; the next plane's loads are issued after publishing
    const uint32_t vo_r = (uint32_t)node_xy * (uint32_t)sizeof(R), vo_s = (uint32_t)node_xy * (uint32_t)sizeof(S);
    auto fetch = [&](int p, R *l) {
        if (!r0) return;
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc2(lam_in + (int64_t)wrapz(p) * plane, plane);
#pragma unroll
        for (int k = 0; k < 10; ++k) l[k] = load_field2<R>(rs, vo_r, k);
    };
    // Forward states for the node-local maps, loaded one plane ahead:
    // M(t) of R1 nodes and M(t-1) of interior nodes.
    S st1[10], st0[10];
    auto fetch_state = [&](const S *st, int d, S *v) {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc2(st + (int64_t)wrapz(d) * plane, plane);
#pragma unroll
        for (int k = 0; k < 10; ++k) v[k] = load_field2<S>(rs, vo_s, k);
    };

    auto publish = [&](const R *l, R *P, int n, int h, R *own) {
        Layer<R> L0, L1, L2;
        adjoint_layer<Q, -1, R>(l, L0);
        adjoint_layer<Q, 0, R>(l, L1);
        adjoint_layer<Q, 1, R>(l, L2);
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            if (lds_slot<Q>(-1, sl) >= 0) P[lds_slot<Q>(-1, sl) * n + h] = L0.v[sl];
            if (lds_slot<Q>(0, sl) >= 0) P[lds_slot<Q>(0, sl) * n + h] = L1.v[sl];
            if (lds_slot<Q>(1, sl) >= 0) P[lds_slot<Q>(1, sl) * n + h] = L2.v[sl];
        }
        own[0] = L0.v[4];
        own[1] = L1.v[4];
        own[2] = L2.v[4];
    };

    // Layer CZ gathered from x + c (where the forward step streamed to);
    // source plane p feeds destination plane p - CZ, accumulator acc[1 - CZ].
    auto gather_layer = [&](auto czc, const R *P, int n, int hx_, int h, R own, MomentAcc<R> *acc) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> f;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            f.v[sl] = R(0);
            if (sl == 4) f.v[sl] = own;
            else if (lds_slot<Q>(CZ, sl) >= 0) f.v[sl] = P[lds_slot<Q>(CZ, sl) * n + h + cy * hx_ + cx];
        }
        accumulate_layer<Q, CZ, R>(acc[1 - CZ], f);
    };

    auto finish = [&](const MomentAcc<R> &a, const S *v, R *lam) -> double {
        return adjoint_node<S>(a, v, omega, inv_s_pi, lam);
    };

    auto plane_step = [&](int p, R *l) {
        R own0[3], own1[3];
        if (r0) publish(l, p0, N0, h0, own0);
        __syncthreads();
        if (p + 1 <= z_end + 1) fetch(p + 1, l);

        if (r1) {
            gather_layer(std::integral_constant<int, -1>(), p0, N0, HX0, h0, own0[0], a1);
            gather_layer(std::integral_constant<int, 0>(), p0, N0, HX0, h0, own0[1], a1);
            gather_layer(std::integral_constant<int, 1>(), p0, N0, HX0, h0, own0[2], a1);
            // lam(t) of plane p-1 has gathered from p-2, p-1 and p.
            if (p >= z0) {
                const int d = p - 1;
                R lt[10];
                const double e = finish(a1[0], st1, lt);
                if (d + 1 <= z_end) fetch_state(state_t1, d + 1, st1);
                if (active && d >= z0 && d < z_end) dom += e;
                publish(lt, p1, N1, h1, own1);
            }
            a1[0] = a1[1];
            a1[1] = a1[2];
            a1[2].zero();
        }
        __syncthreads();

        if (p >= z0 && ri) {
            gather_layer(std::integral_constant<int, -1>(), p1, N1, HX1, h1, own1[0], a2);
            gather_layer(std::integral_constant<int, 0>(), p1, N1, HX1, h1, own1[1], a2);
            gather_layer(std::integral_constant<int, 1>(), p1, N1, HX1, h1, own1[2], a2);
            // lam(t-1) of plane p-2 has gathered from lam(t) of p-3, p-2, p-1.
            const int d = p - 2;
            if (d >= z0) {
                R lo[10];
                const double e = finish(a2[0], st0, lo);
                if (d + 1 < z_end) fetch_state(state_t0, d + 1, st0);
                if (active) {
                    dom += e;
                    const __amdgpu_buffer_rsrc_t rs = plane_rsrc2(lam_out + (int64_t)d * plane, plane);
#pragma unroll
                    for (int k = 0; k < 10; ++k)
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, lo[k]), rs, vo_r,
                                                              k * kBlock * 4, 2);
                }
            }
            a2[0] = a2[1];
            a2[1] = a2[2];
            a2[2].zero();
        }
    };

    if (r1) fetch_state(state_t1, z0 - 1, st1);
    if (ri) fetch_state(state_t0, z0, st0);
    fetch(z0 - 2, la);
    for (int p = z0 - 2; p <= z_end + 1; ++p) plane_step(p, la);

    // Fixed-order block sum of the sensitivity (NT is a multiple of 64).
    red[tid] = dom;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (tid < s && tid + s < NT) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partials[blockIdx.x] = red[0];
}

// Adds scale * sum(partials[0..n)) to *accum, in a fixed order.
__global__ __launch_bounds__(256) void k_add_partials2(const double *__restrict__ partials, int n, double scale,
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

// 64 x 8 tiles (832 threads, 4 waves per SIMD; a few registers spill) with
// the co-state loaded one plane ahead measured 2 % faster than 32 x 16 tiles
// with two planes in flight, and 16 % faster than 64 x 8 with two planes.
#ifndef LBM_ADJ_SWEEP_IX
#define LBM_ADJ_SWEEP_IX 64
#endif
#ifndef LBM_ADJ_SWEEP_IY
#define LBM_ADJ_SWEEP_IY 8
#endif

template <int Q, class S, int IX, int IY>
hipError_t run(const lbm_ctx *c, const void *state_t1, const void *state_t0, const void *lam_in, void *lam_out,
               double *dtau_accum)
{
    using R = typename Store<S>::real;
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.lay = c->lay;
    g.tiles_x = (c->nx + IX - 1) / IX;
    g.tiles_y = (c->ny + IY - 1) / IY;
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y, 256);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > (int64_t)kReduceBlocks * 5) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_adjoint_sweep2<Q, S, IX, IY>), dim3((unsigned)blocks), dim3(kAdjSweepThreads<IX, IY>), 0,
                       c->stream, static_cast<const S *>(state_t1), static_cast<const S *>(state_t0),
                       static_cast<const R *>(lam_in), static_cast<R *>(lam_out), g, (R)c->omega,
                       (R)(1.0 / c->s_pi), c->partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dtau_accum) return e;
    // dL/dtau = dL/domega * domega/dtau = -omega^2 dL/domega
    hipLaunchKernelGGL(k_add_partials2, dim3(1), dim3(256), 0, c->stream, c->partials, (int)blocks,
                       -c->omega * c->omega, dtau_accum);
    return hipGetLastError();
}

template <int Q>
hipError_t dispatch(const lbm_ctx *c, const void *s1, const void *s0, const void *li, void *lo, double *dt)
{
    switch (c->storage) {
    case LBM_STORE_F32: return run<Q, float, LBM_ADJ_SWEEP_IX, LBM_ADJ_SWEEP_IY>(c, s1, s0, li, lo, dt);
    case LBM_STORE_F16: return run<Q, f16, LBM_ADJ_SWEEP_IX, LBM_ADJ_SWEEP_IY>(c, s1, s0, li, lo, dt);
    case LBM_STORE_BF16: return run<Q, bf16, LBM_ADJ_SWEEP_IX, LBM_ADJ_SWEEP_IY>(c, s1, s0, li, lo, dt);
    default: return hipErrorNotSupported;
    }
}

} // namespace

hipError_t launch_adjoint_sweep2(const lbm_ctx *c, const void *state_t1, const void *state_t0, const void *lam_in,
                                 void *lam_out, double *dtau_accum)
{
    if (!moment_sweep2_supported(c)) return hipErrorNotSupported;
    return c->q == 19 ? dispatch<19>(c, state_t1, state_t0, lam_in, lam_out, dtau_accum)
                      : dispatch<27>(c, state_t1, state_t0, lam_in, lam_out, dtau_accum);
}

} // namespace lbm
