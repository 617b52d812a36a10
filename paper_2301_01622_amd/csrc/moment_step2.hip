// Two time steps per sweep of the moment-only scheme (one species),
// LDS-tiled for gfx950.
//
// The single step reads every stored moment once and writes it once, 80 B
// per node and step at FP32, and HBM bandwidth bounds it.  Here a workgroup
// carries its tile through two consecutive steps (Sec. II-III, Eqs. 4-9,
// applied twice) while it marches along z, so the state crosses HBM once per
// two steps:
//
//   * source region R0 = interior tile plus a two-node ring: each node loads
//     its 10 moments of plane p, collides them and writes its q populations
//     to LDS buffer P0;
//   * region R1 = interior plus a one-node ring: each node pulls the
//     populations of plane p from P0 into three accumulator planes (p-1, p,
//     p+1).  Plane p-1 of the intermediate state is then complete; it is
//     rounded to the storage format exactly as a stored state would be,
//     collided, and its populations are written to LDS buffer P1;
//   * interior nodes pull from P1 into three more accumulator planes; plane
//     p-2 of the second step is then complete and is stored.
//
// Each thread holds one node in all its roles (interior nodes first, row by
// row, then the one-node ring, then the outer ring), so the populations a
// node keeps in its own column stay in registers and the interior's loads
// and stores cover whole rows.  Each node of R1 and of the interior computes exactly the
// arithmetic of the single step (the same collision, reconstruction and
// layer sums, FMAs explicit), so a sweep equals two single steps bit for bit.
// The cost is the redundant work on the two rings (R0 and R1 are 1.59x and
// 1.29x the interior of a 64 x 8 tile): the sweep is bound by arithmetic and
// LDS rather than HBM (without any global access it still takes 80 % of its
// time).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

template <int IX, int IY>
constexpr int kSweepThreads = ((IX + 4) * (IY + 4) + 63) / 64 * 64;

// Buffer addressing of one z-plane of the stored state: the descriptor (base
// and range of the plane) sits in scalar registers, the node's byte offset is
// one 32-bit vector register and the field offset an immediate, so no 64-bit
// address arithmetic runs in the vector unit (measured 3-4 % faster than
// global loads and stores).  The range is the plane: planes must stay below
// 2 GiB (moment_sweep2_supported checks it).
template <class S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const S *p, int64_t plane)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(p), (short)0, (int)(plane * (int64_t)sizeof(S)),
                                             0x00020000);
}
template <class S>
__device__ __forceinline__ S load_field(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int k)
{
    if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, k * kBlock * 4, 0));
    else if constexpr (sizeof(S) == 2)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(rs, vo, k * kBlock * 2, 0));
}
// Nontemporal store (cache-policy bit 1), as the other kernels' stores.
template <class S>
__device__ __forceinline__ void store_field(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int k, S v)
{
    if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, vo, k * kBlock * 4, 2);
    else if constexpr (sizeof(S) == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), rs, vo, k * kBlock * 2, 2);
}

// Position (x, y) of the m-th node of the one-node-wide ring of a W x H
// rectangle: top row, bottom row, left column, right column.
__device__ __forceinline__ void ring_pos(int m, int W, int H, int &x, int &y)
{
    if (m < W) { x = m; y = 0; }
    else if (m < 2 * W) { x = m - W; y = H - 1; }
    else if (m < 2 * W + H - 2) { x = 0; y = 1 + (m - 2 * W); }
    else { x = W - 1; y = 1 + (m - 2 * W - (H - 2)); }
}

// MID: the intermediate state (after the first step) is stored to `mid`
// as well, for the recomputation of forward states in reverse mode.
template <int Q, class S, int IX, int IY, bool MID>
__global__ __launch_bounds__((kSweepThreads<IX, IY>)) void k_moment_sweep2(const S *__restrict__ in,
                                                                        S *__restrict__ out, S *__restrict__ mid,
                                                                        TileGrid g,
                                                                        typename Store<S>::real omega,
                                                                        typename Store<S>::real s_pi,
                                                                        typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    constexpr int HX0 = IX + 4, HY0 = IY + 4, N0 = HX0 * HY0;  // R0: sources of the first step
    constexpr int HX1 = IX + 2, HY1 = IY + 2, N1 = HX1 * HY1;  // R1: results of the first step
    constexpr int NI = IX * IY;
    constexpr int NS = kLdsSlots<Q>;  // directions leaving the own column
    __shared__ R p0[NS * N0];
    __shared__ R p1[NS * N1];

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * IX, y0 = ty * IY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = g.lay.plane;

    // Thread t holds one node in all its roles: t < NI an interior node (row
    // by row, so waves cover whole 64-node rows), then the nodes of the
    // one-node ring, then those of the outer ring.  A node's own-column
    // populations therefore never leave its thread's registers.
    const int tid = threadIdx.x;
    const bool r0 = tid < N0, r1 = tid < N1, ri = tid < NI;
    int hx, hy;  // position in the R0 frame
    if (ri) { hx = tid % IX + 2; hy = tid / IX + 2; }
    else if (r1) { ring_pos(tid - NI, HX1, HY1, hx, hy); hx += 1; hy += 1; }
    else { ring_pos(r0 ? tid - N1 : 0, HX0, HY0, hx, hy); }
    const int h0 = hy * HX0 + hx;              // slot in P0
    const int h1 = (hy - 1) * HX1 + (hx - 1);  // slot in P1 (R1 nodes)
    const int ix = tid % IX, iy = tid / IX;
    const bool active = ri && (x0 + ix < g.nx) && (y0 + iy < g.ny);
    const int64_t src_xy = r0 ? g.lay.xy(wrap_coord(x0 - 2 + hx, g.nx), wrap_coord(y0 - 2 + hy, g.ny)) : 0;
    const int64_t dst_xy = active ? g.lay.xy(x0 + ix, y0 + iy) : 0;

    MomentAcc<R> a1[3], a2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a1[k].zero();
        a2[k].zero();
    }

    Moments<R> m_a, m_b;  // moments of source planes p and p+1 (loads in flight)
    auto fetch = [&](int p, Moments<R> &m) {
        if (!r0) return;
        const int zs = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(in + (int64_t)zs * plane, plane);
        const uint32_t vo = (uint32_t)src_xy * (uint32_t)sizeof(S);
#pragma unroll
        for (int k = 0; k < 10; ++k) m.v[k] = Store<S>::load(load_field<S>(rs, vo, k));
    };

    auto collide_node = [&](const Moments<R> &v) { return collide_stored<S>(v, omega, inv_s_pi); };
    auto stored_values = [&](const MomentAcc<R> &a, S *v) { stored_moments<S>(a, s_pi, v); };

    // Writes the populations leaving the own column to slot h of P (n
    // slots per direction); the own-column ones go to own[3].
    auto publish = [&](const Collided<R> &c, R *P, int n, int h, R *own) {
        Layer<R> L0, L1, L2;
        reconstruct_layer<Q, -1, R>(c, L0);
        reconstruct_layer<Q, 0, R>(c, L1);
        reconstruct_layer<Q, 1, R>(c, L2);
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

    // Layer CZ of the populations streaming into slot h of P (rows of hx),
    // added to acc.
    auto pull_layer = [&](auto czc, const R *P, int n, int hx_, int h, R own, MomentAcc<R> &acc) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> f;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            f.v[sl] = R(0);
            if (sl == 4) f.v[sl] = own;
            else if (lds_slot<Q>(CZ, sl) >= 0) f.v[sl] = P[lds_slot<Q>(CZ, sl) * n + h - cy * hx_ - cx];
        }
        accumulate_layer<Q, CZ, R>(acc, f);
    };

    // One source plane p: first-step populations of p, intermediate plane
    // p-1, second-step plane p-2.
    auto plane_step = [&](int p, Moments<R> &m) {
        R own0[3], own1[3];
        S vm[10];  // the intermediate state, stored after the second barrier (MID)
        if (r0) publish(collide_node(m), p0, N0, h0, own0);
        __syncthreads();
        if (p + 2 <= z_end + 1) fetch(p + 2, m);

        if (r1) {
            pull_layer(std::integral_constant<int, -1>(), p0, N0, HX0, h0, own0[0], a1[0]);
            pull_layer(std::integral_constant<int, 0>(), p0, N0, HX0, h0, own0[1], a1[1]);
            pull_layer(std::integral_constant<int, 1>(), p0, N0, HX0, h0, own0[2], a1[2]);
            // Intermediate plane p-1 has received from p-2, p-1 and p.
            if (p >= z0) {
                S *v = vm;
                stored_values(a1[0], v);
                Moments<R> mi;
#pragma unroll
                for (int k = 0; k < 10; ++k) mi.v[k] = Store<S>::load(v[k]);
                publish(collide_node(mi), p1, N1, h1, own1);
            }
            a1[0] = a1[1];
            a1[1] = a1[2];
            a1[2].zero();
        }
        __syncthreads();

        if (p >= z0 && ri) {
            pull_layer(std::integral_constant<int, -1>(), p1, N1, HX1, h1, own1[0], a2[0]);
            pull_layer(std::integral_constant<int, 0>(), p1, N1, HX1, h1, own1[1], a2[1]);
            pull_layer(std::integral_constant<int, 1>(), p1, N1, HX1, h1, own1[2], a2[2]);
            // Second-step plane p-2 has received from intermediate planes p-3, p-2, p-1.
            const int d = p - 2;
            if (d >= z0 && active) {
                S v[10];
                stored_values(a2[0], v);
                const __amdgpu_buffer_rsrc_t rs = plane_rsrc(out + (int64_t)d * plane, plane);
                const uint32_t vo = (uint32_t)dst_xy * (uint32_t)sizeof(S);
#pragma unroll
                for (int k = 0; k < 10; ++k) store_field<S>(rs, vo, k, v[k]);
            }
            if (MID && active && p - 1 >= z0 && p - 1 < z_end) {
                const __amdgpu_buffer_rsrc_t rs = plane_rsrc(mid + (int64_t)(p - 1) * plane, plane);
                const uint32_t vo = (uint32_t)dst_xy * (uint32_t)sizeof(S);
#pragma unroll
                for (int k = 0; k < 10; ++k) store_field<S>(rs, vo, k, vm[k]);
            }
            a2[0] = a2[1];
            a2[1] = a2[2];
            a2[2].zero();
        }
    };

    // Source planes z0-2 .. z_end+1 feed second-step planes z0 .. z_end-1.
    fetch(z0 - 2, m_a);
    fetch(z0 - 1, m_b);
    for (int p = z0 - 2; p <= z_end + 1; p += 2) {
        plane_step(p, m_a);
        if (p + 1 <= z_end + 1) plane_step(p + 1, m_b);
    }
}

#ifndef LBM_SWEEP_WG
#define LBM_SWEEP_WG 1
#endif

template <int Q, class S, int IX, int IY>
hipError_t run(const lbm_ctx *c, const void *in, void *out, void *mid)
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
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y, 256 * LBM_SWEEP_WG);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (mid)
        hipLaunchKernelGGL((k_moment_sweep2<Q, S, IX, IY, true>), dim3((unsigned)blocks), dim3(kSweepThreads<IX, IY>),
                           0, c->stream, static_cast<const S *>(in), static_cast<S *>(out), static_cast<S *>(mid), g,
                           (R)c->omega, (R)c->s_pi, (R)(1.0 / c->s_pi));
    else
        hipLaunchKernelGGL((k_moment_sweep2<Q, S, IX, IY, false>), dim3((unsigned)blocks),
                           dim3(kSweepThreads<IX, IY>), 0, c->stream, static_cast<const S *>(in),
                           static_cast<S *>(out), nullptr, g, (R)c->omega, (R)c->s_pi, (R)(1.0 / c->s_pi));
    return hipGetLastError();
}

// Interior tile 64 x 8: full 64-node rows of the stored blocks, 832 threads,
// 159 KB of LDS for D3Q27 FP32 (the largest 64-wide tile that fits).
// Measured on 256^3 D3Q27 FP32: 92 GLUPS, against 84 for 32 x 16 tiles and
// 65 for 16 x 16 (two workgroups per CU) or 64 x 4.
#ifndef LBM_SWEEP_IX
#define LBM_SWEEP_IX 64
#endif
#ifndef LBM_SWEEP_IY
#define LBM_SWEEP_IY 8
#endif

template <int Q>
hipError_t dispatch_storage(const lbm_ctx *c, const void *in, void *out, void *mid)
{
    switch (c->storage) {
    case LBM_STORE_F32: return run<Q, float, LBM_SWEEP_IX, LBM_SWEEP_IY>(c, in, out, mid);
    case LBM_STORE_F16: return run<Q, f16, LBM_SWEEP_IX, LBM_SWEEP_IY>(c, in, out, mid);
    case LBM_STORE_BF16: return run<Q, bf16, LBM_SWEEP_IX, LBM_SWEEP_IY>(c, in, out, mid);
    default: return hipErrorNotSupported;
    }
}

} // namespace

bool moment_sweep2_supported(const lbm_ctx *c)
{
    // The buffer descriptors address one z-plane of at most 2 GiB.
    const bool plane_fits = c->lay.plane * (int64_t)c->elem < ((int64_t)1 << 31);
    return c->scheme == LBM_SCHEME_MOMENT && c->species == 1 && !c->split && c->storage != LBM_STORE_F64 &&
           plane_fits;
}

hipError_t launch_moment_sweep2(const lbm_ctx *c, const void *in, void *out, void *mid)
{
    if (!moment_sweep2_supported(c)) return hipErrorNotSupported;
    return c->q == 19 ? dispatch_storage<19>(c, in, out, mid) : dispatch_storage<27>(c, in, out, mid);
}

} // namespace lbm
