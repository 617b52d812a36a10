// Fused moment-only time step (one species), LDS-tiled for gfx950.
//
// The paper's step (Sec. II-III): every node's populations are rebuilt from
// its moments (Eq. 4), relaxed (Eqs. 7-8), pulled by the neighbours (Eq. 9),
// and only the moments of the streamed set (Eqs. 1-3) are stored.  Here each
// node is collided exactly once per step and its q post-collision
// populations are exchanged through LDS instead of being re-derived by each
// of its neighbours:
//
//   * a workgroup owns a TX x TY tile of the xy-plane and marches along z
//     over a chunk of planes;
//   * per source plane: every node of the tile plus a one-node halo loads its
//     10 moments (one coalesced pass over HBM), collides them in moment
//     space and writes its q shifted populations h~_i to LDS
//     (direction-major, so reads and writes are bank-conflict free);
//   * after a barrier, each interior node reads the q populations that
//     stream into its column (constant LDS offsets) and adds them to three
//     register accumulator sets, one per destination plane z-1, z, z+1;
//   * the accumulator set of plane z-1 is then complete and is stored.
//
// The moments of the next source plane are fetched into registers while the
// LDS phase of the current plane runs.  Tiles are numbered so that the
// workgroups an XCD receives (consecutive ids modulo 8) cover a contiguous
// block of tiles, keeping halo re-reads inside one L2.
//
// The paper's split approach (Sec. III.A) is available for comparison: a
// node-local collision pass relaxes the stored moments in place, and the
// tile kernel, instantiated with COLLIDED, then only reconstructs, pulls and
// sums.  It moves 36 stored values per node instead of 20.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

template <int Q, class S, int TX, int TY, bool COLLIDED>
__global__ __launch_bounds__(TX *TY) void k_moment_tile(const S *__restrict__ in, S *__restrict__ out, TileGrid g,
                                                        typename Store<S>::real omega,
                                                        typename Store<S>::real s_pi,
                                                        typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    constexpr bool kScaled = sizeof(S) == 2;  // 16-bit storage keeps S * s_pi
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int RING = HN - NT;             // halo nodes around the tile
    static_assert(RING <= NT, "halo ring must fit one pass");
    __shared__ R lds[kLdsSlots<Q> * HN];

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = g.lay.plane;  // stored elements per z-plane

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < g.nx) && (y0 + ly < g.ny);
    const int h0 = (ly + 1) * HX + (lx + 1);  // this thread's interior slot

    // Source nodes: pass 0 is the thread's own interior node, pass 1 a node
    // of the halo ring (threads tid < RING).  Periodic wrap is done once.
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
    auto wrap_xy = [&](int h) -> int64_t {
        const int hx = h % HX, hy = h / HX;
        return g.lay.xy(wrap_coord(x0 - 1 + hx, g.nx), wrap_coord(y0 - 1 + hy, g.ny));
    };
    const int64_t own_xy = wrap_xy(h0);
    const int64_t ring_xy = has_ring ? wrap_xy(hr) : 0;

    MomentAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();

    // Two register sets of source moments: while plane p is collided from
    // one, the loads of plane p+1 (issued a full plane earlier) land in the
    // other.
    Moments<R> own_a, own_b, ring_a, ring_b;
    auto fetch = [&](int p, Moments<R> &own, Moments<R> &ring) {
        const int zs = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
        load_moments<S>(in, kBlock, own_xy + (int64_t)zs * plane, own);
        if (has_ring) load_moments<S>(in, kBlock, ring_xy + (int64_t)zs * plane, ring);
    };

    auto collide_node = [&](const Moments<R> &v) {
        if constexpr (COLLIDED) {
            const R sc = kScaled ? inv_s_pi : R(1);
            return collided_from<R>(v.v[0], v.v[1], v.v[2], v.v[3], v.v[4] * sc, v.v[5] * sc, v.v[6] * sc,
                                    v.v[7] * sc, v.v[8] * sc, v.v[9] * sc);
        }
        return collide_stored<S>(v, omega, inv_s_pi);
    };

    // Writes the populations of one source node into LDS slot h; returns the
    // node's own-column values (slot 4 of each layer) through `own4`.
    auto publish = [&](const Collided<R> &c, int h, R *own4) {
        Layer<R> L0, L1, L2;
        reconstruct_layer<Q, -1, R>(c, L0);
        reconstruct_layer<Q, 0, R>(c, L1);
        reconstruct_layer<Q, 1, R>(c, L2);
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

    // Gathers layer CZ of the populations streaming into this thread's node.
    auto pull_layer = [&](auto czc, R own) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> f;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            if (sl == 4) f.v[sl] = own;
            else if (lds_slot<Q>(CZ, sl) >= 0) f.v[sl] = lds[lds_slot<Q>(CZ, sl) * HN + h0 - cy * HX - cx];
        }
        accumulate_layer<Q, CZ, R>(acc[CZ + 1], f);
    };

    auto plane_step = [&](int p, Moments<R> &own_m, Moments<R> &ring_m) {
        R own4[3];
        publish(collide_node(own_m), h0, own4);
        if (has_ring) publish(collide_node(ring_m), hr, nullptr);
        __syncthreads();
        if (p + 2 <= z_end) fetch(p + 2, own_m, ring_m);

        // Pull: direction c arrives from (x - c); layer cz feeds plane p + cz.
        pull_layer(std::integral_constant<int, -1>(), own4[0]);
        pull_layer(std::integral_constant<int, 0>(), own4[1]);
        pull_layer(std::integral_constant<int, 1>(), own4[2]);
        __syncthreads();

        // Plane p-1 has now received from p-2, p-1 and p.
        const int d = p - 1;
        if (d >= z0 && active) {
            const int64_t o = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)d * plane;
            S v[10];
            stored_moments<S>(acc[0], s_pi, v);
#pragma unroll
            for (int k = 0; k < 10; ++k) store_out(out + k * kBlock + o, v[k]);
        }
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    };

    fetch(z0 - 1, own_a, ring_a);
    fetch(z0, own_b, ring_b);
    for (int p = z0 - 1; p <= z_end; p += 2) {
        plane_step(p, own_a, ring_a);
        if (p + 1 <= z_end) plane_step(p + 1, own_b, ring_b);
    }
}

// Collision pass of the split approach: (dr, j, S) -> (dr, j, S') in place
// at every stored node slot (dr and j unchanged, not rewritten).  One thread
// per slot; the slots of unused block edges hold zeros and stay zero.
template <class S>
__global__ __launch_bounds__(256) void k_moment_collide(S *__restrict__ st, int64_t slots,
                                                        typename Store<S>::real omega,
                                                        typename Store<S>::real s_pi,
                                                        typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    constexpr bool kScaled = sizeof(S) == 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= slots) return;
    const int64_t base = (t / kBlock) * (10 * kBlock) + t % kBlock;
    Moments<R> v;
    load_moments<S>(st, kBlock, base, v);
    const R si = kScaled ? inv_s_pi : R(1);
    const Collided<R> p = collide<R>(v.v[0], v.v[1], v.v[2], v.v[3], v.v[4] * si, v.v[5] * si, v.v[6] * si,
                                     v.v[7] * si, v.v[8] * si, v.v[9] * si, omega);
    const R so = kScaled ? s_pi : R(1);
    store_out(st + base + 4 * kBlock, Store<S>::make(kScaled ? p.sxx * so : p.sxx));
    store_out(st + base + 5 * kBlock, Store<S>::make(kScaled ? p.syy * so : p.syy));
    store_out(st + base + 6 * kBlock, Store<S>::make(kScaled ? p.szz * so : p.szz));
    store_out(st + base + 7 * kBlock, Store<S>::make(kScaled ? p.sxy * so : p.sxy));
    store_out(st + base + 8 * kBlock, Store<S>::make(kScaled ? p.sxz * so : p.sxz));
    store_out(st + base + 9 * kBlock, Store<S>::make(kScaled ? p.syz * so : p.syz));
}

template <class S>
hipError_t run_collide(const lbm_ctx *c, void *state)
{
    using R = typename Store<S>::real;
    const int64_t slots = c->lay.plane / 10 * c->nz;
    const int64_t blocks = (slots + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_moment_collide<S>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                       static_cast<S *>(state), slots, (R)c->omega, (R)c->s_pi, (R)(1.0 / c->s_pi));
    return hipGetLastError();
}

template <int Q, class S, int TX, int TY, int WG_PER_CU, bool COLLIDED>
hipError_t run(const lbm_ctx *c, const void *in, void *out)
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
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_moment_tile<Q, S, TX, TY, COLLIDED>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                       static_cast<const S *>(in), static_cast<S *>(out), g, (R)c->omega, (R)c->s_pi,
                       (R)(1.0 / c->s_pi));
    return hipGetLastError();
}

// Tiles for FP32 and 16-bit storage: 1024 threads, one workgroup per CU.
// Where 256-node rows cover nx exactly, 256 x 4 tiles (each plane of a tile is
// one contiguous 1 KB run per field across four stored blocks; 149 KB of LDS
// for D3Q27 FP32) measured 3-4 % faster than 64 x 16 tiles (one stored block,
// 114 KB), despite a halo ring of half the tile; other grids use 64 x 16.
// FP64 uses 32 x 8 (two per CU), its populations taking twice the LDS.
template <int Q, class S, bool COLLIDED>
hipError_t run_wide(const lbm_ctx *c, const void *in, void *out)
{
    return c->nx % 256 == 0 ? run<Q, S, 256, 4, 1, COLLIDED>(c, in, out) : run<Q, S, 64, 16, 1, COLLIDED>(c, in, out);
}

template <int Q, bool COLLIDED>
hipError_t dispatch_storage(const lbm_ctx *c, const void *in, void *out)
{
    switch (c->storage) {
    case LBM_STORE_F64: return run<Q, double, 32, 8, 2, COLLIDED>(c, in, out);
    case LBM_STORE_F32: return run_wide<Q, float, COLLIDED>(c, in, out);
    case LBM_STORE_F16: return run_wide<Q, f16, COLLIDED>(c, in, out);
    case LBM_STORE_BF16: return run_wide<Q, bf16, COLLIDED>(c, in, out);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_moment_step(const lbm_ctx *c, const void *in, void *out, bool collided)
{
    if (c->species != 1) return hipErrorNotSupported;
    if (collided) return c->q == 19 ? dispatch_storage<19, true>(c, in, out) : dispatch_storage<27, true>(c, in, out);
    return c->q == 19 ? dispatch_storage<19, false>(c, in, out) : dispatch_storage<27, false>(c, in, out);
}

hipError_t launch_moment_collide(const lbm_ctx *c, void *state)
{
    if (c->species != 1) return hipErrorNotSupported;
    switch (c->storage) {
    case LBM_STORE_F64: return run_collide<double>(c, state);
    case LBM_STORE_F32: return run_collide<float>(c, state);
    case LBM_STORE_F16: return run_collide<f16>(c, state);
    case LBM_STORE_BF16: return run_collide<bf16>(c, state);
    default: return hipErrorInvalidValue;
    }
}

} // namespace lbm
