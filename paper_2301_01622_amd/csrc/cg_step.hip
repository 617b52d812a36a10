// Fused moment-only time step for two components (colour-gradient model).
//
// The paper carries two species on one flow field (Sec. III.A): per species
// only a density is stored, the density gradient is taken on the streamed
// (pre-collision) state, and the perturbation and recolouring operators act
// on the populations of Eq. 8.  Stored state per node (11 arrays): the
// mixture deviation dr = rho - 1, rho1, j, S = P - rho c_s^2 I.
//
// Per source node y (tile plus one-node halo):
//   phi   = (rho1 - rho2)/rho on a radius-2 footprint, kept in LDS for the
//           three planes z-1, z, z+1 (computed one plane ahead);
//   G     = (1/c_s^2) sum_i w_i c_i phi(y + c_i),  D = sqrt(|G|^2 + 1e-6),  n = G/D;
//   S'    = (1 - omega) S + omega j j/rho + (A/9)(G G - |G|^2 I)/D  (collision
//           plus the second moment of the perturbation operator);
//   h~_i  = w_i [T + 3 c_i.j + 4.5 c_i c_i : S'],  T = dr - 1.5 tr S';
//   f1_i  = (rho1/rho)(w_i + h~_i) + beta (rho1 rho2/rho) w_i (c_i.n)/|c_i|.
// Both h~_i and f1_i go through LDS; each interior node pulls them from
// x - c_i, sums the mixture moments from h~ and rho1 from f1.  The structure
// (z-marching tiles, three accumulator planes, two-plane prefetch,
// XCD-aware tile order) is that of the one-component kernel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cg_math.hpp"
#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

// Buffer addressing of one z-plane: the descriptor (base and byte range of
// the plane) sits in scalar registers, the node's byte offset in one 32-bit
// vector register and the field offset in a scalar one, so no 64-bit address
// arithmetic runs in the vector unit (the stored fields lie 4 KiB apart,
// beyond the immediate offset of global accesses).  Accesses beyond the range
// read 0 and write nothing.  A plane must stay below 2 GiB (lbm_create checks
// it for two species).
template <class R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_buf(const R *p, int64_t elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R *>(p), (short)0, (int)(elems * (int64_t)sizeof(R)),
                                             0x00020000);
}
template <class R>
__device__ __forceinline__ R buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int so)
{
    if constexpr (sizeof(R) == 4)
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
    else
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
}
// Nontemporal store (cache-policy bit 1), as the other kernels' stores.
template <class R>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int so, R v)
{
    if constexpr (sizeof(R) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, vo, so, 2);
    } else {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0u, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), rs, vo, so, 2);
    }
}

template <class R>
struct CgAcc {
    MomentAcc<R> m;
    R rho1;
    __device__ __forceinline__ void zero()
    {
        m.zero();
        rho1 = R(0);
    }
};

template <int Q>
__host__ __device__ constexpr double inv_speed(int cx, int cy, int cz)
{
    return (cx * cx + cy * cy + cz * cz) == 1 ? 1.0 : (cx * cx + cy * cy + cz * cz) == 2 ? 0.70710678118654752440
                                                                                           : 0.57735026918962576451;
}

// LDS layout of the published populations.  Slot s (one moving direction
// c, the own column (0, 0, +-1) excepted; see lds_slot) holds one value per
// node that can send c into the tile: the tile widened by one node on the
// side c comes from, i.e. x in [-1, TX) for c_x = 1, [0, TX] for c_x = -1,
// [0, TX) for c_x = 0, and likewise in y.  Region s is a (TX + |c_x|) x
// (TY + |c_y|) block, row-major, at offset O(s); a node at source-region
// coordinates (hx, hy) = (x + 1, y + 1) sits at OFF(s) + hy W(s) + hx with
// W(s) = TX + |c_x|, so every index is a per-node base (hy TX + hx or
// hy (TX + 1) + hx) plus a compile-time offset.
template <int Q, int TX, int TY>
struct SlotLayout {
    struct Dir {
        int cx, cy, cz;
    };
    static constexpr Dir dir(int s)
    {
        int k = 0;
        for (int z = -1; z <= 1; ++z)
            for (int sl = 0; sl < 9; ++sl) {
                if (sl == 4 || !has_dir<Q>(sl % 3 - 1, sl / 3 - 1, z)) continue;
                if (k == s) return Dir{sl % 3 - 1, sl / 3 - 1, z};
                ++k;
            }
        return Dir{0, 0, 0};
    }
    static constexpr int width(int s) { return TX + (dir(s).cx != 0 ? 1 : 0); }
    static constexpr int height(int s) { return TY + (dir(s).cy != 0 ? 1 : 0); }
    static constexpr int start(int s)
    {
        int o = 0;
        for (int k = 0; k < s; ++k) o += width(k) * height(k);
        return o;
    }
    static constexpr int total() { return start(kLdsSlots<Q>); }
    // OFF(s): start(s) minus the region coordinates of source node (0, 0).
    static constexpr int off(int s)
    {
        return start(s) - (dir(s).cy > 0 ? 0 : 1) * width(s) - (dir(s).cx > 0 ? 0 : 1);
    }
};

// FORCE: a body force (three arrays of N values, x fastest) enters the
// mixture collision with Guo's forcing: u* = (j + F/2)/rho in the
// equilibrium, (1 - omega/2)(u* F + F u*) added to the collided S, j + F
// streamed; the phase field phi = 2 rho1/rho - 1 of the stored output is
// written to phi_out (N values, x fastest) for the next step's force.
// fdirty holds the near-contact pass's per-block flags: where a node's block
// flag is zero its force is zero and is not read.
// COLL (split schedule): `in` holds post-collision moments (S' with the
// perturbation, j + F under a force) and frc the interface normal n (three
// arrays of N values); the step then only reconstructs, recolours, pulls and
// sums, with the same arithmetic per node as the fused step.
// Threads of a workgroup: one per interior node; with SR (separate ring
// threads) the halo ring's nodes get threads of their own after them (rows,
// then columns, each from a multiple of 64), so that no thread handles two
// nodes.
template <int TX, int TY, bool SR>
constexpr int kCgThreads = SR ? TX * TY + (2 * TX + 63) / 64 * 64 + (2 * (TY + 2) + 63) / 64 * 64 : TX * TY;

template <int Q, class R, int TX, int TY, bool FORCE, int WPE, bool COLL = false, bool SR = false>
__global__ __launch_bounds__((kCgThreads<TX, TY, SR>), WPE) void k_cg_tile(
    const R *__restrict__ in, R *__restrict__ out, TileGrid g, R omega, R A9, R beta, const R *__restrict__ frc,
    R *__restrict__ phi_out, const uint8_t *__restrict__ fdirty)
{
    static_assert(!(FORCE && COLL), "the split schedule applies the force in its collision pass");
    constexpr bool VEC3 = FORCE || COLL;  // three extra arrays per node (F, or n)
    constexpr int NT = TX * TY;
    constexpr int SX = TX + 2, SY = TY + 2, SN = SX * SY;  // source region (radius 1)
    constexpr int FX = TX + 4, FY = TY + 4, FN = FX * FY;  // phase-field region (radius 2)
    constexpr int RING = SN - NT;                          // radius-1 halo nodes
    constexpr int OUTER = FN - SN;                         // radius-2 ring (phi only)
    static_assert(RING <= NT && OUTER <= NT, "halo rings must fit one pass");
    constexpr int NS = kLdsSlots<Q>;
    using SL = SlotLayout<Q, TX, TY>;
    // Per published direction and node: the shifted mixture population h~
    // and the species-1 population f1, side by side (one wide LDS access).
    struct alignas(2 * sizeof(R)) HF {
        R h, f;
    };
    __shared__ HF lds_hf[SL::total()];
    __shared__ R lds_phi[3 * FN];  // phase field of three planes

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = g.lay.plane;  // stored elements per z-plane

    const int tid = threadIdx.x;
    const bool interior = !SR || tid < NT;
    const int lx = tid % TX, ly = interior ? tid / TX : 0;
    const bool active = interior && (x0 + lx < g.nx) && (y0 + ly < g.ny);
    const int h0 = (ly + 1) * SX + (lx + 1);

    // Radius-1 ring node of this thread (source region coordinates).  The
    // ring nodes of the top and bottom rows (x inside the tile) take threads
    // [0, 2 TX); those of the left and right columns (corners included) take
    // threads from the next multiple of 64 on, so that every wave holds ring
    // nodes of one orientation only.  A ring node sends into the tile only
    // the directions with c_y = d (rows) or c_x = d (columns), d its inward
    // sign.
    constexpr int R0 = SR ? NT : 0;  // first ring thread
    constexpr int ROWS = 2 * TX, CB = R0 + (ROWS + 63) / 64 * 64, COLS = 2 * SY;
    static_assert(ROWS + COLS == RING && CB + COLS <= kCgThreads<TX, TY, SR>, "ring threads must fit the workgroup");
    const bool ring_row = tid >= R0 && tid < R0 + ROWS;
    const bool ring_col = tid >= CB && tid < CB + COLS;
    const bool has_ring = ring_row || ring_col;
    int hr = 0, dsign = 1;
    if (ring_row) {
        const bool top = tid - R0 < TX;
        hr = (top ? 0 : SY - 1) * SX + 1 + (top ? tid - R0 : tid - R0 - TX);
        dsign = top ? 1 : -1;
    } else if (ring_col) {
        const int m = tid - CB;
        const bool left = m < SY;
        hr = (left ? m : m - SY) * SX + (left ? 0 : SX - 1);
        dsign = left ? 1 : -1;
    }
    // Radius-2 ring node of this thread (phase-field region coordinates);
    // with SR on the ring threads.
    static_assert(!SR || OUTER <= kCgThreads<TX, TY, SR> - NT, "outer ring must fit the ring threads");
    const bool has_outer = tid >= R0 && tid - R0 < OUTER;
    int ko;
    {
        const int m = tid - R0;
        int kx, ky;
        if (m < FX) { kx = m; ky = 0; }
        else if (m < 2 * FX) { kx = m - FX; ky = FY - 1; }
        else if (m < 2 * FX + SY) { kx = 0; ky = 1 + (m - 2 * FX); }
        else { kx = FX - 1; ky = 1 + (m - 2 * FX - SY); }
        ko = ky * FX + kx;
    }
    auto src_to_phi = [](int h) { return (h / SX + 1) * FX + (h % SX + 1); };
    auto xy_src = [&](int h) -> int64_t {
        return g.lay.xy(wrap_coord(x0 - 1 + h % SX, g.nx), wrap_coord(y0 - 1 + h / SX, g.ny));
    };
    const int64_t own_xy = xy_src(h0);
    const int64_t ring_xy = has_ring ? xy_src(hr) : 0;
    const int ring_y = hr / SX - 1;  // tile row of the ring node (-1 .. TY)
    // Offsets of the force arrays (public layout) of the two source nodes.
    auto lin_src = [&](int h) -> int64_t {
        return (int64_t)wrap_coord(x0 - 1 + h % SX, g.nx) + (int64_t)g.nx * wrap_coord(y0 - 1 + h / SX, g.ny);
    };
    const int64_t own_lin = VEC3 ? lin_src(h0) : 0;
    const int64_t ring_lin = VEC3 && has_ring ? lin_src(hr) : 0;
    // Force-flag blocks of the two source nodes (FORCE), in plane 0.
    const int fgx = (g.nx + kNcBlockX - 1) / kNcBlockX;
    const int64_t fgxy = (int64_t)fgx * ((g.ny + kNcBlockY - 1) / kNcBlockY);
    auto blk_src = [&](int h) -> int64_t {
        return wrap_coord(x0 - 1 + h % SX, g.nx) / kNcBlockX +
               (int64_t)fgx * (wrap_coord(y0 - 1 + h / SX, g.ny) / kNcBlockY);
    };
    const int64_t own_blk = FORCE ? blk_src(h0) : 0;
    const int64_t ring_blk = FORCE && has_ring ? blk_src(hr) : 0;
    const int64_t plane_lin = (int64_t)g.nx * g.ny;
    const int64_t outer_xy =
        has_outer ? g.lay.xy(wrap_coord(x0 - 2 + ko % FX, g.nx), wrap_coord(y0 - 2 + ko / FX, g.ny))
                  : 0;
    const int k_own = src_to_phi(h0), k_ring = src_to_phi(hr);
    // LDS bases (SlotLayout) of the two source nodes: hy TX + hx and
    // hy (TX + 1) + hx.
    auto base_a = [](int h) { return (h / SX) * TX + h % SX; };
    auto base_b = [](int h) { return (h / SX) * (TX + 1) + h % SX; };
    const int ba0 = base_a(h0), bb0 = base_b(h0), bar = base_a(hr), bbr = base_b(hr);
    auto lds_at = [&](int s, int ba, int bb) { return SL::off(s) + (SL::width(s) == TX ? ba : bb); };

    using M11 = Moments<R, 11>;
    struct PlaneRegs {
        M11 own, ring;
        R outer_dr, outer_r1;
        R fox, foy, foz, frx, fry, frz;  // force at the two source nodes (FORCE)
    };
    PlaneRegs pa, pb;
    auto zwrap = [&](int p) { return p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p); };
    // Byte offsets within one plane: the stored state (fields kBlock apart)
    // and the public-layout arrays (one descriptor per field).
    constexpr int FB = kBlock * (int)sizeof(R);
    const uint32_t own_vo = (uint32_t)own_xy * (uint32_t)sizeof(R);
    const uint32_t ring_vo = (uint32_t)ring_xy * (uint32_t)sizeof(R);
    const uint32_t outer_vo = (uint32_t)outer_xy * (uint32_t)sizeof(R);
    const uint32_t own_lvo = (uint32_t)own_lin * (uint32_t)sizeof(R);
    const uint32_t ring_lvo = (uint32_t)ring_lin * (uint32_t)sizeof(R);
    const uint32_t dst_vo = active ? (uint32_t)g.lay.xy(x0 + lx, y0 + ly) * (uint32_t)sizeof(R) : 0u;
    const uint32_t dst_lvo = active ? (uint32_t)((x0 + lx) + g.nx * (y0 + ly)) * (uint32_t)sizeof(R) : 0u;
    // With SR a ring thread keeps its node in the `own` registers.
    const uint32_t node_vo = SR && !interior ? ring_vo : own_vo;
    const uint32_t node_lvo = SR && !interior ? ring_lvo : own_lvo;
    const int64_t node_blk = SR && !interior ? ring_blk : own_blk;
    // FORCE: the force flags of the two source nodes for the next plane
    // fetched, loaded one fetch ahead (before that fetch's moments, so that
    // waiting for them never waits for the moments in flight).
    uint8_t nfo = 1, nfr = 1;
    auto load_flags = [&](int p) {
        if (!FORCE) return;
        const int64_t zb = (int64_t)zwrap(p) * fgxy;
        if (!SR || interior || has_ring) nfo = fdirty[zb + node_blk];
        if (!SR && has_ring) nfr = fdirty[zb + ring_blk];
    };
    // Planes are fetched in increasing order up to z_end + 1.
    auto fetch = [&](int p, PlaneRegs &r) {
        const bool fo = !FORCE || nfo != 0, fr = !FORCE || nfr != 0;
        if (p + 1 <= z_end + 1) load_flags(p + 1);
        const __amdgpu_buffer_rsrc_t rs = plane_buf(in + (int64_t)zwrap(p) * plane, plane);
        if (!SR || interior || has_ring) {
#pragma unroll
            for (int k = 0; k < 11; ++k) r.own.v[k] = buf_load<R>(rs, node_vo, k * FB);
        }
        if (!SR && has_ring) {
#pragma unroll
            for (int k = 0; k < 11; ++k) r.ring.v[k] = buf_load<R>(rs, ring_vo, k * FB);
        }
        if (!COLL && has_outer) {
            r.outer_dr = buf_load<R>(rs, outer_vo, 0);
            r.outer_r1 = buf_load<R>(rs, outer_vo, FB);
        }
        if (VEC3) {
            const int64_t zl = (int64_t)zwrap(p) * plane_lin;
            const __amdgpu_buffer_rsrc_t fx = plane_buf(frc + zl, plane_lin);
            const __amdgpu_buffer_rsrc_t fy = plane_buf(frc + g.N + zl, plane_lin);
            const __amdgpu_buffer_rsrc_t fz = plane_buf(frc + 2 * g.N + zl, plane_lin);
            if (!SR || interior || has_ring) {
                if (fo) {
                    r.fox = buf_load<R>(fx, node_lvo, 0);
                    r.foy = buf_load<R>(fy, node_lvo, 0);
                    r.foz = buf_load<R>(fz, node_lvo, 0);
                } else {
                    r.fox = r.foy = r.foz = R(0);
                }
            }
            if (!SR && has_ring) {
                if (fr) {
                    r.frx = buf_load<R>(fx, ring_lvo, 0);
                    r.fry = buf_load<R>(fy, ring_lvo, 0);
                    r.frz = buf_load<R>(fz, ring_lvo, 0);
                } else {
                    r.frx = r.fry = r.frz = R(0);
                }
            }
        }
    };
    auto phi_of = [](R dr, R r1) { return phase_field<R>(dr, r1); };
    auto slot_of = [&](int p) { return (p - z0 + 2) % 3; };
    auto write_phi = [&](int p, const PlaneRegs &r) {
        if (COLL) return;
        R *ph = lds_phi + slot_of(p) * FN;
        if constexpr (SR) {
            if (interior || has_ring) ph[interior ? k_own : k_ring] = phi_of(r.own.v[0], r.own.v[1]);
        } else {
            ph[k_own] = phi_of(r.own.v[0], r.own.v[1]);
            if (has_ring) ph[k_ring] = phi_of(r.ring.v[0], r.ring.v[1]);
        }
        if (has_outer) ph[ko] = phi_of(r.outer_dr, r.outer_r1);
    };

    CgAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();

    // Post-collision state of one source node (region slot h): the collided
    // moments with the perturbation, the interface normal n = G/D, rho1/rho
    // and the recolouring amplitude beta rho1 rho2/rho.
    struct NodePrep {
        Collided<R> c;
        R nx, ny, nz, a, B;
    };
    auto prep = [&](int p, const M11 &v, int h, R fx, R fy, R fz) -> NodePrep {
        if constexpr (COLL) {
            // Stored post-collision moments and normal (fx, fy, fz = n).
            NodePrep o;
            o.c = collided_from<R>(v.v[0], v.v[2], v.v[3], v.v[4], v.v[5], v.v[6], v.v[7], v.v[8], v.v[9], v.v[10]);
            o.nx = fx;
            o.ny = fy;
            o.nz = fz;
            const R dr = v.v[0], r1 = v.v[1];
            const R inv_rho = reciprocal<R>(R(1) + dr);
            o.a = r1 * inv_rho;
            o.B = beta * (o.a * (R(1) + dr - r1));
            return o;
        }
        const int kc = src_to_phi(h);
        const R *phm = lds_phi + slot_of(p - 1) * FN;
        const R *ph0 = lds_phi + slot_of(p) * FN;
        const R *php = lds_phi + slot_of(p + 1) * FN;
        R G[3];
        colour_gradient<Q, R>(
            [&](int cx, int cy, int cz) { return (cz < 0 ? phm : (cz == 0 ? ph0 : php))[kc + cy * FX + cx]; }, G);
        const CgCollided<R> cc = cg_collide<R, FORCE>(v.v, G, omega, A9, fx, fy, fz);
        NodePrep o;
        o.c = cc.c;
        o.nx = cc.nx;
        o.ny = cc.ny;
        o.nz = cc.nz;
        const R dr = v.v[0], r1 = v.v[1];
        const R inv_rho = reciprocal<R>(R(1) + dr);
        o.a = r1 * inv_rho;                             // rho1/rho
        o.B = beta * (o.a * (R(1) + dr - r1));          // beta rho1 rho2/rho
        return o;
    };

    // c.n for a direction given at compile time, from the in-plane sums
    // n_a +- n_b (formed once per node); the same expression for a direction
    // wherever the node sits in the tile, so results do not depend on the
    // tiling.
    struct NSums {
        R nx, ny, nz, sxy, dxy, sxz, dxz, syz, dyz;
    };
    auto nsums = [](const NodePrep &o) {
        return NSums{o.nx, o.ny, o.nz, o.nx + o.ny, o.nx - o.ny, o.nx + o.nz, o.nx - o.nz, o.ny + o.nz, o.ny - o.nz};
    };
    auto c_dot_n = [](const NSums &n, int cx, int cy, int cz) -> R {
        const int cls = cx * cx + cy * cy + cz * cz;
        if (cls == 1) return cx ? (cx > 0 ? n.nx : -n.nx) : cy ? (cy > 0 ? n.ny : -n.ny) : (cz > 0 ? n.nz : -n.nz);
        if (cls == 2) {
            if (cz == 0) return cx == cy ? (cx > 0 ? n.sxy : -n.sxy) : (cx > 0 ? n.dxy : -n.dxy);
            if (cy == 0) return cx == cz ? (cx > 0 ? n.sxz : -n.sxz) : (cx > 0 ? n.dxz : -n.dxz);
            return cy == cz ? (cy > 0 ? n.syz : -n.syz) : (cy > 0 ? n.dyz : -n.dyz);
        }
        const R t = cy == cx ? n.sxy : n.dxy;  // cx nx + cy ny, up to the sign of cx
        const R txy = cx > 0 ? t : -t;
        return cz > 0 ? txy + n.nz : txy - n.nz;
    };
    // f1_i = (rho1/rho) (w_i + h~_i) + B w_i (c_i.n)/|c_i|, written as
    // fma(B w_i/|c_i|, c_i.n, fma(rho1/rho, h~_i, (rho1/rho) w_i)) with the
    // per-class products formed once.
    struct F1Coef {
        R a, aw[3], bw[3];
    };
    auto f1coef = [](const NodePrep &o) {
        constexpr double wf = weight<Q>(1, 0, 0), we = weight<Q>(1, 1, 0), wc = weight<Q>(1, 1, 1);
        return F1Coef{o.a,
                      {o.a * R(wf), o.a * R(we), o.a * R(wc)},
                      {o.B * R(wf), o.B * R(we * inv_speed<Q>(1, 1, 0)), o.B * R(wc * inv_speed<Q>(1, 1, 1))}};
    };

    // Interior node: publishes h~ and f1 of every moving direction (the own
    // column (0, 0, +-1) and the rest population stay in registers).
    auto publish = [&](int p, const M11 &v, int h, R *own_h, R *own_f, R fx, R fy, R fz) {
        const NodePrep o = prep(p, v, h, fx, fy, fz);
        Layer<R> L[3];
        reconstruct_layer<Q, -1, R>(o.c, L[0]);
        reconstruct_layer<Q, 0, R>(o.c, L[1]);
        reconstruct_layer<Q, 1, R>(o.c, L[2]);
        const NSums ns = nsums(o);
        const F1Coef k = f1coef(o);
        // Moving directions; the rest population takes what is left of rho1,
        // so that each node emits exactly its species-1 mass (the identity
        // sum_i f1_i = rho1 holds in exact arithmetic: the weights sum to one
        // and the recolouring terms cancel in +-c pairs).
        // One velocity layer at a time with cz a compile-time constant, so
        // that every index below is static (a loop over cz is not always
        // unrolled for D3Q27, and its arrays then go to scratch memory).
        R f1_moving = R(0);
        auto layer = [&](auto czc) {
            constexpr int cz = decltype(czc)::value;
#pragma unroll
            for (int sl = 0; sl < 9; ++sl) {
                const int cx = sl % 3 - 1, cy = sl / 3 - 1;
                if (!has_dir<Q>(cx, cy, cz) || (cx == 0 && cy == 0 && cz == 0)) continue;
                const R hv = L[cz + 1].v[sl];
                const int cls = cx * cx + cy * cy + cz * cz;
                const R f1 = fma_(k.bw[cls - 1], c_dot_n(ns, cx, cy, cz), fma_(k.a, hv, k.aw[cls - 1]));
                f1_moving += f1;
                const int s = lds_slot<Q>(cz, sl);
                if (s >= 0) {
                    lds_hf[lds_at(s, ba0, bb0)] = HF{hv, f1};
                } else {  // own column (0, 0, +-1)
                    own_h[cz + 1] = hv;
                    own_f[cz + 1] = f1;
                }
            }
        };
        layer(std::integral_constant<int, -1>());
        layer(std::integral_constant<int, 0>());
        layer(std::integral_constant<int, 1>());
        own_h[1] = L[1].v[4];
        own_f[1] = v.v[1] - f1_moving;
    };

    // Ring node with inward sign D across a ring row (ROW: directions
    // (t, D, cz)) or a ring column (directions (D, t, cz)): publishes only
    // those, with the interior's arithmetic for each direction.
    auto publish_ring = [&](auto rowc, auto dc, int p, const M11 &v, int h, R fx, R fy, R fz) {
        constexpr bool ROW = decltype(rowc)::value;
        constexpr int D = decltype(dc)::value;
        const NodePrep o = prep(p, v, h, fx, fy, fz);
        Layer<R> L[3];
        reconstruct_layer<Q, -1, R>(o.c, L[0]);
        reconstruct_layer<Q, 0, R>(o.c, L[1]);
        reconstruct_layer<Q, 1, R>(o.c, L[2]);
        const NSums ns = nsums(o);
        const F1Coef k = f1coef(o);
        auto layer = [&](auto czc) {  // cz static, as in publish()
            constexpr int cz = decltype(czc)::value;
#pragma unroll
            for (int t = -1; t <= 1; ++t) {
                const int cx = ROW ? t : D, cy = ROW ? D : t;
                if (!has_dir<Q>(cx, cy, cz)) continue;
                const int sl = (cx + 1) + 3 * (cy + 1);
                const int cls = cx * cx + cy * cy + cz * cz;
                const R hv = L[cz + 1].v[sl];
                const R f1 = fma_(k.bw[cls - 1], c_dot_n(ns, cx, cy, cz), fma_(k.a, hv, k.aw[cls - 1]));
                const int s = lds_slot<Q>(cz, sl);
                // A corner of a ring column lies outside the regions of the
                // directions that leave it beside the tile; it skips them.
                if (!ROW && !(t == 0 ? (ring_y >= 0 && ring_y < TY) : (t > 0 ? ring_y < TY : ring_y >= 0)))
                    continue;
                lds_hf[lds_at(s, bar, bbr)] = HF{hv, f1};
            }
        };
        layer(std::integral_constant<int, -1>());
        layer(std::integral_constant<int, 0>());
        layer(std::integral_constant<int, 1>());
    };
    using Up = std::integral_constant<int, 1>;
    using Down = std::integral_constant<int, -1>;

    auto pull_layer = [&](auto czc, CgAcc<R> &ac, R oh, R of) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> fh;
        R r1 = of;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            if (sl == 4) {
                fh.v[sl] = oh;
            } else if (lds_slot<Q>(CZ, sl) >= 0) {
                const int s = lds_slot<Q>(CZ, sl);
                const int idx = lds_at(s, ba0, bb0) - cy * SL::width(s) - cx;
                const HF v = lds_hf[idx];
                fh.v[sl] = v.h;
                r1 += v.f;
            }
        }
        accumulate_layer<Q, CZ, R>(ac.m, fh);
        ac.rho1 += r1;
    };

    auto plane_step = [&](int p, PlaneRegs &cur, PlaneRegs &nxt) {
        write_phi(p + 1, nxt);
        __syncthreads();
        R oh[3], of[3];
        if (interior) publish(p, cur.own, h0, oh, of, cur.fox, cur.foy, cur.foz);
        const M11 &rv = SR ? cur.own : cur.ring;
        const R rfx = SR ? cur.fox : cur.frx, rfy = SR ? cur.foy : cur.fry, rfz = SR ? cur.foz : cur.frz;
        if (ring_row) {
            if (dsign > 0) publish_ring(std::true_type(), Up(), p, rv, hr, rfx, rfy, rfz);
            else publish_ring(std::true_type(), Down(), p, rv, hr, rfx, rfy, rfz);
        } else if (ring_col) {
            if (dsign > 0) publish_ring(std::false_type(), Up(), p, rv, hr, rfx, rfy, rfz);
            else publish_ring(std::false_type(), Down(), p, rv, hr, rfx, rfy, rfz);
        }
        __syncthreads();
        if (p + 2 <= z_end + 1) fetch(p + 2, cur);
        if (interior) {
            pull_layer(std::integral_constant<int, -1>(), acc[0], oh[0], of[0]);
            pull_layer(std::integral_constant<int, 0>(), acc[1], oh[1], of[1]);
            pull_layer(std::integral_constant<int, 1>(), acc[2], oh[2], of[2]);
        }

        const int d = p - 1;
        if (d >= z0 && active) {
            const __amdgpu_buffer_rsrc_t ws = plane_buf(out + (int64_t)d * plane, plane);
            const MomentAcc<R> &a = acc[0].m;
            const R m3 = R(-1.0 / 3.0);
            buf_store<R>(ws, dst_vo, 0, a.r);
            buf_store<R>(ws, dst_vo, FB, acc[0].rho1);
            buf_store<R>(ws, dst_vo, 2 * FB, a.jx);
            buf_store<R>(ws, dst_vo, 3 * FB, a.jy);
            buf_store<R>(ws, dst_vo, 4 * FB, a.jz);
            buf_store<R>(ws, dst_vo, 5 * FB, fma_(m3, a.r, a.mxx));
            buf_store<R>(ws, dst_vo, 6 * FB, fma_(m3, a.r, a.myy));
            buf_store<R>(ws, dst_vo, 7 * FB, fma_(m3, a.r, a.mzz));
            buf_store<R>(ws, dst_vo, 8 * FB, a.mxy);
            buf_store<R>(ws, dst_vo, 9 * FB, a.mxz);
            buf_store<R>(ws, dst_vo, 10 * FB, a.myz);
            if (FORCE)
                buf_store<R>(plane_buf(phi_out + (int64_t)d * plane_lin, plane_lin), dst_lvo, 0,
                             phi_of(a.r, acc[0].rho1));
        }
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    };

    // Prologue: phase field of planes z0-2 and z0-1, moments of z0-1 and z0.
    load_flags(z0 - 2);
    fetch(z0 - 2, pa);
    write_phi(z0 - 2, pa);
    fetch(z0 - 1, pa);
    fetch(z0, pb);
    write_phi(z0 - 1, pa);
    for (int p = z0 - 1; p <= z_end; p += 2) {
        plane_step(p, pa, pb);
        if (p + 1 <= z_end) plane_step(p + 1, pb, pa);
    }
}

// Chunk length along z for `tiles` tiles on `slots` resident workgroups: the
// number of chunks (1 to 8) that minimises rounds x (planes per chunk + the
// two planes each chunk starts with), rounds = ceil(tiles x chunks / slots).
inline int balanced_zchunk(int nz, int tiles, int slots)
{
    int best = nz, best_cost = 0;
    for (int ch = 1; ch <= 8; ++ch) {
        const int zc = (nz + ch - 1) / ch;
        if (ch > 1 && zc < 16) break;
        const int64_t rounds = ((int64_t)tiles * ((nz + zc - 1) / zc) + slots - 1) / slots;
        const int64_t cost = rounds * (zc + 2);
        if (ch == 1 || cost < best_cost) {
            best = zc;
            best_cost = (int)cost;
        }
    }
    return best;
}

// Resident workgroups per CU each variant is sized for: WG for the plain
// step, WGF for the step with the near-contact force, WGC for the streaming
// pass of the split schedule.
// Launch shape of one variant of the step: TY tile rows, WG resident
// workgroups per CU the z-chunks (and the register allocation) are sized for,
// SR separate ring threads.
template <int TY_, int WG_, bool SR_>
struct CgShape {
    static constexpr int TY = TY_, WG = WG_;
    static constexpr bool SR = SR_;
};

template <int Q, class R, int TX, class SH, bool FORCE, bool COLL>
hipError_t launch_tile(const lbm_ctx *c, const void *in, void *out, const R *frc, R *phi_out,
                       const uint8_t *fdirty = nullptr)
{
    constexpr int TY = SH::TY, NTH = kCgThreads<TX, TY, SH::SR>;
    // Waves per SIMD the register allocation must leave room for.
    constexpr int WPE = (NTH / 64 * SH::WG + 3) / 4;
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.lay = c->lay;
    g.tiles_x = (c->nx + TX - 1) / TX;
    g.tiles_y = (c->ny + TY - 1) / TY;
    g.zchunk = balanced_zchunk(c->nz, g.tiles_x * g.tiles_y, 256 * SH::WG);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_cg_tile<Q, R, TX, TY, FORCE, WPE, COLL, SH::SR>), dim3((unsigned)blocks), dim3(NTH), 0,
                       c->stream, static_cast<const R *>(in), static_cast<R *>(out), g, (R)c->omega,
                       (R)(c->A / 9.0), (R)c->beta, frc, phi_out, fdirty);
    return hipGetLastError();
}

// P, F, C: shapes of the plain step, the step with the near-contact force and
// the streaming pass of the split schedule.
template <int Q, class R, int TX, class P, class F, class C>
hipError_t run(const lbm_ctx *c, const void *in, void *out, bool phi_cached, const void *normal = nullptr)
{
    if (normal)  // streaming pass of the split schedule
        return launch_tile<Q, R, TX, C, false, true>(c, in, out, static_cast<const R *>(normal), nullptr);
    if (c->nc_A != 0.0) {
        // Near-contact force of this state first (into the context's scratch:
        // F, then the phase field, reused when the previous step wrote it).
        R *phi = static_cast<R *>(c->scratch_nc) + 3 * c->N;
        hipError_t e = phi_cached ? launch_nc_force(c, nullptr, phi) : launch_nc_force(c, in, nullptr);
        if (e != hipSuccess) return e;
        return launch_tile<Q, R, TX, F, true, false>(c, in, out, static_cast<const R *>(c->scratch_nc), phi,
                                                     nc_block_flags(c) + nc_blocks(c));
    }
    return launch_tile<Q, R, TX, P, false, false>(c, in, out, nullptr, nullptr);
}

} // namespace

// D3Q19 FP32 tiles: 64 x 4 nodes (full 64-wide rows of the stored blocks).
// The plain step gives the halo ring threads of their own (448 threads, 7
// waves, each thread one node, so every wave collides one node per plane; 128
// VGPRs without spills) and is sized for two resident workgroups per CU (14
// waves; on 512 x 256 x 256 each marches a whole column): 0.725 -> 0.686 ms
// per step against 256 threads that collide an interior and a ring node each
// at three workgroups per CU.  The step with the near-contact force (176
// VGPRs; 128 would spill) and the streaming pass of the split schedule
// (slower with ring threads) keep 256 threads at two workgroups per CU.
// 64 x 8 tiles with ring threads (11 waves, one workgroup per CU) ran 7 %
// slower for the plain step and 6 % for the force variant on 512 x 256 x 256
// (4 % faster for the latter on 128^3).  Also measured against 32 x 8, 32 x 16
// and 128 x 4 tiles and other chunkings; each shape is a compile-time choice
// (LBM_CG_P, LBM_CG_F, LBM_CG_C: tile rows, workgroups per CU, ring threads).
#ifndef LBM_CG_P
#define LBM_CG_P 4, 2, true
#endif
#ifndef LBM_CG_F
#define LBM_CG_F 4, 2, false
#endif
#ifndef LBM_CG_C
#define LBM_CG_C 4, 2, false
#endif

hipError_t launch_cg_step(const lbm_ctx *c, const void *in, void *out, bool phi_cached, const void *normal)
{
    if (c->species != 2) return hipErrorNotSupported;
    using S2 = CgShape<4, 2, false>;
    using S8 = CgShape<8, 2, false>;
#ifndef LBM_CG_Q27P
#define LBM_CG_Q27P 8, 2, false
#endif
    if (c->storage == LBM_STORE_F32)
        return c->q == 19 ? run<19, float, 64, CgShape<LBM_CG_P>, CgShape<LBM_CG_F>, CgShape<LBM_CG_C>>(
                                c, in, out, phi_cached, normal)
                          : run<27, float, 32, CgShape<LBM_CG_Q27P>, S8, S8>(c, in, out, phi_cached, normal);
    if (c->storage == LBM_STORE_F64)
        return c->q == 19 ? run<19, double, 32, S2, S2, S2>(c, in, out, phi_cached, normal)
                          : run<27, double, 32, S2, S2, S2>(c, in, out, phi_cached, normal);
    return hipErrorInvalidValue;
}

} // namespace lbm
