// Pieces shared by the tiled step kernels: tile geometry, XCD-aware tile
// numbering, z-chunk sizing, nontemporal stores and the LDS slot map.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"
#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {

constexpr int kXcds = 8;

struct TileGrid {
    int nx, ny, nz;
    int64_t N;
    int tiles_x, tiles_y, chunks, zchunk;
    MomentLayout lay;  // stored layout of the moment state
};

// Moments of one source node, already unpacked to the arithmetic type.
// load_moments reads field k at in[k * stride + idx] (stride kBlock for the
// stored moment state, N for arrays in the public layout).
template <class R, int NF = 10>
struct Moments {
    R v[NF];
};

template <class S, int NF>
__device__ __forceinline__ void load_moments(const S *__restrict__ in, int64_t N, int64_t idx,
                                             Moments<typename Store<S>::real, NF> &m)
{
#pragma unroll
    for (int k = 0; k < NF; ++k) m.v[k] = Store<S>::load(in[k * N + idx]);
}

// Collision of one node from its stored moments (Eqs. 7-8 in moment form);
// 16-bit storage keeps S * s_pi, undone here.
template <class S>
__device__ __forceinline__ Collided<typename Store<S>::real> collide_stored(const Moments<typename Store<S>::real> &v,
                                                                            typename Store<S>::real omega,
                                                                            typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    if constexpr (sizeof(S) == 2)
        return collide<R>(v.v[0], v.v[1], v.v[2], v.v[3], v.v[4] * inv_s_pi, v.v[5] * inv_s_pi, v.v[6] * inv_s_pi,
                          v.v[7] * inv_s_pi, v.v[8] * inv_s_pi, v.v[9] * inv_s_pi, omega);
    else
        return collide<R>(v.v[0], v.v[1], v.v[2], v.v[3], v.v[4], v.v[5], v.v[6], v.v[7], v.v[8], v.v[9], omega);
}

// The 10 stored values of a finished accumulator (Eqs. 1-3): deviations
// rho - 1, j and S = P - rho c_s^2 I (times s_pi for 16-bit storage).
template <class S>
__device__ __forceinline__ void stored_moments(const MomentAcc<typename Store<S>::real> &a,
                                               typename Store<S>::real s_pi, S *v)
{
    using R = typename Store<S>::real;
    constexpr bool kScaled = sizeof(S) == 2;
    const R m3 = R(-1.0 / 3.0);
    const R sc = kScaled ? s_pi : R(1);
    v[0] = Store<S>::make(a.r);
    v[1] = Store<S>::make(a.jx);
    v[2] = Store<S>::make(a.jy);
    v[3] = Store<S>::make(a.jz);
    v[4] = Store<S>::make(kScaled ? fma_(m3, a.r, a.mxx) * sc : fma_(m3, a.r, a.mxx));
    v[5] = Store<S>::make(kScaled ? fma_(m3, a.r, a.myy) * sc : fma_(m3, a.r, a.myy));
    v[6] = Store<S>::make(kScaled ? fma_(m3, a.r, a.mzz) * sc : fma_(m3, a.r, a.mzz));
    v[7] = Store<S>::make(kScaled ? a.mxy * sc : a.mxy);
    v[8] = Store<S>::make(kScaled ? a.mxz * sc : a.mxz);
    v[9] = Store<S>::make(kScaled ? a.myz * sc : a.myz);
}

// Workgroup id -> logical tile id.  Workgroups are handed to the 8 XCDs
// round-robin (id mod 8); the remap gives each XCD a contiguous range of
// tiles so that halo re-reads of neighbouring tiles hit the same L2.
__device__ __forceinline__ int xcd_tile_id()
{
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    return nb % kXcds == 0 ? (b % kXcds) * (nb / kXcds) + b / kXcds : b;
}

// Periodic wrap of a coordinate that may be off by any amount.
__device__ __forceinline__ int wrap_coord(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <class S>
__device__ __forceinline__ void store_out(S *p, S v)
{
    __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void store_out<bf16>(bf16 *p, bf16 v)
{
    __builtin_nontemporal_store(v.bits, reinterpret_cast<uint16_t *>(p));
}

// LDS slot of direction (slot, layer CZ), slot = (cx+1) + 3 (cy+1); the
// own-column slot 4 never goes through LDS.  Directions absent from the
// lattice get no slot.  Returns -1 for "no slot".
template <int Q>
__host__ __device__ constexpr int lds_slot(int cz, int slot)
{
    int k = 0;
    for (int z = -1; z <= 1; ++z)
        for (int sl = 0; sl < 9; ++sl) {
            if (sl == 4 || !has_dir<Q>(sl % 3 - 1, sl / 3 - 1, z)) continue;
            if (z == cz && sl == slot) return k;
            ++k;
        }
    return -1;
}
template <int Q>
constexpr int kLdsSlots = Q - 3;

// Chunk length along z.  Each chunk re-reads two halo planes that the
// neighbouring chunk also reads, at another time and usually on another XCD,
// so the re-read costs HBM bandwidth: chunks are made as long as possible
// while still giving about one resident round of workgroups on 256 CUs.
inline int choose_zchunk(int nz, int tiles_xy, int target_blocks)
{
    int chunks = (target_blocks + tiles_xy - 1) / tiles_xy;
    if (chunks < 1) chunks = 1;
    int zc = (nz + chunks - 1) / chunks;
    if (zc < 16) zc = 16;
    if (zc > nz) zc = nz;
    return zc;
}

} // namespace lbm
