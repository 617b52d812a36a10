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
