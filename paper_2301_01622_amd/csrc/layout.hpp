// Stored layout of the moment-scheme state.
//
// The public layout (one array per field, x fastest) is only an interface
// format.  Inside the library the nf stored fields of each 64 x 16 block of
// an xy-plane are one contiguous run of nf x 1024 elements (field-major
// within the block, then 16 rows of 64 nodes), blocks follow each other
// along x, then y, then z:
//
//   offset(x, y, z, k) = z * plane + ((y / 16) * nbx + x / 64) * nf * 1024
//                        + k * 1024 + (y % 16) * 64 + x % 64,
//   nbx = ceil(nx / 64), nby = ceil(ny / 16), plane = nbx * nby * nf * 1024.
//
// A workgroup marching a tile along z then reads and writes one contiguous
// block per field set and plane instead of nf separate strided rows, which
// the memory system serves at a markedly higher rate.  Grids whose nx or ny
// is not a multiple of 64 or 16 leave unused slots at the block edges; no
// kernel reads them as nodes, and they are zeroed when the state is created.
#pragma once

#include <stdint.h>

namespace lbm {

constexpr int kBX = 64, kBY = 16, kBlock = kBX * kBY;

struct MomentLayout {
    int nbx;        // blocks along x
    int nf;         // stored fields
    int64_t plane;  // elements per z-plane (all fields)

    // Offset of field 0 of node (x, y) inside a z-plane; field k adds k * kBlock.
    __host__ __device__ int64_t xy(int x, int y) const
    {
        return ((int64_t)(y / kBY) * nbx + x / kBX) * ((int64_t)nf * kBlock) + (y % kBY) * kBX + x % kBX;
    }
    __host__ __device__ int64_t node(int x, int y, int z) const { return (int64_t)z * plane + xy(x, y); }
};

inline MomentLayout moment_layout(int nx, int ny, int nf)
{
    MomentLayout L;
    L.nbx = (nx + kBX - 1) / kBX;
    L.nf = nf;
    const int nby = (ny + kBY - 1) / kBY;
    L.plane = (int64_t)L.nbx * nby * nf * kBlock;
    return L;
}

} // namespace lbm
