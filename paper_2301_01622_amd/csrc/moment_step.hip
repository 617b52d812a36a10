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
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {
namespace {

constexpr int kXcds = 8;

struct TileGrid {
    int nx, ny, nz;
    int64_t N;
    int tiles_x, tiles_y, chunks, zchunk;
};

// Moments of one source node, already unpacked to the arithmetic type.
template <class R>
struct Moments {
    R v[10];
};

template <class S>
__device__ __forceinline__ void load_moments(const S *__restrict__ in, int64_t N, int64_t idx,
                                             Moments<typename Store<S>::real> &m)
{
#pragma unroll
    for (int k = 0; k < 10; ++k) m.v[k] = Store<S>::load(in[k * N + idx]);
}

template <int Q, class S, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_moment_tile(const S *__restrict__ in, S *__restrict__ out, TileGrid g,
                                                        typename Store<S>::real omega,
                                                        typename Store<S>::real s_pi,
                                                        typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    using L = Lattice<Q>;
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int NSRC = (HN + NT - 1) / NT;  // source nodes per thread
    __shared__ R lds[Q * HN];

    // XCD-aware tile numbering (falls back to the identity when the grid
    // does not split evenly over the XCDs).
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if (nb % kXcds == 0) b = (b % kXcds) * (nb / kXcds) + b / kXcds;
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
    const int h0 = (ly + 1) * HX + (lx + 1);  // this thread's interior slot

    // xy offsets of this thread's source nodes (periodic wrap done once).
    int64_t src_xy[NSRC];
    bool src_ok[NSRC];
#pragma unroll
    for (int k = 0; k < NSRC; ++k) {
        const int h = tid + k * NT;
        src_ok[k] = h < HN;
        const int hx = h % HX, hy = h / HX;
        int gx = (x0 - 1 + hx) % g.nx, gy = (y0 - 1 + hy) % g.ny;
        gx += gx < 0 ? g.nx : 0;
        gy += gy < 0 ? g.ny : 0;
        src_xy[k] = (int64_t)gx + (int64_t)g.nx * gy;
    }

    MomentAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();

    Moments<R> m[NSRC];
    auto fetch = [&](int p) {
        int zs = p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p);
#pragma unroll
        for (int k = 0; k < NSRC; ++k)
            if (src_ok[k]) load_moments<S>(in, g.N, src_xy[k] + (int64_t)zs * plane, m[k]);
    };

    fetch(z0 - 1);
    for (int p = z0 - 1; p <= z_end; ++p) {
        // Collide each source node once and publish its populations.
#pragma unroll
        for (int k = 0; k < NSRC; ++k) {
            if (!src_ok[k]) continue;
            const Moments<R> &v = m[k];
            const Collided<R> c = collide<R>(v.v[0], v.v[1], v.v[2], v.v[3], v.v[4] * inv_s_pi, v.v[5] * inv_s_pi,
                                             v.v[6] * inv_s_pi, v.v[7] * inv_s_pi, v.v[8] * inv_s_pi,
                                             v.v[9] * inv_s_pi, omega);
            const int h = tid + k * NT;
#pragma unroll
            for (int i = 0; i < Q; ++i) lds[i * HN + h] = reconstruct<Q, R>(c, i);
        }
        __syncthreads();
        if (p < z_end) fetch(p + 1);

        // Pull: direction i arrives from (x - c_i); cz selects the plane.
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R h = lds[i * HN + h0 - L::cy(i) * HX - L::cx(i)];
            accumulate<Q, R>(acc[L::cz(i) + 1], h, i);
        }
        __syncthreads();

        // Plane p-1 has now received from p-2, p-1 and p.
        const int d = p - 1;
        if (d >= z0 && active) {
            const int64_t o = (int64_t)(x0 + lx) + (int64_t)g.nx * (y0 + ly) + (int64_t)d * plane;
            const MomentAcc<R> &a = acc[0];
            const R third = a.r * R(1.0 / 3.0);
            out[o] = Store<S>::make(a.r);
            out[g.N + o] = Store<S>::make(a.jx);
            out[2 * g.N + o] = Store<S>::make(a.jy);
            out[3 * g.N + o] = Store<S>::make(a.jz);
            out[4 * g.N + o] = Store<S>::make((a.mxx - third) * s_pi);
            out[5 * g.N + o] = Store<S>::make((a.myy - third) * s_pi);
            out[6 * g.N + o] = Store<S>::make((a.mzz - third) * s_pi);
            out[7 * g.N + o] = Store<S>::make(a.mxy * s_pi);
            out[8 * g.N + o] = Store<S>::make(a.mxz * s_pi);
            out[9 * g.N + o] = Store<S>::make(a.myz * s_pi);
        }
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    }
}

// Chunk length along z: aim for about four resident waves of workgroups on
// 256 CUs while keeping the two recomputed halo planes a small fraction.
inline int choose_zchunk(int nz, int tiles_xy)
{
    const int target_blocks = 2048;
    int chunks = (target_blocks + tiles_xy - 1) / tiles_xy;
    if (chunks < 1) chunks = 1;
    int zc = (nz + chunks - 1) / chunks;
    if (zc < 16) zc = 16;
    if (zc > nz) zc = nz;
    return zc;
}

template <int Q, class S, int TX, int TY>
hipError_t run(const lbm_ctx *c, const void *in, void *out)
{
    using R = typename Store<S>::real;
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.tiles_x = (c->nx + TX - 1) / TX;
    g.tiles_y = (c->ny + TY - 1) / TY;
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_moment_tile<Q, S, TX, TY>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                       static_cast<const S *>(in), static_cast<S *>(out), g, (R)c->omega, (R)c->s_pi,
                       (R)(1.0 / c->s_pi));
    return hipGetLastError();
}

template <int Q>
hipError_t dispatch_storage(const lbm_ctx *c, const void *in, void *out)
{
    switch (c->storage) {
    case LBM_STORE_F64: return run<Q, double, 32, 8>(c, in, out);
    case LBM_STORE_F32: return run<Q, float, 32, 16>(c, in, out);
    case LBM_STORE_F16: return run<Q, f16, 32, 16>(c, in, out);
    case LBM_STORE_BF16: return run<Q, bf16, 32, 16>(c, in, out);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_moment_step(const lbm_ctx *c, const void *in, void *out)
{
    if (c->species != 1) return hipErrorNotSupported;
    return c->q == 19 ? dispatch_storage<19>(c, in, out) : dispatch_storage<27>(c, in, out);
}

} // namespace lbm
