// Fused moment-only time step (one species).
//
// One thread per destination node x.  For each direction i it reads the
// stored moments of the source node y = x - c_i, collides them (Eqs. 7-8 in
// moment form), rebuilds the single population h'_i(y) that travels to x
// (Eqs. 4-6), and accumulates the moments of the streamed set (Eq. 9, then
// Eqs. 1-3).  The result goes to the other copy of the arrays.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {
namespace {

template <int Q, class S>
__global__ __launch_bounds__(256) void k_moment_gather(const S *__restrict__ in, S *__restrict__ out, int nx,
                                                       int ny, int nz, int64_t N,
                                                       typename Store<S>::real omega,
                                                       typename Store<S>::real s_pi,
                                                       typename Store<S>::real inv_s_pi)
{
    using R = typename Store<S>::real;
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);

    MomentAcc<R> a;
    a.zero();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int xs = x - L::cx(i), ys = y - L::cy(i), zs = z - L::cz(i);
        xs += xs < 0 ? nx : 0;
        xs -= xs >= nx ? nx : 0;
        ys += ys < 0 ? ny : 0;
        ys -= ys >= ny ? ny : 0;
        zs += zs < 0 ? nz : 0;
        zs -= zs >= nz ? nz : 0;
        const int64_t s = (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
        const Collided<R> p =
            collide<R>(Store<S>::load(in[s]), Store<S>::load(in[N + s]), Store<S>::load(in[2 * N + s]),
                       Store<S>::load(in[3 * N + s]), Store<S>::load(in[4 * N + s]) * inv_s_pi,
                       Store<S>::load(in[5 * N + s]) * inv_s_pi, Store<S>::load(in[6 * N + s]) * inv_s_pi,
                       Store<S>::load(in[7 * N + s]) * inv_s_pi, Store<S>::load(in[8 * N + s]) * inv_s_pi,
                       Store<S>::load(in[9 * N + s]) * inv_s_pi, omega);
        accumulate<Q, R>(a, reconstruct<Q, R>(p, i), i);
    }
    const R third = a.r * R(1.0 / 3.0);
    out[n] = Store<S>::make(a.r);
    out[N + n] = Store<S>::make(a.jx);
    out[2 * N + n] = Store<S>::make(a.jy);
    out[3 * N + n] = Store<S>::make(a.jz);
    out[4 * N + n] = Store<S>::make((a.mxx - third) * s_pi);
    out[5 * N + n] = Store<S>::make((a.myy - third) * s_pi);
    out[6 * N + n] = Store<S>::make((a.mzz - third) * s_pi);
    out[7 * N + n] = Store<S>::make(a.mxy * s_pi);
    out[8 * N + n] = Store<S>::make(a.mxz * s_pi);
    out[9 * N + n] = Store<S>::make(a.myz * s_pi);
}

template <int Q, class S>
hipError_t run(const lbm_ctx *c, const void *in, void *out)
{
    using R = typename Store<S>::real;
    const int64_t blocks = (c->N + 255) / 256;
    hipLaunchKernelGGL((k_moment_gather<Q, S>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                       static_cast<const S *>(in), static_cast<S *>(out), c->nx, c->ny, c->nz, c->N,
                       (R)c->omega, (R)c->s_pi, (R)(1.0 / c->s_pi));
    return hipGetLastError();
}

template <int Q>
hipError_t dispatch_storage(const lbm_ctx *c, const void *in, void *out)
{
    switch (c->storage) {
    case LBM_STORE_F64: return run<Q, double>(c, in, out);
    case LBM_STORE_F32: return run<Q, float>(c, in, out);
    case LBM_STORE_F16: return run<Q, f16>(c, in, out);
    case LBM_STORE_BF16: return run<Q, bf16>(c, in, out);
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
