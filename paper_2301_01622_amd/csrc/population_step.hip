// Population-storing BGK step (the comparison scheme, one species).
//
// State: the q post-collision populations of every node, shifted by their
// rest value (f~_i = f_i - w_i), one array per direction.  Pull scheme with
// two buffers: the thread of node x gathers f~_i(x - c_i), takes the moments
// (Eqs. 1-3), relaxes towards the equilibrium of Eq. 5 with Eq. 7, and
// writes its q post-collision populations to the other buffer.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {
namespace {

template <int Q, class S>
__global__ __launch_bounds__(256) void k_population_pull(const S *__restrict__ in, S *__restrict__ out, int nx,
                                                         int ny, int nz, int64_t N, typename Store<S>::real omega)
{
    using R = typename Store<S>::real;
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);

    R f[Q];
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
        f[i] = Store<S>::load(in[(int64_t)i * N + s]);
        accumulate<Q, R>(a, f[i], i);
    }
    // Equilibrium (Eq. 5) in shifted form: reconstruction of S = j j / rho.
    const R inv_rho = reciprocal<R>(R(1) + a.r);
    Collided<R> eq;
    eq.jx = a.jx;
    eq.jy = a.jy;
    eq.jz = a.jz;
    eq.sxx = a.jx * a.jx * inv_rho;
    eq.syy = a.jy * a.jy * inv_rho;
    eq.szz = a.jz * a.jz * inv_rho;
    eq.sxy = a.jx * a.jy * inv_rho;
    eq.sxz = a.jx * a.jz * inv_rho;
    eq.syz = a.jy * a.jz * inv_rho;
    eq.T = a.r - R(1.5) * (eq.sxx + eq.syy + eq.szz);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R feq = reconstruct<Q, R>(eq, i);
        out[(int64_t)i * N + n] = Store<S>::make(fma_(omega, feq - f[i], f[i]));
    }
}

template <int Q, class S>
hipError_t run(const lbm_ctx *c, const void *in, void *out)
{
    using R = typename Store<S>::real;
    const int64_t blocks = (c->N + 255) / 256;
    hipLaunchKernelGGL((k_population_pull<Q, S>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                       static_cast<const S *>(in), static_cast<S *>(out), c->nx, c->ny, c->nz, c->N, (R)c->omega);
    return hipGetLastError();
}

} // namespace

hipError_t launch_population_step(const lbm_ctx *c, const void *in, void *out)
{
    if (c->species != 1) return hipErrorNotSupported;
    if (c->storage == LBM_STORE_F64) return c->q == 19 ? run<19, double>(c, in, out) : run<27, double>(c, in, out);
    if (c->storage == LBM_STORE_F32) return c->q == 19 ? run<19, float>(c, in, out) : run<27, float>(c, in, out);
    return hipErrorInvalidValue;
}

} // namespace lbm
