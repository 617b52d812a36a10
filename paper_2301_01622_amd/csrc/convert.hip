// Conversions between caller moment buffers and the stored state, and the
// FP64 global totals.
//
// Public layout: field k of a caller buffer starts at base + k*stride; fields
// are (rho | rho1, rho2), jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz.
// Stored moment state: delta_rho, [rho1], j, S * s_pi with S = P - rho/3 I.
// Stored population state (pull scheme): post-collision shifted populations
// f~_i = f_i - w_i, so that the populations arriving at x are f~_i(x - c_i).
// Conversions run in FP64 whatever the storage; only the final store rounds.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {
namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// In-place population scheme after an odd number of steps: arrivals stored
// reversed at their own node.
inline bool aa_odd(const lbm_ctx *c) { return c->scheme == LBM_SCHEME_POPULATION_AA && (c->steps & 1); }

// ---- moment scheme -------------------------------------------------------------

// Stored offset of public node n (x fastest) in the blocked moment layout.
__device__ __forceinline__ int64_t stored_node(const MomentLayout &L, int64_t n, int nx, int ny)
{
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    return L.node(x, (int)(t % ny), (int)(t / ny));
}

template <class S, class T>
__global__ void k_set_moment_state(const T *__restrict__ src, int64_t stride, S *__restrict__ st, int64_t N, int nx,
                                   int ny, MomentLayout lay, int species, double s_pi)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t so = stored_node(lay, n, nx, ny);
    double rho, rho1 = 0.0;
    int off;
    if (species == 1) {
        rho = (double)src[n];
        off = 1;
    } else {
        rho1 = (double)src[n];
        rho = rho1 + (double)src[stride + n];
        off = 2;
    }
    const int js = species == 1 ? 1 : 2;  // first stored j field
    st[so] = Store<S>::make((typename Store<S>::real)(rho - 1.0));
    if (species == 2) st[kBlock + so] = Store<S>::make((typename Store<S>::real)rho1);
    for (int a = 0; a < 3; ++a)
        st[(js + a) * kBlock + so] = Store<S>::make((typename Store<S>::real)src[(off + a) * stride + n]);
    for (int k = 0; k < 6; ++k) {
        double p = (double)src[(off + 3 + k) * stride + n];
        if (k < 3) p -= rho / 3.0;
        st[(js + 3 + k) * kBlock + so] = Store<S>::make((typename Store<S>::real)(p * s_pi));
    }
}

template <class S, class T>
__global__ void k_get_moment_state(const S *__restrict__ st, T *__restrict__ dst, int64_t stride, int64_t N, int nx,
                                   int ny, MomentLayout lay, int species, double inv_s_pi)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t so = stored_node(lay, n, nx, ny);
    const double rho = 1.0 + (double)Store<S>::load(st[so]);
    const int js = species == 1 ? 1 : 2;
    int off;
    if (species == 1) {
        dst[n] = (T)rho;
        off = 1;
    } else {
        const double rho1 = (double)Store<S>::load(st[kBlock + so]);
        dst[n] = (T)rho1;
        dst[stride + n] = (T)(rho - rho1);
        off = 2;
    }
    for (int a = 0; a < 3; ++a) dst[(off + a) * stride + n] = (T)(double)Store<S>::load(st[(js + a) * kBlock + so]);
    for (int k = 0; k < 6; ++k) {
        double p = (double)Store<S>::load(st[(js + 3 + k) * kBlock + so]) * inv_s_pi;
        if (k < 3) p += rho / 3.0;
        dst[(off + 3 + k) * stride + n] = (T)p;
    }
}

// ---- co-states ----------------------------------------------------------------

// Public layout: field k at pub + k*stride (element type P); stored layout:
// the blocked layout of the state with the kernels' real type R.
template <class P, class R>
__global__ void k_costate_convert(const void *__restrict__ src, void *__restrict__ dst, int64_t stride, int64_t N,
                                  int nx, int ny, MomentLayout lay, int nf, bool to_stored)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t so = stored_node(lay, n, nx, ny);
    if (to_stored) {
        const P *s = static_cast<const P *>(src);
        R *d = static_cast<R *>(dst);
        for (int k = 0; k < nf; ++k) d[k * kBlock + so] = (R)s[k * stride + n];
    } else {
        const R *s = static_cast<const R *>(src);
        P *d = static_cast<P *>(dst);
        for (int k = 0; k < nf; ++k) d[k * stride + n] = (P)s[k * kBlock + so];
    }
}

// ---- population scheme -------------------------------------------------------------

// A_i[y] = shifted R(M(y + c_i))_i (Eq. 4 without collision).
template <int Q, class S, class T>
__global__ void k_set_population_state(const T *__restrict__ src, int64_t stride, S *__restrict__ A, int nx,
                                       int ny, int nz, int64_t N)
{
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = (x + L::cx(i) + nx) % nx, ys = (y + L::cy(i) + ny) % ny, zs = (z + L::cz(i) + nz) % nz;
        const int64_t s = (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
        const double rho = (double)src[s];
        Collided<double> p;
        p.jx = (double)src[stride + s];
        p.jy = (double)src[2 * stride + s];
        p.jz = (double)src[3 * stride + s];
        p.sxx = (double)src[4 * stride + s] - rho / 3.0;
        p.syy = (double)src[5 * stride + s] - rho / 3.0;
        p.szz = (double)src[6 * stride + s] - rho / 3.0;
        p.sxy = (double)src[7 * stride + s];
        p.sxz = (double)src[8 * stride + s];
        p.syz = (double)src[9 * stride + s];
        p.T = (rho - 1.0) - 1.5 * (p.sxx + p.syy + p.szz);
        A[(int64_t)i * N + n] = Store<S>::make((typename Store<S>::real)reconstruct<Q, double>(p, i));
    }
}

// Moments of the populations arriving at x: f~_i = A_i[x - c_i], or, for the
// in-place scheme after an odd number of steps (odd), f~_i = A_{-i}[x].
template <int Q, class S, class T>
__global__ void k_get_population_state(const S *__restrict__ A, T *__restrict__ dst, int64_t stride, int nx,
                                       int ny, int nz, int64_t N, bool odd)
{
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    MomentAcc<double> a;
    a.zero();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = (x - L::cx(i) + nx) % nx, ys = (y - L::cy(i) + ny) % ny, zs = (z - L::cz(i) + nz) % nz;
        const int64_t s = (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
        const int64_t at = odd ? (int64_t)opposite<Q>(i) * N + n : (int64_t)i * N + s;
        accumulate<Q, double>(a, (double)Store<S>::load(A[at]), i);
    }
    const double rho = 1.0 + a.r;
    dst[n] = (T)rho;
    dst[stride + n] = (T)a.jx;
    dst[2 * stride + n] = (T)a.jy;
    dst[3 * stride + n] = (T)a.jz;
    dst[4 * stride + n] = (T)(a.mxx + 1.0 / 3.0);
    dst[5 * stride + n] = (T)(a.myy + 1.0 / 3.0);
    dst[6 * stride + n] = (T)(a.mzz + 1.0 / 3.0);
    dst[7 * stride + n] = (T)a.mxy;
    dst[8 * stride + n] = (T)a.mxz;
    dst[9 * stride + n] = (T)a.myz;
}

// Two species: A^k_i[y] = (rho^k/rho)(y + c_i) R(M(y + c_i))_i, unshifted FP32.
template <int Q, class T>
__global__ void k_set_population2_state(const T *__restrict__ src, int64_t stride, float *__restrict__ A, int nx,
                                        int ny, int nz, int64_t N)
{
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = (x + L::cx(i) + nx) % nx, ys = (y + L::cy(i) + ny) % ny, zs = (z + L::cz(i) + nz) % nz;
        const int64_t s = (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
        const double r1 = (double)src[s], r2 = (double)src[stride + s], rho = r1 + r2;
        Collided<double> p;
        p.jx = (double)src[2 * stride + s];
        p.jy = (double)src[3 * stride + s];
        p.jz = (double)src[4 * stride + s];
        p.sxx = (double)src[5 * stride + s] - rho / 3.0;
        p.syy = (double)src[6 * stride + s] - rho / 3.0;
        p.szz = (double)src[7 * stride + s] - rho / 3.0;
        p.sxy = (double)src[8 * stride + s];
        p.sxz = (double)src[9 * stride + s];
        p.syz = (double)src[10 * stride + s];
        p.T = (rho - 1.0) - 1.5 * (p.sxx + p.syy + p.szz);
        const double f = L::w(i) + reconstruct<Q, double>(p, i);
        A[(int64_t)i * N + n] = (float)(r1 / rho * f);
        A[(int64_t)(Q + i) * N + n] = (float)(r2 / rho * f);
    }
}

template <int Q, class T>
__global__ void k_get_population2_state(const float *__restrict__ A, T *__restrict__ dst, int64_t stride, int nx,
                                        int ny, int nz, int64_t N)
{
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    MomentAcc<double> a;
    a.zero();
    double r1 = 0.0, r2 = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = (x - L::cx(i) + nx) % nx, ys = (y - L::cy(i) + ny) % ny, zs = (z - L::cz(i) + nz) % nz;
        const int64_t s = (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
        const double f1 = (double)A[(int64_t)i * N + s], f2 = (double)A[(int64_t)(Q + i) * N + s];
        r1 += f1;
        r2 += f2;
        accumulate<Q, double>(a, f1 + f2, i);
    }
    dst[n] = (T)r1;
    dst[stride + n] = (T)r2;
    dst[2 * stride + n] = (T)a.jx;
    dst[3 * stride + n] = (T)a.jy;
    dst[4 * stride + n] = (T)a.jz;
    dst[5 * stride + n] = (T)a.mxx;
    dst[6 * stride + n] = (T)a.myy;
    dst[7 * stride + n] = (T)a.mzz;
    dst[8 * stride + n] = (T)a.mxy;
    dst[9 * stride + n] = (T)a.mxz;
    dst[10 * stride + n] = (T)a.myz;
}

// ---- primitive fields -> equilibrium moments (public layout) ---------------------
//
// M = (rho^k, rho u, rho c_s^2 I + rho u u): the moments of the equilibrium
// populations of Eq. 5 (zero non-equilibrium part), FP64 arithmetic, rounded
// once at the store.  Primitive fields: rho (one species) or rho1, rho2, then
// ux, uy, uz.

template <class T, class O>
__global__ void k_primitive_to_moments(const T *__restrict__ src, int64_t stride, O *__restrict__ pub,
                                       int64_t ostride, int64_t N, int species)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double rho;
    int off;
    if (species == 1) {
        rho = (double)src[n];
        pub[n] = (O)rho;
        off = 1;
    } else {
        const double r1 = (double)src[n], r2 = (double)src[stride + n];
        rho = r1 + r2;
        pub[n] = (O)r1;
        pub[ostride + n] = (O)r2;
        off = 2;
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (double)src[(off + a) * stride + n];
    for (int a = 0; a < 3; ++a) pub[(off + a) * ostride + n] = (O)(rho * u[a]);
    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k)
        pub[(off + 3 + k) * ostride + n] = (O)(rho * u[pa[k]] * u[pb[k]] + (k < 3 ? rho / 3.0 : 0.0));
}

// Transpose of the Jacobian of the map above at the primitive fields `src`,
// applied to the moment gradient g (public layout): with g_j and g_P the
// gradients of j and of the six stored P components,
//   dL/drho^k = g_rho^k + u.g_j + sum_ab g_P_ab (u_a u_b + delta_ab/3),
//   dL/du_c   = rho g_j_c + rho sum_ab g_P_ab (delta_ac u_b + u_a delta_bc),
// a stored off-diagonal component counting once.  FP64 arithmetic.
template <class T, class G, class O>
__global__ void k_primitive_to_moments_adjoint(const T *__restrict__ src, int64_t stride, const G *__restrict__ g,
                                               int64_t gstride, O *__restrict__ out, int64_t ostride, int64_t N,
                                               int species)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int off = species == 1 ? 1 : 2;
    const double rho = species == 1 ? (double)src[n] : (double)src[n] + (double)src[stride + n];
    double u[3], gj[3], gp[6];
    for (int a = 0; a < 3; ++a) {
        u[a] = (double)src[(off + a) * stride + n];
        gj[a] = (double)g[(off + a) * gstride + n];
    }
    for (int k = 0; k < 6; ++k) gp[k] = (double)g[(off + 3 + k) * gstride + n];
    // Shared part of the density gradient (every species enters through rho).
    const double grho = u[0] * gj[0] + u[1] * gj[1] + u[2] * gj[2] + gp[0] * (u[0] * u[0] + 1.0 / 3.0) +
                        gp[1] * (u[1] * u[1] + 1.0 / 3.0) + gp[2] * (u[2] * u[2] + 1.0 / 3.0) +
                        gp[3] * u[0] * u[1] + gp[4] * u[0] * u[2] + gp[5] * u[1] * u[2];
    if (species == 1) {
        out[n] = (O)((double)g[n] + grho);
    } else {
        out[n] = (O)((double)g[n] + grho);
        out[ostride + n] = (O)((double)g[gstride + n] + grho);
    }
    const double gux = gj[0] + 2.0 * gp[0] * u[0] + gp[3] * u[1] + gp[4] * u[2];
    const double guy = gj[1] + 2.0 * gp[1] * u[1] + gp[3] * u[0] + gp[5] * u[2];
    const double guz = gj[2] + 2.0 * gp[2] * u[2] + gp[4] * u[0] + gp[5] * u[1];
    out[off * ostride + n] = (O)(rho * gux);
    out[(off + 1) * ostride + n] = (O)(rho * guy);
    out[(off + 2) * ostride + n] = (O)(rho * guz);
}

// ---- FP64 totals -------------------------------------------------------------------

// Block-level deterministic tree sum of 5 values per thread.
__device__ void block_sum5(double v[5], double *out)
{
    __shared__ double sh[5][kThreads];
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = sh[k][0];
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_reduce_moment(const S *__restrict__ st, int64_t N, int nx, int ny,
                                                            MomentLayout lay, int species,
                                                            double *__restrict__ partials)
{
    double v[5] = {0, 0, 0, 0, 0};
    const int js = species == 1 ? 1 : 2;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += (int64_t)gridDim.x * kThreads) {
        const int64_t so = stored_node(lay, n, nx, ny);
        if (species == 1) {
            v[0] += (double)Store<S>::load(st[so]);
        } else {
            v[0] += (double)Store<S>::load(st[kBlock + so]);
            v[1] += (double)Store<S>::load(st[so]);
        }
        for (int a = 0; a < 3; ++a) v[2 + a] += (double)Store<S>::load(st[(js + a) * kBlock + so]);
    }
    block_sum5(v, partials + 5 * blockIdx.x);
}

template <int Q, class S>
__global__ __launch_bounds__(kThreads) void k_reduce_population(const S *__restrict__ A, int64_t N,
                                                                double *__restrict__ partials)
{
    using L = Lattice<Q>;
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double f = (double)Store<S>::load(A[(int64_t)i * N + n]);
            v[0] += f;
            v[2] += L::cx(i) * f;
            v[3] += L::cy(i) * f;
            v[4] += L::cz(i) * f;
        }
    }
    block_sum5(v, partials + 5 * blockIdx.x);
}

// Two-species populations: v0 = sum rho1, v1 = sum rho2, v2..4 = sum j (raw).
template <int Q>
__global__ __launch_bounds__(kThreads) void k_reduce_population2(const float *__restrict__ A, int64_t N,
                                                                 double *__restrict__ partials)
{
    using L = Lattice<Q>;
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double f1 = A[(int64_t)i * N + n], f2 = A[(int64_t)(Q + i) * N + n];
            v[0] += f1;
            v[1] += f2;
            v[2] += L::cx(i) * (f1 + f2);
            v[3] += L::cy(i) * (f1 + f2);
            v[4] += L::cz(i) * (f1 + f2);
        }
    }
    block_sum5(v, partials + 5 * blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_reduce_final(const double *__restrict__ partials, int nblocks,
                                                           double *__restrict__ out)
{
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kThreads)
        for (int k = 0; k < 5; ++k) v[k] += partials[5 * b + k];
    block_sum5(v, out);
}

// ---- dispatch helpers -----------------------------------------------------------------

template <class F>
hipError_t with_storage(const lbm_ctx *c, F &&f)
{
    switch (c->storage) {
    case LBM_STORE_F64: return f((double *)nullptr);
    case LBM_STORE_F32: return f((float *)nullptr);
    case LBM_STORE_F16: return f((f16 *)nullptr);
    case LBM_STORE_BF16: return f((bf16 *)nullptr);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_set_moments(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *state)
{
    return with_storage(c, [&](auto *tag) -> hipError_t {
        using S = std::remove_pointer_t<decltype(tag)>;
        auto go = [&](auto *ttag) -> hipError_t {
            using T = std::remove_pointer_t<decltype(ttag)>;
            const T *s = static_cast<const T *>(src);
            if (c->scheme == LBM_SCHEME_MOMENT) {
                hipLaunchKernelGGL((k_set_moment_state<S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0, c->stream,
                                   s, stride, static_cast<S *>(state), c->N, c->nx, c->ny, c->lay, c->species,
                                   c->s_pi);
            } else if (c->species == 2) {
                if (c->q == 19)
                    hipLaunchKernelGGL((k_set_population2_state<19, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                       c->stream, s, stride, static_cast<float *>(state), c->nx, c->ny, c->nz, c->N);
                else
                    hipLaunchKernelGGL((k_set_population2_state<27, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                       c->stream, s, stride, static_cast<float *>(state), c->nx, c->ny, c->nz, c->N);
            } else if (c->q == 19) {
                hipLaunchKernelGGL((k_set_population_state<19, S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                   c->stream, s, stride, static_cast<S *>(state), c->nx, c->ny, c->nz, c->N);
            } else {
                hipLaunchKernelGGL((k_set_population_state<27, S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                   c->stream, s, stride, static_cast<S *>(state), c->nx, c->ny, c->nz, c->N);
            }
            return hipGetLastError();
        };
        return dtype == LBM_DTYPE_F64 ? go((double *)nullptr) : go((float *)nullptr);
    });
}

hipError_t launch_get_moments(const lbm_ctx *c, const void *state, void *dst, int64_t stride, int dtype)
{
    return with_storage(c, [&](auto *tag) -> hipError_t {
        using S = std::remove_pointer_t<decltype(tag)>;
        auto go = [&](auto *ttag) -> hipError_t {
            using T = std::remove_pointer_t<decltype(ttag)>;
            T *d = static_cast<T *>(dst);
            const S *st = static_cast<const S *>(state);
            if (c->scheme == LBM_SCHEME_MOMENT) {
                hipLaunchKernelGGL((k_get_moment_state<S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0, c->stream,
                                   st, d, stride, c->N, c->nx, c->ny, c->lay, c->species, 1.0 / c->s_pi);
            } else if (c->species == 2) {
                const float *A = reinterpret_cast<const float *>(state);
                if (c->q == 19)
                    hipLaunchKernelGGL((k_get_population2_state<19, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                       c->stream, A, d, stride, c->nx, c->ny, c->nz, c->N);
                else
                    hipLaunchKernelGGL((k_get_population2_state<27, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                       c->stream, A, d, stride, c->nx, c->ny, c->nz, c->N);
            } else if (c->q == 19) {
                hipLaunchKernelGGL((k_get_population_state<19, S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                   c->stream, st, d, stride, c->nx, c->ny, c->nz, c->N, aa_odd(c));
            } else {
                hipLaunchKernelGGL((k_get_population_state<27, S, T>), dim3(blocks_for(c->N)), dim3(kThreads), 0,
                                   c->stream, st, d, stride, c->nx, c->ny, c->nz, c->N, aa_odd(c));
            }
            return hipGetLastError();
        };
        return dtype == LBM_DTYPE_F64 ? go((double *)nullptr) : go((float *)nullptr);
    });
}

// Calls f((T*)nullptr) with T the element type of a caller buffer.
template <class F>
hipError_t with_dtype(int dtype, F &&f)
{
    return dtype == LBM_DTYPE_F64 ? f((double *)nullptr) : f((float *)nullptr);
}

hipError_t launch_equilibrium(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *dst,
                              int64_t dstride, int ddtype)
{
    return with_dtype(dtype, [&](auto *t) -> hipError_t {
        using T = std::remove_pointer_t<decltype(t)>;
        return with_dtype(ddtype, [&](auto *o) -> hipError_t {
            using O = std::remove_pointer_t<decltype(o)>;
            hipLaunchKernelGGL((k_primitive_to_moments<T, O>), dim3(blocks_for(c->N)), dim3(kThreads), 0, c->stream,
                               static_cast<const T *>(src), stride, static_cast<O *>(dst), dstride, c->N, c->species);
            return hipGetLastError();
        });
    });
}

hipError_t launch_equilibrium_adjoint(const lbm_ctx *c, const void *prim, int64_t pstride, int pdtype,
                                      const void *grad, int64_t gstride, int gdtype, void *out, int64_t ostride,
                                      int odtype)
{
    return with_dtype(pdtype, [&](auto *t) -> hipError_t {
        using T = std::remove_pointer_t<decltype(t)>;
        return with_dtype(gdtype, [&](auto *gt) -> hipError_t {
            using G = std::remove_pointer_t<decltype(gt)>;
            return with_dtype(odtype, [&](auto *o) -> hipError_t {
                using O = std::remove_pointer_t<decltype(o)>;
                hipLaunchKernelGGL((k_primitive_to_moments_adjoint<T, G, O>), dim3(blocks_for(c->N)), dim3(kThreads),
                                   0, c->stream, static_cast<const T *>(prim), pstride, static_cast<const G *>(grad),
                                   gstride, static_cast<O *>(out), ostride, c->N, c->species);
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_set_equilibrium(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *state)
{
    const int nf = c->species == 1 ? 10 : 11;
    double *pub = nullptr;
    hipError_t e = hipMallocAsync((void **)&pub, sizeof(double) * nf * c->N, c->stream);
    if (e != hipSuccess) return e;
    e = launch_equilibrium(c, src, stride, dtype, pub, c->N, LBM_DTYPE_F64);
    if (e == hipSuccess) e = launch_set_moments(c, pub, c->N, LBM_DTYPE_F64, state);
    hipError_t e2 = hipFreeAsync(pub, c->stream);
    return e != hipSuccess ? e : e2;
}

hipError_t launch_reduce(const lbm_ctx *c, const void *state)
{
    hipError_t e = with_storage(c, [&](auto *tag) -> hipError_t {
        using S = std::remove_pointer_t<decltype(tag)>;
        const S *st = static_cast<const S *>(state);
        if (c->scheme == LBM_SCHEME_MOMENT)
            hipLaunchKernelGGL((k_reduce_moment<S>), dim3(kReduceBlocks), dim3(kThreads), 0, c->stream, st, c->N,
                               c->nx, c->ny, c->lay, c->species, c->partials);
        else if (c->species == 2 && c->q == 19)
            hipLaunchKernelGGL((k_reduce_population2<19>), dim3(kReduceBlocks), dim3(kThreads), 0, c->stream,
                               reinterpret_cast<const float *>(state), c->N, c->partials);
        else if (c->species == 2)
            hipLaunchKernelGGL((k_reduce_population2<27>), dim3(kReduceBlocks), dim3(kThreads), 0, c->stream,
                               reinterpret_cast<const float *>(state), c->N, c->partials);
        else if (c->q == 19)
            hipLaunchKernelGGL((k_reduce_population<19, S>), dim3(kReduceBlocks), dim3(kThreads), 0, c->stream, st,
                               c->N, c->partials);
        else
            hipLaunchKernelGGL((k_reduce_population<27, S>), dim3(kReduceBlocks), dim3(kThreads), 0, c->stream, st,
                               c->N, c->partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kThreads), 0, c->stream, c->partials, kReduceBlocks,
                       c->red_out);
    return hipGetLastError();
}

hipError_t launch_costate_convert(const lbm_ctx *c, const void *src, void *dst, bool to_stored, int64_t stride,
                                  int pub_dtype)
{
    if (stride <= 0) stride = c->N;
    if (pub_dtype < 0) pub_dtype = c->storage == LBM_STORE_F64 ? LBM_DTYPE_F64 : LBM_DTYPE_F32;
    return with_dtype(pub_dtype, [&](auto *pt) -> hipError_t {
        using P = std::remove_pointer_t<decltype(pt)>;
        if (c->storage == LBM_STORE_F64)
            hipLaunchKernelGGL((k_costate_convert<P, double>), dim3(blocks_for(c->N)), dim3(kThreads), 0, c->stream,
                               src, dst, stride, c->N, c->nx, c->ny, c->lay, c->nfields, to_stored);
        else
            hipLaunchKernelGGL((k_costate_convert<P, float>), dim3(blocks_for(c->N)), dim3(kThreads), 0, c->stream,
                               src, dst, stride, c->N, c->nx, c->ny, c->lay, c->nfields, to_stored);
        return hipGetLastError();
    });
}

} // namespace lbm
