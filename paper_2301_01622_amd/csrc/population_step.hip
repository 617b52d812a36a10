// Population-storing schemes (the comparison "LB with populations").
//
// One species: the q post-collision populations of every node, shifted by
// their rest value (f~_i = f_i - w_i), one array per direction.  Pull scheme
// with two buffers: the thread of node x gathers f~_i(x - c_i), takes the
// moments (Eqs. 1-3), relaxes towards the equilibrium of Eq. 5 with Eq. 7,
// and writes its q post-collision populations to the other buffer.
//
// One species in place (AA pattern, one copy of the q arrays): slot i of node
// y holds, after an even number of steps, the post-collision population f*_i
// of y (the layout of the two-buffer scheme); a step from that state pulls
// f_i(x) from slot i of x - c_i, collides, and pushes f*_i(x) into the
// reversed slot of its destination, slot -i of x + c_i; after an odd number of
// steps slot -i of y therefore holds the population arriving at y, and the
// next step is node-local (read slot -i of x, write slot i of x).  In the
// non-local step the slots a node writes are exactly the slots it read
// ((j, x - c_j) for all j), so the update is race free in place.
//
// Two species (standard colour-gradient LB with stored populations): 2q
// arrays, species 1 then species 2, post-collision.  Each step is two
// kernels, as in split colour-gradient codes: a density pass that pulls both
// species and writes the phase field phi = (rho1 - rho2)/rho, then the
// collision pass that pulls again, takes the colour gradient from phi at the
// neighbours, relaxes the mixture (Eq. 7), adds the perturbation operator
// Df_i = (A/2)[w_i (c_i.G)^2 - B_i |G|^2]/D per population (its full form,
// fourth-order part included) and recolours.
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

// BGK relaxation of the shifted populations f (in place), Eqs. 5 and 7.
template <int Q, class R>
__device__ __forceinline__ void bgk_relax(R *f, R omega)
{
    MomentAcc<R> a;
    a.zero();
#pragma unroll
    for (int i = 0; i < Q; ++i) accumulate<Q, R>(a, f[i], i);
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
    for (int i = 0; i < Q; ++i) f[i] = fma_(omega, reconstruct<Q, R>(eq, i) - f[i], f[i]);
}

// One AA step on the single population array A; ODD: the state has gone
// through an odd number of steps (arrivals stored reversed at their node).
template <int Q, class S, bool ODD>
__global__ __launch_bounds__(256) void k_population_aa(S *__restrict__ A, int nx, int ny, int nz, int64_t N,
                                                       typename Store<S>::real omega)
{
    using R = typename Store<S>::real;
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);
    auto node = [&](int dx, int dy, int dz) -> int64_t {
        int xs = x + dx, ys = y + dy, zs = z + dz;
        xs += xs < 0 ? nx : 0;
        xs -= xs >= nx ? nx : 0;
        ys += ys < 0 ? ny : 0;
        ys -= ys >= ny ? ny : 0;
        zs += zs < 0 ? nz : 0;
        zs -= zs >= nz ? nz : 0;
        return (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
    };
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t at = ODD ? (int64_t)opposite<Q>(i) * N + n : (int64_t)i * N + node(-L::cx(i), -L::cy(i), -L::cz(i));
        f[i] = Store<S>::load(A[at]);
    }
    bgk_relax<Q, R>(f, omega);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t at = ODD ? (int64_t)i * N + n : (int64_t)opposite<Q>(i) * N + node(L::cx(i), L::cy(i), L::cz(i));
        A[at] = Store<S>::make(f[i]);
    }
}

template <int Q, class S>
hipError_t run_aa(const lbm_ctx *c, void *state, bool odd)
{
    using R = typename Store<S>::real;
    const int64_t blocks = (c->N + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (odd)
        hipLaunchKernelGGL((k_population_aa<Q, S, true>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           static_cast<S *>(state), c->nx, c->ny, c->nz, c->N, (R)c->omega);
    else
        hipLaunchKernelGGL((k_population_aa<Q, S, false>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           static_cast<S *>(state), c->nx, c->ny, c->nz, c->N, (R)c->omega);
    return hipGetLastError();
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

// ---- two species ---------------------------------------------------------------

template <int Q>
__device__ __forceinline__ int64_t pull_index(int x, int y, int z, int i, int nx, int ny, int nz)
{
    using L = Lattice<Q>;
    int xs = x - L::cx(i), ys = y - L::cy(i), zs = z - L::cz(i);
    xs += xs < 0 ? nx : 0;
    xs -= xs >= nx ? nx : 0;
    ys += ys < 0 ? ny : 0;
    ys -= ys >= ny ? ny : 0;
    zs += zs < 0 ? nz : 0;
    zs -= zs >= nz ? nz : 0;
    return (int64_t)xs + (int64_t)nx * ((int64_t)ys + (int64_t)ny * zs);
}

template <int Q>
__global__ __launch_bounds__(256) void k_pop_cg_phi(const float *__restrict__ in, float *__restrict__ phi, int nx,
                                                    int ny, int nz, int64_t N)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    float r1 = 0.f, r2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t s = pull_index<Q>(x, y, z, i, nx, ny, nz);
        r1 += in[(int64_t)i * N + s];
        r2 += in[(int64_t)(Q + i) * N + s];
    }
    phi[n] = (r1 - r2) / (r1 + r2);
}

// FORCE: a body force (three arrays of N values) enters with Guo's forcing
// (equilibrium at u* = (j + F/2)/rho, source (1 - omega/2) S_i).
template <int Q, bool FORCE>
__global__ __launch_bounds__(256) void k_pop_cg_step(const float *__restrict__ in, float *__restrict__ out,
                                                     const float *__restrict__ phi, int nx, int ny, int nz, int64_t N,
                                                     float omega, float A, float beta, const float *__restrict__ frc)
{
    using L = Lattice<Q>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % nx);
    const int64_t t = n / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);

    float f[Q];
    float r1 = 0.f, r2 = 0.f, rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t s = pull_index<Q>(x, y, z, i, nx, ny, nz);
        const float a = in[(int64_t)i * N + s], b = in[(int64_t)(Q + i) * N + s];
        r1 += a;
        r2 += b;
        f[i] = a + b;
        rho += f[i];
        if (L::cx(i)) jx = L::cx(i) > 0 ? jx + f[i] : jx - f[i];
        if (L::cy(i)) jy = L::cy(i) > 0 ? jy + f[i] : jy - f[i];
        if (L::cz(i)) jz = L::cz(i) > 0 ? jz + f[i] : jz - f[i];
    }
    // Colour gradient from the phase field of the neighbours.
    float Gx = 0.f, Gy = 0.f, Gz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (L::cx(i) == 0 && L::cy(i) == 0 && L::cz(i) == 0) continue;
        const int64_t s = pull_index<Q>(x, y, z, opposite<Q>(i), nx, ny, nz);  // x + c_i
        const float wp = (float)(3.0 * L::w(i)) * phi[s];
        if (L::cx(i)) Gx = L::cx(i) > 0 ? Gx + wp : Gx - wp;
        if (L::cy(i)) Gy = L::cy(i) > 0 ? Gy + wp : Gy - wp;
        if (L::cz(i)) Gz = L::cz(i) > 0 ? Gz + wp : Gz - wp;
    }
    const float G2 = fma_(Gx, Gx, fma_(Gy, Gy, Gz * Gz));
    const float invD = 1.0f / __builtin_sqrtf(G2 + 1e-6f);
    const float inv_rho = reciprocal<float>(rho);
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (FORCE) {
        Fx = frc[n];
        Fy = frc[N + n];
        Fz = frc[2 * N + n];
    }
    const float ux = FORCE ? fma_(0.5f, Fx, jx) * inv_rho : jx * inv_rho;
    const float uy = FORCE ? fma_(0.5f, Fy, jy) * inv_rho : jy * inv_rho;
    const float uz = FORCE ? fma_(0.5f, Fz, jz) * inv_rho : jz * inv_rho;
    const float uF = fma_(ux, Fx, fma_(uy, Fy, uz * Fz));
    const float src = 1.0f - 0.5f * omega;
    const float uu = fma_(ux, ux, fma_(uy, uy, uz * uz));
    const float s1 = r1 * inv_rho, s2 = r2 * inv_rho;
    const float C = beta * r1 * r2 * inv_rho;
    // Moving directions first; the rest population of each species takes
    // what is left of its density, so every node emits exactly its mass
    // (in exact arithmetic the relaxation, the perturbation and the
    // recolouring all conserve it; FP32 weights do not sum to one exactly).
    float sum1 = 0.f, sum2 = 0.f;
    int rest = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
        if (cx == 0 && cy == 0 && cz == 0) {
            rest = i;
            continue;
        }
        const float w = (float)L::w(i);
        const float cu = (float)cx * ux + (float)cy * uy + (float)cz * uz;
        const float feq = w * rho * fma_(4.5f, cu * cu, fma_(3.0f, cu, 1.0f - 1.5f * uu));
        const float cG = (float)cx * Gx + (float)cy * Gy + (float)cz * Gz;
        const float df = 0.5f * A * fma_(w, cG * cG, -w * G2) * invD;
        float fp = fma_(omega, feq - f[i], f[i]) + df;
        if (FORCE) {
            const float cF = (float)cx * Fx + (float)cy * Fy + (float)cz * Fz;
            fp = fma_(src * w, fma_(9.0f * cu, cF, 3.0f * (cF - uF)), fp);
        }
        const float inv_c = (float)(1.0 / __builtin_sqrt((double)(cx * cx + cy * cy + cz * cz)));
        const float rc = C * w * inv_c * (cG * invD);
        const float o1 = fma_(s1, fp, rc), o2 = fma_(s2, fp, -rc);
        out[(int64_t)i * N + n] = o1;
        out[(int64_t)(Q + i) * N + n] = o2;
        sum1 += o1;
        sum2 += o2;
    }
    out[(int64_t)rest * N + n] = r1 - sum1;
    out[(int64_t)(Q + rest) * N + n] = r2 - sum2;
}

template <int Q>
hipError_t run_cg(const lbm_ctx *c, const void *in, void *out)
{
    const int64_t blocks = (c->N + 255) / 256;
    hipLaunchKernelGGL((k_pop_cg_phi<Q>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                       static_cast<const float *>(in), c->scratch_phi, c->nx, c->ny, c->nz, c->N);
    if (c->nc_A != 0.0) {
        hipError_t e = launch_nc_force(c, nullptr, c->scratch_phi);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_pop_cg_step<Q, true>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           static_cast<const float *>(in), static_cast<float *>(out), c->scratch_phi, c->nx, c->ny,
                           c->nz, c->N, (float)c->omega, (float)c->A, (float)c->beta,
                           static_cast<const float *>(c->scratch_nc));
    } else {
        hipLaunchKernelGGL((k_pop_cg_step<Q, false>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           static_cast<const float *>(in), static_cast<float *>(out), c->scratch_phi, c->nx, c->ny,
                           c->nz, c->N, (float)c->omega, (float)c->A, (float)c->beta, nullptr);
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_population_step(const lbm_ctx *c, const void *in, void *out)
{
    if (c->species == 2) {
        if (c->storage != LBM_STORE_F32 || !c->scratch_phi) return hipErrorInvalidValue;
        return c->q == 19 ? run_cg<19>(c, in, out) : run_cg<27>(c, in, out);
    }
    if (c->species != 1) return hipErrorNotSupported;
    if (c->storage == LBM_STORE_F64) return c->q == 19 ? run<19, double>(c, in, out) : run<27, double>(c, in, out);
    if (c->storage == LBM_STORE_F32) return c->q == 19 ? run<19, float>(c, in, out) : run<27, float>(c, in, out);
    return hipErrorInvalidValue;
}

hipError_t launch_population_aa_step(const lbm_ctx *c, void *state, bool odd)
{
    if (c->species != 1) return hipErrorNotSupported;
    if (c->storage == LBM_STORE_F64)
        return c->q == 19 ? run_aa<19, double>(c, state, odd) : run_aa<27, double>(c, state, odd);
    if (c->storage == LBM_STORE_F32)
        return c->q == 19 ? run_aa<19, float>(c, state, odd) : run_aa<27, float>(c, state, odd);
    return hipErrorInvalidValue;
}

} // namespace lbm
