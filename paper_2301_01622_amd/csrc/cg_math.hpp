// Per-node arithmetic of the two-component (colour-gradient) step, shared by
// the fused step and the split schedule so that both compute every node
// bit for bit alike.
//
//   G  = (1/c_s^2) sum_i w_i c_i phi(y + c_i)            (colour gradient)
//   D  = sqrt(|G|^2 + eps^2),  n = G/D                     (smoothed normal)
//   S' = (1 - omega) S + omega j j/rho + (A/9)(G G - |G|^2 I)/D
// with Guo's forcing of a body force F when present: the equilibrium is taken
// at j* = j + F/2, (1 - omega/2)(u* F + F u*) is added to S' and j + F is
// streamed.
#pragma once

#include "moment_math.hpp"

#pragma clang fp contract(off)

namespace lbm {

// Smoothed gradient norm D = sqrt(|G|^2 + kEpsG^2): n = G/D is the unit
// normal on every interface and fades smoothly to zero where the gradient
// vanishes; the perturbation uses the same D.
constexpr double kEpsG = 1e-3;

template <class R>
__device__ __forceinline__ R sqrt_(R x)
{
    return __builtin_sqrt(x);
}
template <>
__device__ __forceinline__ float sqrt_<float>(float x)
{
    return __builtin_sqrtf(x);
}

// 1/sqrt(x): FP32 uses the hardware reciprocal square root (about 1 ulp);
// FP64 keeps the correctly rounded quotient.
template <class R>
__device__ __forceinline__ R rsqrt_(R x)
{
    return R(1) / sqrt_<R>(x);
}
template <>
__device__ __forceinline__ float rsqrt_<float>(float x)
{
    return __builtin_amdgcn_rsqf(x);
}

// Phase field phi = (rho1 - rho2)/rho = 2 rho1/rho - 1 from the stored
// mixture deviation dr = rho - 1 and rho1.
template <class R>
__device__ __forceinline__ R phase_field(R dr, R r1)
{
    return fma_(R(2) * r1, reciprocal<R>(R(1) + dr), R(-1));
}

// G = 3 sum_i w_i c_i phi(y + c_i): the signed phi values (phi_at(cx, cy,
// cz) = phi(y + c)) are summed per weight class (faces, edges, corners) in a
// fixed order and each class is scaled once.
template <int Q, class R, class PhiAt>
__device__ __forceinline__ void colour_gradient(PhiAt phi_at, R G[3])
{
    R gf[3] = {R(0), R(0), R(0)}, ge[3] = {R(0), R(0), R(0)}, gc[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
        for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
            for (int cx = -1; cx <= 1; ++cx) {
                if ((cx == 0 && cy == 0 && cz == 0) || !has_dir<Q>(cx, cy, cz)) continue;
                const R f = phi_at(cx, cy, cz);
                const int cls = cx * cx + cy * cy + cz * cz;
                R *acc_c = cls == 1 ? gf : (cls == 2 ? ge : gc);
                if (cx != 0) acc_c[0] = cx > 0 ? acc_c[0] + f : acc_c[0] - f;
                if (cy != 0) acc_c[1] = cy > 0 ? acc_c[1] + f : acc_c[1] - f;
                if (cz != 0) acc_c[2] = cz > 0 ? acc_c[2] + f : acc_c[2] - f;
            }
    constexpr double w3f = 3.0 * weight<Q>(1, 0, 0), w3e = 3.0 * weight<Q>(1, 1, 0), w3c = 3.0 * weight<Q>(1, 1, 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        G[a] = fma_(R(w3e), ge[a], R(w3f) * gf[a]);
        if (Q == 27) G[a] = fma_(R(w3c), gc[a], G[a]);
    }
}

template <class R>
struct CgCollided {
    Collided<R> c;  // post-collision moments with the perturbation (j + F under a force)
    R nx, ny, nz;   // n = G/D
};

// Collision of one node with the perturbation (and Guo's forcing if FORCE).
// v: dr, rho1, jx, jy, jz, Sxx, Syy, Szz, Sxy, Sxz, Syz.
template <class R, bool FORCE>
__device__ __forceinline__ CgCollided<R> cg_collide(const R *v, const R G[3], R omega, R A9, R fx, R fy, R fz)
{
    const R Gx = G[0], Gy = G[1], Gz = G[2];
    const R G2 = fma_(Gx, Gx, fma_(Gy, Gy, Gz * Gz));
    const R invD = rsqrt_<R>(G2 + R(kEpsG * kEpsG));
    CgCollided<R> o;
    o.nx = Gx * invD;
    o.ny = Gy * invD;
    o.nz = Gz * invD;
    const R dr = v[0];
    Collided<R> &c = o.c;
    if (FORCE) {
        // Guo's forcing: equilibrium at j* = j + F/2, source (1 - omega/2)(u* F + F u*).
        const R jsx = fma_(R(0.5), fx, v[2]), jsy = fma_(R(0.5), fy, v[3]), jsz = fma_(R(0.5), fz, v[4]);
        c = collide<R>(dr, jsx, jsy, jsz, v[5], v[6], v[7], v[8], v[9], v[10], omega);
        const R k = (R(1) - R(0.5) * omega) * reciprocal<R>(R(1) + dr);
        const R kx = k * jsx, ky = k * jsy, kz = k * jsz;
        c.sxx = fma_(R(2) * kx, fx, c.sxx);
        c.syy = fma_(R(2) * ky, fy, c.syy);
        c.szz = fma_(R(2) * kz, fz, c.szz);
        c.sxy = fma_(kx, fy, fma_(ky, fx, c.sxy));
        c.sxz = fma_(kx, fz, fma_(kz, fx, c.sxz));
        c.syz = fma_(ky, fz, fma_(kz, fy, c.syz));
        c.jx = v[2] + fx;
        c.jy = v[3] + fy;
        c.jz = v[4] + fz;
    } else {
        c = collide<R>(dr, v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], omega);
    }
    // Perturbation: A/9 (G G - |G|^2 I)/D.
    const R a9 = A9 * invD;
    c.sxx = fma_(a9, fma_(Gx, Gx, -G2), c.sxx);
    c.syy = fma_(a9, fma_(Gy, Gy, -G2), c.syy);
    c.szz = fma_(a9, fma_(Gz, Gz, -G2), c.szz);
    c.sxy = fma_(a9, Gx * Gy, c.sxy);
    c.sxz = fma_(a9, Gx * Gz, c.sxz);
    c.syz = fma_(a9, Gy * Gz, c.syz);
    // The trace of the perturbation is -2A|G|/9; T follows the collided S'.
    c.T = fma_(R(-1.5), (c.sxx + c.syy) + c.szz, dr);
    return o;
}

} // namespace lbm
