// Per-node arithmetic of the moment-only step, in shifted variables.
//
// The state of a node is stored as deviations from the rest state:
//   dr = rho - 1,  j = rho u,  S = P - rho c_s^2 I.
// With omega = 1/tau the BGK collision (Eqs. 7-8) acts on the moments as
//   S' = (1 - omega) S + omega j j / rho          (rho and j unchanged),
// and, writing Q_i:X = 4.5 c_i c_i : X - 1.5 tr X (c_s^2 = 1/3), the
// reconstructed post-collision population of Eqs. 4-6 becomes
//   h'_i = w_i + w_i [T + 3 c_i.j + 4.5 c_i c_i : S'],   T = dr - 1.5 tr S'.
// The kernels carry the shifted population h~_i = h'_i - w_i, whose moments
// are again deviations: sum h~ = dr', sum c h~ = j',
// sum c_a c_b h~ - (dr'/3) delta_ab = S'_new.  Every quantity is small, so
// FP32 arithmetic and 16-bit storage keep their relative precision.
#pragma once

#include "lattice.hpp"

namespace lbm {

// Post-collision moments of one node, ready for reconstruction.
template <class R>
struct Collided {
    R T, jx, jy, jz, sxx, syy, szz, sxy, sxz, syz;
};

template <class R>
__device__ __forceinline__ Collided<R> collide(R dr, R jx, R jy, R jz, R sxx, R syy, R szz, R sxy, R sxz,
                                               R syz, R omega)
{
    Collided<R> p;
    const R inv_rho = R(1) / (R(1) + dr);
    const R om1 = R(1) - omega;
    const R ox = omega * inv_rho * jx, oy = omega * inv_rho * jy, oz = omega * inv_rho * jz;
    p.sxx = om1 * sxx + ox * jx;
    p.syy = om1 * syy + oy * jy;
    p.szz = om1 * szz + oz * jz;
    p.sxy = om1 * sxy + ox * jy;
    p.sxz = om1 * sxz + ox * jz;
    p.syz = om1 * syz + oy * jz;
    p.T = dr - R(1.5) * (p.sxx + p.syy + p.szz);
    p.jx = jx;
    p.jy = jy;
    p.jz = jz;
    return p;
}

// Shifted population h~_i of direction i (compile-time after unrolling).
template <int Q, class R>
__device__ __forceinline__ R reconstruct(const Collided<R> &p, int i)
{
    using L = Lattice<Q>;
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    R lin = p.T;
    if (cx != 0) lin += (cx > 0 ? R(3) : R(-3)) * p.jx;
    if (cy != 0) lin += (cy > 0 ? R(3) : R(-3)) * p.jy;
    if (cz != 0) lin += (cz > 0 ? R(3) : R(-3)) * p.jz;
    R quad = R(0);
    if (cx != 0) quad += p.sxx;
    if (cy != 0) quad += p.syy;
    if (cz != 0) quad += p.szz;
    if (cx * cy != 0) quad += (cx * cy > 0 ? R(2) : R(-2)) * p.sxy;
    if (cx * cz != 0) quad += (cx * cz > 0 ? R(2) : R(-2)) * p.sxz;
    if (cy * cz != 0) quad += (cy * cz > 0 ? R(2) : R(-2)) * p.syz;
    return R(L::w(i)) * (lin + R(4.5) * quad);
}

// Moment accumulators of the streamed shifted set (Eqs. 1-3).
template <class R>
struct MomentAcc {
    R r, jx, jy, jz, mxx, myy, mzz, mxy, mxz, myz;
    __device__ __forceinline__ void zero()
    {
        r = jx = jy = jz = mxx = myy = mzz = mxy = mxz = myz = R(0);
    }
};

template <int Q, class R>
__device__ __forceinline__ void accumulate(MomentAcc<R> &a, R h, int i)
{
    using L = Lattice<Q>;
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    a.r += h;
    if (cx != 0) { if (cx > 0) a.jx += h; else a.jx -= h; a.mxx += h; }
    if (cy != 0) { if (cy > 0) a.jy += h; else a.jy -= h; a.myy += h; }
    if (cz != 0) { if (cz > 0) a.jz += h; else a.jz -= h; a.mzz += h; }
    if (cx * cy != 0) { if (cx * cy > 0) a.mxy += h; else a.mxy -= h; }
    if (cx * cz != 0) { if (cx * cz > 0) a.mxz += h; else a.mxz -= h; }
    if (cy * cz != 0) { if (cy * cz > 0) a.myz += h; else a.myz -= h; }
}

} // namespace lbm
