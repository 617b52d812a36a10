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
//
// Both the reconstruction and the moment sums are organised by velocity
// layers c_z = -1, 0, +1: within a layer the nine (c_x, c_y) combinations
// share partial sums, which roughly halves the arithmetic of writing every
// direction out on its own.
#pragma once

#include "lattice.hpp"

// Every fused multiply-add below is written out: with implicit contraction
// the compiler may fuse the same expression differently at two inlined call
// sites (e.g. a node collided as a tile node and as a halo node), and the
// result would then depend on the tiling.
#pragma clang fp contract(off)

namespace lbm {

template <class R>
__device__ __forceinline__ R fma_(R a, R b, R c)
{
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_<float>(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}

// Post-collision moments of one node, ready for reconstruction.
template <class R>
struct Collided {
    R T, jx, jy, jz, sxx, syy, szz, sxy, sxz, syz;
};

template <class R>
__device__ __forceinline__ R reciprocal(R x)
{
    return R(1) / x;
}
// FP32: the hardware reciprocal (1 ulp); 1/rho only scales the O(u^2) term.
template <>
__device__ __forceinline__ float reciprocal<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}

template <class R>
__device__ __forceinline__ Collided<R> collide(R dr, R jx, R jy, R jz, R sxx, R syy, R szz, R sxy, R sxz,
                                               R syz, R omega)
{
    Collided<R> p;
    const R inv_rho = reciprocal<R>(R(1) + dr);
    const R om1 = R(1) - omega;
    const R oi = omega * inv_rho;
    const R ox = oi * jx, oy = oi * jy, oz = oi * jz;
    p.sxx = fma_(ox, jx, om1 * sxx);
    p.syy = fma_(oy, jy, om1 * syy);
    p.szz = fma_(oz, jz, om1 * szz);
    p.sxy = fma_(ox, jy, om1 * sxy);
    p.sxz = fma_(ox, jz, om1 * sxz);
    p.syz = fma_(oy, jz, om1 * syz);
    p.T = fma_(R(-1.5), (p.sxx + p.syy) + p.szz, dr);
    p.jx = jx;
    p.jy = jy;
    p.jz = jz;
    return p;
}

// The same record built from moments that are already post-collision (the
// split approach of Sec. III.A stores them between its two passes); equal to
// collide() applied to the pre-collision moments when S' was stored exactly.
template <class R>
__device__ __forceinline__ Collided<R> collided_from(R dr, R jx, R jy, R jz, R sxx, R syy, R szz, R sxy, R sxz,
                                                     R syz)
{
    Collided<R> p;
    p.sxx = sxx;
    p.syy = syy;
    p.szz = szz;
    p.sxy = sxy;
    p.sxz = sxz;
    p.syz = syz;
    p.T = fma_(R(-1.5), (p.sxx + p.syy) + p.szz, dr);
    p.jx = jx;
    p.jy = jy;
    p.jz = jz;
    return p;
}

// Shifted population h~_i of direction i written out on its own (used by
// the conversion kernels; the step kernels use the layered form below).
template <int Q, class R>
__device__ __forceinline__ R reconstruct(const Collided<R> &p, int i)
{
    using L = Lattice<Q>;
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    R lin = p.T;
    if (cx != 0) lin = fma_(cx > 0 ? R(3) : R(-3), p.jx, lin);
    if (cy != 0) lin = fma_(cy > 0 ? R(3) : R(-3), p.jy, lin);
    if (cz != 0) lin = fma_(cz > 0 ? R(3) : R(-3), p.jz, lin);
    R quad = R(0);
    if (cx != 0) quad += p.sxx;
    if (cy != 0) quad += p.syy;
    if (cz != 0) quad += p.szz;
    if (cx * cy != 0) quad = fma_(cx * cy > 0 ? R(2) : R(-2), p.sxy, quad);
    if (cx * cz != 0) quad = fma_(cx * cz > 0 ? R(2) : R(-2), p.sxz, quad);
    if (cy * cz != 0) quad = fma_(cy * cz > 0 ? R(2) : R(-2), p.syz, quad);
    return R(L::w(i)) * fma_(R(4.5), quad, lin);
}

// The nine (c_x, c_y) slots of one layer, index (cx+1) + 3 (cy+1).
template <class R>
struct Layer {
    R v[9];
};

// Does the lattice contain direction (cx, cy, cz)?
template <int Q>
__host__ __device__ constexpr bool has_dir(int cx, int cy, int cz)
{
    return Q == 27 || (cx * cx + cy * cy + cz * cz) <= 2;
}

template <int Q>
__host__ __device__ constexpr double weight(int cx, int cy, int cz)
{
    if (Q == 27) return Lattice<27>::w1(cx) * Lattice<27>::w1(cy) * Lattice<27>::w1(cz);
    const int s = cx * cx + cy * cy + cz * cz;
    return s == 0 ? 1.0 / 3.0 : s == 1 ? 1.0 / 18.0 : s == 2 ? 1.0 / 36.0 : 0.0;
}

// Shifted populations of layer c_z = CZ.  With
//   A  = T + 3 cz jz + 4.5 cz^2 Szz,  Bx = 3 jx + 9 cz Sxz,  By = 3 jy + 9 cz Syz,
// the bracket is A + cx Bx + cy By + 4.5 (cx^2 Sxx + cy^2 Syy) + 9 cx cy Sxy.
// Slots of directions absent from the lattice are left unset.
template <int Q, int CZ, class R>
__device__ __forceinline__ void reconstruct_layer(const Collided<R> &p, Layer<R> &o)
{
    const R jx3 = R(3) * p.jx, jy3 = R(3) * p.jy;
    R A, Bx, By;
    if (CZ == 0) {
        A = p.T;
        Bx = jx3;
        By = jy3;
    } else {
        A = fma_(R(3 * CZ), p.jz, fma_(R(4.5), p.szz, p.T));
        Bx = fma_(R(9 * CZ), p.sxz, jx3);
        By = fma_(R(9 * CZ), p.syz, jy3);
    }
    const R Px = fma_(R(4.5), p.sxx, A), Py = fma_(R(4.5), p.syy, A);
    o.v[4] = R(weight<Q>(0, 0, CZ)) * A;
    o.v[5] = R(weight<Q>(1, 0, CZ)) * (Px + Bx);
    o.v[3] = R(weight<Q>(-1, 0, CZ)) * (Px - Bx);
    o.v[7] = R(weight<Q>(0, 1, CZ)) * (Py + By);
    o.v[1] = R(weight<Q>(0, -1, CZ)) * (Py - By);
    if (has_dir<Q>(1, 1, CZ)) {
        const R Pxy = fma_(R(4.5), p.syy, Px);
        const R D1 = fma_(R(9), p.sxy, Pxy), D2 = fma_(R(-9), p.sxy, Pxy);
        const R E1 = Bx + By, E2 = Bx - By;
        o.v[8] = R(weight<Q>(1, 1, CZ)) * (D1 + E1);
        o.v[0] = R(weight<Q>(-1, -1, CZ)) * (D1 - E1);
        o.v[2] = R(weight<Q>(1, -1, CZ)) * (D2 + E2);
        o.v[6] = R(weight<Q>(-1, 1, CZ)) * (D2 - E2);
    }
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

// Adds the streamed populations of layer c_z = CZ (slots as in Layer) to
// the accumulators of their destination plane.  Rows of fixed c_y are
// summed first (sum, sum c_x, sum c_x^2), then the rows are combined.
template <int Q, int CZ, class R>
__device__ __forceinline__ void accumulate_layer(MomentAcc<R> &a, const Layer<R> &f)
{
    constexpr bool corners = has_dir<Q>(1, 1, CZ);
    // Row c_y = 0: slots 3 (cx=-1), 4 (cx=0), 5 (cx=+1).
    const R r0_2 = f.v[3] + f.v[5], r0_1 = f.v[5] - f.v[3], r0_0 = r0_2 + f.v[4];
    R s, sx, sy, sxx, syy, sxy;
    if (corners) {
        // Rows c_y = -1 (slots 0,1,2) and +1 (slots 6,7,8).
        const R rm_2 = f.v[0] + f.v[2], rm_1 = f.v[2] - f.v[0], rm_0 = rm_2 + f.v[1];
        const R rp_2 = f.v[6] + f.v[8], rp_1 = f.v[8] - f.v[6], rp_0 = rp_2 + f.v[7];
        syy = rp_0 + rm_0;
        s = syy + r0_0;
        sy = rp_0 - rm_0;
        sx = r0_1 + (rp_1 + rm_1);
        sxy = rp_1 - rm_1;
        sxx = r0_2 + (rp_2 + rm_2);
    } else {
        syy = f.v[7] + f.v[1];
        s = syy + r0_0;
        sy = f.v[7] - f.v[1];
        sx = r0_1;
        sxy = R(0);
        sxx = r0_2;
    }
    a.r += s;
    a.jx += sx;
    a.jy += sy;
    a.mxx += sxx;
    a.myy += syy;
    if (corners) a.mxy += sxy;
    if (CZ != 0) {
        if (CZ > 0) { a.jz += s; a.mxz += sx; a.myz += sy; }
        else { a.jz -= s; a.mxz -= sx; a.myz -= sy; }
        a.mzz += s;
    }
}

} // namespace lbm
