// Node-level pieces of the discrete adjoint of the one-species moment step,
// shared by the one-step and the two-step adjoint kernels (the transposed
// step itself is written out at the top of adjoint_step.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "moment_math.hpp"
#include "storage.hpp"

namespace lbm {

// b = w_i (lam_rho + c.lam_j + c c : lam_P) for the nine slots of layer CZ
// (stored off-diagonal components enter once: m_i has c_x c_y for P_xy).
template <int Q, int CZ, class R>
__device__ __forceinline__ void adjoint_layer(const R *l, Layer<R> &o)
{
    // l: rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz
    R A, Bx, By;
    if (CZ == 0) {
        A = l[0];
        Bx = l[1];
        By = l[2];
    } else {
        A = (CZ > 0 ? l[0] + l[3] : l[0] - l[3]) + l[6];
        Bx = CZ > 0 ? l[1] + l[8] : l[1] - l[8];
        By = CZ > 0 ? l[2] + l[9] : l[2] - l[9];
    }
    const R Px = A + l[4], Py = A + l[5];
    o.v[4] = R(weight<Q>(0, 0, CZ)) * A;
    o.v[5] = R(weight<Q>(1, 0, CZ)) * (Px + Bx);
    o.v[3] = R(weight<Q>(-1, 0, CZ)) * (Px - Bx);
    o.v[7] = R(weight<Q>(0, 1, CZ)) * (Py + By);
    o.v[1] = R(weight<Q>(0, -1, CZ)) * (Py - By);
    if (has_dir<Q>(1, 1, CZ)) {
        const R Pxy = Px + l[5];
        const R D1 = Pxy + l[7], D2 = Pxy - l[7], E1 = Bx + By, E2 = Bx - By;
        o.v[8] = R(weight<Q>(1, 1, CZ)) * (D1 + E1);
        o.v[0] = R(weight<Q>(-1, -1, CZ)) * (D1 - E1);
        o.v[2] = R(weight<Q>(1, -1, CZ)) * (D2 + E2);
        o.v[6] = R(weight<Q>(-1, 1, CZ)) * (D2 - E2);
    }
}

// The node-local part of the transposed step: the gathered accumulator a
// (alpha, beta and the second moments of w_i a_i) and the node's forward
// state v (10 stored values) give the co-state lam (10 values); returns the
// node's term of the relaxation-frequency sensitivity, Gamma : (j j/rho - S).
template <class S>
__device__ __forceinline__ double adjoint_node(const MomentAcc<typename Store<S>::real> &a, const S *v,
                                               typename Store<S>::real omega, typename Store<S>::real inv_s_pi,
                                               typename Store<S>::real *lam)
{
    using R = typename Store<S>::real;
    const R dr = Store<S>::load(v[0]);
    const R jx = Store<S>::load(v[1]), jy = Store<S>::load(v[2]), jz = Store<S>::load(v[3]);
    R s[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = Store<S>::load(v[4 + k]) * inv_s_pi;
    const R inv_rho = R(1) / (R(1) + dr);
    // Gamma = 4.5 sum w c c a - 1.5 alpha I
    const R gxx = fma_(R(4.5), a.mxx, R(-1.5) * a.r), gyy = fma_(R(4.5), a.myy, R(-1.5) * a.r),
            gzz = fma_(R(4.5), a.mzz, R(-1.5) * a.r);
    const R gxy = R(4.5) * a.mxy, gxz = R(4.5) * a.mxz, gyz = R(4.5) * a.myz;
    const R Gjx = fma_(gxx, jx, fma_(gxy, jy, gxz * jz));
    const R Gjy = fma_(gxy, jx, fma_(gyy, jy, gyz * jz));
    const R Gjz = fma_(gxz, jx, fma_(gyz, jy, gzz * jz));
    const R jGj = fma_(jx, Gjx, fma_(jy, Gjy, jz * Gjz));
    const R om1 = R(1) - omega;
    const R tr = (gxx + gyy) + gzz;
    lam[0] = fma_(-omega * inv_rho * inv_rho, jGj, fma_(-om1 * R(1.0 / 3.0), tr, a.r));
    const R two_om = R(2) * omega * inv_rho;
    lam[1] = fma_(two_om, Gjx, R(3) * a.jx);
    lam[2] = fma_(two_om, Gjy, R(3) * a.jy);
    lam[3] = fma_(two_om, Gjz, R(3) * a.jz);
    lam[4] = om1 * gxx;
    lam[5] = om1 * gyy;
    lam[6] = om1 * gzz;
    lam[7] = R(2) * om1 * gxy;
    lam[8] = R(2) * om1 * gxz;
    lam[9] = R(2) * om1 * gyz;
    return (double)(gxx * (jx * jx * inv_rho - s[0]) + gyy * (jy * jy * inv_rho - s[1]) +
                    gzz * (jz * jz * inv_rho - s[2])) +
           2.0 * (double)(gxy * (jx * jy * inv_rho - s[3]) + gxz * (jx * jz * inv_rho - s[4]) +
                          gyz * (jy * jz * inv_rho - s[5]));
}

} // namespace lbm
