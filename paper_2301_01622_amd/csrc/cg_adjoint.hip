// Discrete adjoint of the two-component (colour-gradient) moment-only step.
//
// Forward at a source node y (see cg_step.hip; rho = rho1 + rho2,
// s_k = rho^k/rho, phi = s_1 - s_2, D = sqrt(|G|^2 + eps^2), n = G/D):
//   h'_i = w_i [T + 3 c_i.j + 4.5 c_i c_i : S'],  S' = (1-omega)S + omega jj/rho + DP,
//   DP   = (A/9)(G G - |G|^2 I)/D,   T = rho - 1.5 tr S',
//   f1_i = s_1 h'_i + rc_i,  f2_i = s_2 h'_i - rc_i,  rc_i = C w_i (c_i.n)/|c_i|,
//   C = beta rho1 rho2/rho;  node y + c_i receives f1_i, f2_i and (via j, P) h'_i.
// With co-states lam(t+1) = (l1, l2, lj, lP) gathered from y + c_i,
//   e_i = (l1 + l2)/2 + c_i.lj + c_i c_i:lP,   d_i = l1 - l2,
// the co-state of h'_i is A_i = e_i + (phi/2) d_i and that of rc_i is d_i.
// Everything needed at y follows from weighted moments of e and d:
//   E = sum_i w_i (1, c_i, c_i c_i) e_i,  Dm = sum_i w_i (1, c_i, c_i c_i) d_i,
//   V = sum_i w_i d_i c_i/|c_i|,
//   alpha, beta, M2 = E + (phi/2) Dm;  Gamma = 4.5 M2 - 1.5 alpha I;
//   S1 - S2 = sum_i d_i h'_i = T Dm0 + 3 j.Dm1 + 4.5 S':Dm2;
//   lam_rho = alpha - omega j.Gamma.j/rho^2 - (1-omega) tr Gamma/3,
//   lam_j   = 3 beta + 2 omega Gamma j/rho,  lam_P = (1-omega) Gamma (off-diag. x2),
//   lam_1   = lam_rho + (S1-S2) rho2/rho^2 + (V.n) beta rho2^2/rho^2,
//   lam_2   = lam_rho - (S1-S2) rho1/rho^2 + (V.n) beta rho1^2/rho^2,
//   gG      = (A/9)[(2 Gamma G - 2 tr Gamma G)/D - (G.Gamma.G - |G|^2 tr Gamma) G/D^3]
//             + C (V/D - G (G.V)/D^3),
// and, because G(y) reads phi on the radius-1 stencil, a second pass adds
// gphi(z) = sum_k 3 w_k c_k . gG(z - c_k) through dphi/drho1 = 2 rho2/rho^2,
// dphi/drho2 = -2 rho1/rho^2.  dL/dtau at fixed sigma:
//   -omega^2 sum Gamma:(jj/rho - S) - (1/tau) sum Gamma:DP.
//
// First pass: z-marching tiles as in the forward kernel; every node of the
// tile plus halo publishes e_i (all directions) and d to LDS, interior nodes
// gather them from y + c_i into three plane accumulators; a completed plane
// is finished with the node's own state and the phase field (four-plane LDS
// ring).  Second pass: a plain stencil over gG.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

constexpr double kEpsG2 = 1e-6;  // (1e-3)^2, as in the forward step

template <class R>
struct CgAdjAcc {
    MomentAcc<R> e, d;
    R vx, vy, vz;
    __device__ __forceinline__ void zero()
    {
        e.zero();
        d.zero();
        vx = vy = vz = R(0);
    }
};

template <int Q>
__host__ __device__ constexpr double inv_len(int cx, int cy, int cz)
{
    return (cx * cx + cy * cy + cz * cz) == 1 ? 1.0 : (cx * cx + cy * cy + cz * cz) == 2 ? 0.70710678118654752440
                                                                                           : 0.57735026918962576451;
}

// Weighted layer sums: f holds per slot the value to accumulate.
template <int Q, int CZ, class R>
__device__ __forceinline__ void weighted_layer(MomentAcc<R> &a, const Layer<R> &v)
{
    Layer<R> f;
#pragma unroll
    for (int sl = 0; sl < 9; ++sl)
        if (has_dir<Q>(sl % 3 - 1, sl / 3 - 1, CZ)) f.v[sl] = R(weight<Q>(sl % 3 - 1, sl / 3 - 1, CZ)) * v.v[sl];
    accumulate_layer<Q, CZ, R>(a, f);
}

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

// LSTORED: co-states in the stored (blocked) layout of the state instead of
// the public one.
// Launch shapes: the first pass is sized for LBM_CGA_WG resident workgroups
// per CU (200 VGPRs at D3Q19 FP32; three would spill 141); the second marches
// 64 x LBM_CGA_PHI_TY tiles in z-chunks sized for LBM_CGA_PHI_WG resident
// workgroups per CU (64 x 8 in 64-plane chunks on 512 x 256 x 256: 12 % faster
// than whole-column 64 x 16 tiles, one workgroup per CU).
#ifndef LBM_CGA_WG
#define LBM_CGA_WG 2
#endif
#ifndef LBM_CGA_PHI_TY
#define LBM_CGA_PHI_TY 8
#endif
#ifndef LBM_CGA_PHI_WG
#define LBM_CGA_PHI_WG 4
#endif

template <int Q, class R, int TX, int TY, bool LSTORED>
__global__ __launch_bounds__(TX *TY) void k_cg_adjoint_tile(
    const R *__restrict__ state, const R *__restrict__ lam_in, R *__restrict__ lam_out, R *__restrict__ gG, TileGrid g,
    MomentLayout lay3, R omega, R A9, R beta, double tau, double *__restrict__ partials)
{
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int RING = HN - NT;
    static_assert(RING <= NT, "halo ring must fit one pass");
    __shared__ R lds_e[Q * HN];   // e_i of every direction, slot = direction number
    __shared__ R lds_d[HN];       // d = l1 - l2
    __shared__ R lds_phi[4 * HN]; // phase field, planes p-2 .. p+1
    __shared__ double red[NT];

    const int b = xcd_tile_id();
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
    const int h0 = (ly + 1) * HX + (lx + 1);
    // Halo ring node of this thread.  The ring rows (x inside the tile) take
    // threads [0, 2 TX), the ring columns (corners included) the threads from
    // the next multiple of 64 on, so that a wave holds ring nodes of one or two
    // orientations.  A ring node y + c_i is gathered from only by directions i
    // that point out of the tile across its side (c_y = -1 for the row above,
    // +1 below, c_x = -1 for the column on the left, +1 on the right), so it
    // publishes e_i for those alone (5 of 19 for D3Q19, 9 of 27 for D3Q27; a
    // corner publishes those of its column, which include the ones it sends).
    constexpr int ROWS = 2 * TX, CB = (ROWS + 63) / 64 * 64, COLS = 2 * HY;
    static_assert(ROWS + COLS == RING && CB + COLS <= NT, "ring threads must fit the workgroup");
    const bool ring_row = tid < ROWS;
    const bool ring_col = tid >= CB && tid < CB + COLS;
    const bool has_ring = ring_row || ring_col;
    int hr = 0, ring_side = 0;  // 0: above, 1: below, 2: left, 3: right
    if (ring_row) {
        const bool above = tid < TX;
        hr = (above ? 0 : HY - 1) * HX + 1 + (above ? tid : tid - TX);
        ring_side = above ? 0 : 1;
    } else if (ring_col) {
        const int m = tid - CB;
        const bool left = m < HY;
        hr = (left ? m : m - HY) * HX + (left ? 0 : HX - 1);
        ring_side = left ? 2 : 3;
    }
    auto xy_of = [&](int h) -> int64_t {
        return (int64_t)wrap_coord(x0 - 1 + h % HX, g.nx) + (int64_t)g.nx * wrap_coord(y0 - 1 + h / HX, g.ny);
    };
    const int64_t own_xy = xy_of(h0);
    const int64_t ring_xy = has_ring ? xy_of(hr) : 0;
    // The same nodes in the stored (blocked) layout of the state.
    auto sxy_of = [&](int h) -> int64_t {
        return g.lay.xy(wrap_coord(x0 - 1 + h % HX, g.nx), wrap_coord(y0 - 1 + h / HX, g.ny));
    };
    const int64_t own_sxy = sxy_of(h0);
    const int64_t ring_sxy = has_ring ? sxy_of(hr) : 0;
    auto zs_of = [&](int p) { return p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p); };
    auto zoff = [&](int p) -> int64_t { return (int64_t)zs_of(p) * plane; };
    auto ring_slot = [&](int p) { return (p - z0 + 4) & 3; };

    // phi of plane p for this thread's nodes (from the stored dr and rho1):
    // the loads (one plane ahead of their use), then the LDS writes.
    auto load_phi = [&](int p, R *v) {
        const int64_t zo = (int64_t)zs_of(p) * g.lay.plane;
        v[0] = state[own_sxy + zo];
        v[1] = state[kBlock + own_sxy + zo];
        if (has_ring) {
            v[2] = state[ring_sxy + zo];
            v[3] = state[kBlock + ring_sxy + zo];
        }
    };
    auto store_phi = [&](int p, const R *v) {
        R *ph = lds_phi + ring_slot(p) * HN;
        ph[h0] = fma_(R(2) * v[1], reciprocal<R>(R(1) + v[0]), R(-1));
        if (has_ring) ph[hr] = fma_(R(2) * v[3], reciprocal<R>(R(1) + v[2]), R(-1));
    };

    // e_i and d of one co-state node into LDS slot h; SIDE < 0 publishes
    // every direction, SIDE = 0..3 only those leaving the tile across that
    // side of the ring.
    auto publish = [&](auto side, const R *l, int h) {
        constexpr int SIDE = decltype(side)::value;
        lds_d[h] = l[0] - l[1];
        const R gbar = R(0.5) * (l[0] + l[1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = Lattice<Q>::cx(i), cy = Lattice<Q>::cy(i), cz = Lattice<Q>::cz(i);
            if ((SIDE == 0 && cy != -1) || (SIDE == 1 && cy != 1) || (SIDE == 2 && cx != -1) ||
                (SIDE == 3 && cx != 1))
                continue;
            R e = gbar;
            if (cx) e = cx > 0 ? e + l[2] : e - l[2];
            if (cy) e = cy > 0 ? e + l[3] : e - l[3];
            if (cz) e = cz > 0 ? e + l[4] : e - l[4];
            if (cx) e += l[5];
            if (cy) e += l[6];
            if (cz) e += l[7];
            if (cx * cy) e = cx * cy > 0 ? e + l[8] : e - l[8];
            if (cx * cz) e = cx * cz > 0 ? e + l[9] : e - l[9];
            if (cy * cz) e = cy * cz > 0 ? e + l[10] : e - l[10];
            lds_e[i * HN + h] = e;
        }
    };

    CgAdjAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();
    double dtau = 0.0;

    auto gather_layer = [&](auto czc) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> e, d;
        R vx = R(0), vy = R(0), vz = R(0);
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            if (!has_dir<Q>(cx, cy, CZ)) continue;
            int i = 0;
#pragma unroll
            for (int k = 0; k < Q; ++k)
                if (Lattice<Q>::cx(k) == cx && Lattice<Q>::cy(k) == cy && Lattice<Q>::cz(k) == CZ) i = k;
            const int src = h0 + cy * HX + cx;
            e.v[sl] = lds_e[i * HN + src];
            d.v[sl] = lds_d[src];
            if (cx || cy || CZ) {
                const R wd = R(weight<Q>(cx, cy, CZ) * inv_len<Q>(cx, cy, CZ)) * d.v[sl];
                if (cx) vx = cx > 0 ? vx + wd : vx - wd;
                if (cy) vy = cy > 0 ? vy + wd : vy - wd;
                if (CZ) vz = CZ > 0 ? vz + wd : vz - wd;
            }
        }
        CgAdjAcc<R> &a = acc[1 - CZ];
        weighted_layer<Q, CZ, R>(a.e, e);
        weighted_layer<Q, CZ, R>(a.d, d);
        a.vx += vx;
        a.vy += vy;
        a.vz += vz;
    };

    // The node's own state of plane dpl, loaded a plane step before finish()
    // uses it.
    auto load_own = [&](int dpl, R *v) {
        const int64_t so = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)dpl * g.lay.plane;
#pragma unroll
        for (int k = 0; k < 11; ++k) v[k] = state[k * kBlock + so];
    };
    auto finish = [&](int dpl, const R *st) {
        const int64_t so = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)dpl * g.lay.plane;    // stored
        const int64_t op = (int64_t)(x0 + lx) + (int64_t)g.nx * (y0 + ly) + (int64_t)dpl * plane;  // public
        const int64_t o = LSTORED ? so : op;  // co-states
        const int64_t LF = LSTORED ? (int64_t)kBlock : g.N;
        const CgAdjAcc<R> &a = acc[0];
        // Own state.
        const R dr = st[0], r1 = st[1];
        const R jx = st[2], jy = st[3], jz = st[4];
        R s[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = st[5 + k];
        const R rho = R(1) + dr, r2 = rho - r1;
        const R inv_rho = R(1) / rho;
        // Colour gradient from the phase field of planes d-1, d, d+1.
        const R *phm = lds_phi + ring_slot(dpl - 1) * HN;
        const R *ph0 = lds_phi + ring_slot(dpl) * HN;
        const R *php = lds_phi + ring_slot(dpl + 1) * HN;
        R Gx = R(0), Gy = R(0), Gz = R(0);
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                for (int cx = -1; cx <= 1; ++cx) {
                    if ((cx == 0 && cy == 0 && cz == 0) || !has_dir<Q>(cx, cy, cz)) continue;
                    const R *ph = cz < 0 ? phm : (cz == 0 ? ph0 : php);
                    const R wphi = R(3.0 * weight<Q>(cx, cy, cz)) * ph[h0 + cy * HX + cx];
                    if (cx) Gx = cx > 0 ? Gx + wphi : Gx - wphi;
                    if (cy) Gy = cy > 0 ? Gy + wphi : Gy - wphi;
                    if (cz) Gz = cz > 0 ? Gz + wphi : Gz - wphi;
                }
        const R phi = ph0[h0];
        const R G2 = fma_(Gx, Gx, fma_(Gy, Gy, Gz * Gz));
        const R invD = R(1) / sqrt_<R>(G2 + R(kEpsG2));
        const R nx = Gx * invD, ny = Gy * invD, nz = Gz * invD;
        // Collided tensor S' with the perturbation, and T of the unshifted populations.
        const R om1 = R(1) - omega, oi = omega * inv_rho;
        const R a9 = A9 * invD;
        const R dpxx = a9 * fma_(Gx, Gx, -G2), dpyy = a9 * fma_(Gy, Gy, -G2), dpzz = a9 * fma_(Gz, Gz, -G2);
        const R dpxy = a9 * Gx * Gy, dpxz = a9 * Gx * Gz, dpyz = a9 * Gy * Gz;
        const R cxx = fma_(oi * jx, jx, om1 * s[0]) + dpxx, cyy = fma_(oi * jy, jy, om1 * s[1]) + dpyy,
                czz = fma_(oi * jz, jz, om1 * s[2]) + dpzz;
        const R cxy = fma_(oi * jx, jy, om1 * s[3]) + dpxy, cxz = fma_(oi * jx, jz, om1 * s[4]) + dpxz,
                cyz = fma_(oi * jy, jz, om1 * s[5]) + dpyz;
        const R Tfull = fma_(R(-1.5), (cxx + cyy) + czz, rho);
        // Moments of A = e + (phi/2) d.
        const R hp = R(0.5) * phi;
        const R al = fma_(hp, a.d.r, a.e.r);
        const R bx = fma_(hp, a.d.jx, a.e.jx), by = fma_(hp, a.d.jy, a.e.jy), bz = fma_(hp, a.d.jz, a.e.jz);
        const R mxx = fma_(hp, a.d.mxx, a.e.mxx), myy = fma_(hp, a.d.myy, a.e.myy), mzz = fma_(hp, a.d.mzz, a.e.mzz);
        const R mxy = fma_(hp, a.d.mxy, a.e.mxy), mxz = fma_(hp, a.d.mxz, a.e.mxz), myz = fma_(hp, a.d.myz, a.e.myz);
        const R gxx = fma_(R(4.5), mxx, R(-1.5) * al), gyy = fma_(R(4.5), myy, R(-1.5) * al),
                gzz = fma_(R(4.5), mzz, R(-1.5) * al);
        const R gxy = R(4.5) * mxy, gxz = R(4.5) * mxz, gyz = R(4.5) * myz;
        const R tr = (gxx + gyy) + gzz;
        const R Gjx = fma_(gxx, jx, fma_(gxy, jy, gxz * jz));
        const R Gjy = fma_(gxy, jx, fma_(gyy, jy, gyz * jz));
        const R Gjz = fma_(gxz, jx, fma_(gyz, jy, gzz * jz));
        const R jGj = fma_(jx, Gjx, fma_(jy, Gjy, jz * Gjz));
        const R lrho = fma_(-omega * inv_rho * inv_rho, jGj, fma_(-om1 * R(1.0 / 3.0), tr, al));
        // S1 - S2 = sum_i d_i h'_i
        const R sdm = fma_(Tfull, a.d.r, R(3) * fma_(jx, a.d.jx, fma_(jy, a.d.jy, jz * a.d.jz))) +
                      R(4.5) * (fma_(cxx, a.d.mxx, fma_(cyy, a.d.myy, czz * a.d.mzz)) +
                                R(2) * fma_(cxy, a.d.mxy, fma_(cxz, a.d.mxz, cyz * a.d.myz)));
        const R Vn = fma_(a.vx, nx, fma_(a.vy, ny, a.vz * nz));
        const R ir2 = inv_rho * inv_rho;
        lam_out[o] = fma_(sdm * r2, ir2, fma_(Vn * beta * r2 * r2, ir2, lrho));
        lam_out[LF + o] = fma_(-sdm * r1, ir2, fma_(Vn * beta * r1 * r1, ir2, lrho));
        const R two_om = R(2) * omega * inv_rho;
        lam_out[2 * LF + o] = fma_(two_om, Gjx, R(3) * bx);
        lam_out[3 * LF + o] = fma_(two_om, Gjy, R(3) * by);
        lam_out[4 * LF + o] = fma_(two_om, Gjz, R(3) * bz);
        lam_out[5 * LF + o] = om1 * gxx;
        lam_out[6 * LF + o] = om1 * gyy;
        lam_out[7 * LF + o] = om1 * gzz;
        lam_out[8 * LF + o] = R(2) * om1 * gxy;
        lam_out[9 * LF + o] = R(2) * om1 * gxz;
        lam_out[10 * LF + o] = R(2) * om1 * gyz;
        // Co-state of G.
        const R GGx = fma_(gxx, Gx, fma_(gxy, Gy, gxz * Gz));
        const R GGy = fma_(gxy, Gx, fma_(gyy, Gy, gyz * Gz));
        const R GGz = fma_(gxz, Gx, fma_(gyz, Gy, gzz * Gz));
        const R GgG = fma_(Gx, GGx, fma_(Gy, GGy, Gz * GGz));
        const R num = fma_(-G2, tr, GgG);
        const R invD3 = invD * invD * invD;
        const R C = beta * r1 * r2 * inv_rho;
        const R GV = fma_(Gx, a.vx, fma_(Gy, a.vy, Gz * a.vz));
        auto gcomp = [&](R GGa, R Ga, R Va) {
            const R pert = A9 * (R(2) * fma_(-tr, Ga, GGa) * invD - num * Ga * invD3);
            return fma_(C, fma_(-Ga * GV, invD3, Va * invD), pert);
        };
        const int64_t og = lay3.xy(x0 + lx, y0 + ly) + (int64_t)dpl * lay3.plane;  // scratch, 3-field blocks
        gG[og] = gcomp(GGx, Gx, a.vx);
        gG[kBlock + og] = gcomp(GGy, Gy, a.vy);
        gG[2 * kBlock + og] = gcomp(GGz, Gz, a.vz);
        // tau-sensitivity at fixed sigma.
        const R sxx = s[0], syy = s[1], szz = s[2], sxy = s[3], sxz = s[4], syz = s[5];
        const double eo = (double)(gxx * (jx * jx * inv_rho - sxx) + gyy * (jy * jy * inv_rho - syy) +
                                   gzz * (jz * jz * inv_rho - szz)) +
                          2.0 * (double)(gxy * (jx * jy * inv_rho - sxy) + gxz * (jx * jz * inv_rho - sxz) +
                                         gyz * (jy * jz * inv_rho - syz));
        const double ea = (double)(gxx * dpxx + gyy * dpyy + gzz * dpzz) +
                          2.0 * (double)(gxy * dpxy + gxz * dpxz + gyz * dpyz);
        dtau += -(double)omega * (double)omega * eo - ea / tau;
    };

    R la[11], lb[11], rla[11], rlb[11];
    auto fetch = [&](int p, R *own, R *ring) {
        const int64_t LF = LSTORED ? (int64_t)kBlock : g.N;
        const int64_t zo = LSTORED ? (int64_t)zs_of(p) * g.lay.plane : zoff(p);
        const int64_t oxy = LSTORED ? own_sxy : own_xy, rxy = LSTORED ? ring_sxy : ring_xy;
#pragma unroll
        for (int k = 0; k < 11; ++k) own[k] = lam_in[k * LF + oxy + zo];
        if (has_ring) {
#pragma unroll
            for (int k = 0; k < 11; ++k) ring[k] = lam_in[k * LF + rxy + zo];
        }
    };

    R phv[4], stf[11];
    auto plane_step = [&](int p, R *own, R *ring) {
        const int dpl = p - 1;
        const bool fin = dpl >= z0 && active;
        if (fin) load_own(dpl, stf);
        store_phi(p + 1, phv);
        publish(std::integral_constant<int, -1>(), own, h0);
        if (has_ring) {
            switch (ring_side) {
            case 0: publish(std::integral_constant<int, 0>(), ring, hr); break;
            case 1: publish(std::integral_constant<int, 1>(), ring, hr); break;
            case 2: publish(std::integral_constant<int, 2>(), ring, hr); break;
            default: publish(std::integral_constant<int, 3>(), ring, hr); break;
            }
        }
        __syncthreads();
        if (p + 2 <= z_end) fetch(p + 2, own, ring);
        if (p + 1 <= z_end) load_phi(p + 2, phv);
        gather_layer(std::integral_constant<int, -1>());
        gather_layer(std::integral_constant<int, 0>());
        gather_layer(std::integral_constant<int, 1>());
        if (fin) finish(dpl, stf);
        __syncthreads();
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    };

    // Phase field of planes z0-2 .. z0-1 before the loop; plane p+1 is added
    // in each step, so planes d-1 .. d+1 are present when plane d finishes.
    load_phi(z0 - 2, phv);
    store_phi(z0 - 2, phv);
    load_phi(z0 - 1, phv);
    store_phi(z0 - 1, phv);
    load_phi(z0, phv);
    fetch(z0 - 1, la, rla);
    fetch(z0, lb, rlb);
    for (int p = z0 - 1; p <= z_end; p += 2) {
        plane_step(p, la, rla);
        if (p + 1 <= z_end) plane_step(p + 1, lb, rlb);
    }

    red[tid] = dtau;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) partials[blockIdx.x] = red[0];
}

// Second pass: the phase-field chain of the colour gradient,
//   gphi(z) = sum_k 3 w_k c_k . gG(z - c_k),
//   lam1 += gphi 2 rho2/rho^2,  lam2 -= gphi 2 rho1/rho^2.
// A workgroup marches a TX x TY tile along z; the three components of gG for
// the tile plus a one-node halo ring are kept for planes z-1, z, z+1 in an LDS
// ring, so each gG value is read from HBM about once (a one-thread-per-node
// stencil re-reads the neighbouring planes from memory).
template <int Q, class R, int TX, int TY, bool LSTORED>
__global__ __launch_bounds__(TX *TY) void k_cg_adjoint_phi(const R *__restrict__ state, const R *__restrict__ gG,
                                                           R *__restrict__ lam_out, TileGrid g, MomentLayout lay3)
{
    using L = Lattice<Q>;
    constexpr int NT = TX * TY;
    constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int RING = HN - NT;
    static_assert(RING <= NT, "halo ring must fit one pass");
    __shared__ R lds_g[3 * 3 * HN];  // [plane slot][component][halo tile]

    const int b = xcd_tile_id();
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
    const int h0 = (ly + 1) * HX + (lx + 1);
    const bool has_ring = tid < RING;
    int hr;
    {
        const int m = tid;
        int hx, hy;
        if (m < HX) { hx = m; hy = 0; }
        else if (m < 2 * HX) { hx = m - HX; hy = HY - 1; }
        else if (m < 2 * HX + TY) { hx = 0; hy = 1 + (m - 2 * HX); }
        else { hx = HX - 1; hy = 1 + (m - 2 * HX - TY); }
        hr = hy * HX + hx;
    }
    auto xy_of = [&](int h) -> int64_t {  // in the 3-field blocked layout of gG
        return lay3.xy(wrap_coord(x0 - 1 + h % HX, g.nx), wrap_coord(y0 - 1 + h / HX, g.ny));
    };
    const int64_t own_xy = xy_of(h0);
    const int64_t ring_xy = has_ring ? xy_of(hr) : 0;
    auto zs_of = [&](int p) { return p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p); };
    auto slot = [&](int p) { return (p - z0 + 3) % 3; };

    R go[3], gr[3];
    auto fetch = [&](int p) {
        const int64_t zo = (int64_t)zs_of(p) * lay3.plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) go[a] = gG[a * kBlock + own_xy + zo];
        if (has_ring) {
#pragma unroll
            for (int a = 0; a < 3; ++a) gr[a] = gG[a * kBlock + ring_xy + zo];
        }
    };
    auto publish = [&](int p) {
        R *d = lds_g + slot(p) * 3 * HN;
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a * HN + h0] = go[a];
        if (has_ring) {
#pragma unroll
            for (int a = 0; a < 3; ++a) d[a * HN + hr] = gr[a];
        }
    };

    // Planes z0-1 and z0 are in LDS and plane z0+1 in registers before the
    // loop; each step publishes plane p+1, then loads plane p+2 while plane p
    // is computed.  Slot (p+1) mod 3 held plane p-2, last read before the
    // previous step's closing barrier.
    fetch(z0 - 1);
    publish(z0 - 1);
    fetch(z0);
    publish(z0);
    fetch(z0 + 1);
    for (int p = z0; p < z_end; ++p) {
        publish(p + 1);
        __syncthreads();
        fetch(p + 2);
        if (active) {
            R gphi = R(0);
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int cx = L::cx(k), cy = L::cy(k), cz = L::cz(k);
                if (!cx && !cy && !cz) continue;
                const R *d = lds_g + slot(p - cz) * 3 * HN;
                const int h = h0 - cy * HX - cx;
                R c = R(0);
                if (cx) c = cx > 0 ? c + d[h] : c - d[h];
                if (cy) c = cy > 0 ? c + d[HN + h] : c - d[HN + h];
                if (cz) c = cz > 0 ? c + d[2 * HN + h] : c - d[2 * HN + h];
                gphi = fma_(R(3.0 * L::w(k)), c, gphi);
            }
            const int64_t so = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)p * g.lay.plane;
            const int64_t n = LSTORED ? so : (int64_t)(x0 + lx) + (int64_t)g.nx * (y0 + ly) + (int64_t)p * plane;
            const int64_t LF = LSTORED ? (int64_t)kBlock : g.N;
            const R rho = R(1) + state[so], r1 = state[kBlock + so], r2 = rho - r1;
            const R k2 = R(2) * gphi / (rho * rho);
            lam_out[n] = fma_(k2, r2, lam_out[n]);
            lam_out[LF + n] = fma_(-k2, r1, lam_out[LF + n]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_cg_add_partials(const double *__restrict__ partials, int n,
                                                         double *__restrict__ accum)
{
    __shared__ double sh[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partials[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *accum += sh[0];
}

template <int Q, class R, int TX, int TY, bool LSTORED>
hipError_t run(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out, double *dtau, void *gG_buf)
{
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.lay = c->lay;
    g.tiles_x = (c->nx + TX - 1) / TX;
    g.tiles_y = (c->ny + TY - 1) / TY;
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y, 256 * LBM_CGA_WG);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > 5 * kReduceBlocks) return hipErrorInvalidConfiguration;
    R *gG = static_cast<R *>(gG_buf);
    hipLaunchKernelGGL((k_cg_adjoint_tile<Q, R, TX, TY, LSTORED>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                       static_cast<const R *>(state), static_cast<const R *>(lam_in), static_cast<R *>(lam_out), gG,
                       g, c->lay3, (R)c->omega, (R)(c->A / 9.0), (R)c->beta, c->tau, c->partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TileGrid gp = g;
    gp.tiles_x = (c->nx + 63) / 64;
    gp.tiles_y = (c->ny + LBM_CGA_PHI_TY - 1) / LBM_CGA_PHI_TY;
    gp.zchunk = choose_zchunk(c->nz, gp.tiles_x * gp.tiles_y, 256 * LBM_CGA_PHI_WG);
    gp.chunks = (c->nz + gp.zchunk - 1) / gp.zchunk;
    const int64_t pblocks = (int64_t)gp.tiles_x * gp.tiles_y * gp.chunks;
    if (pblocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_cg_adjoint_phi<Q, R, 64, LBM_CGA_PHI_TY, LSTORED>), dim3((unsigned)pblocks),
                       dim3(64 * LBM_CGA_PHI_TY), 0, c->stream,
                       static_cast<const R *>(state), static_cast<const R *>(gG), static_cast<R *>(lam_out), gp, c->lay3);
    e = hipGetLastError();
    if (e != hipSuccess || !dtau) return e;
    hipLaunchKernelGGL(k_cg_add_partials, dim3(1), dim3(256), 0, c->stream, c->partials, (int)blocks, dtau);
    return hipGetLastError();
}

template <bool LS>
hipError_t dispatch(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out, double *dtau, void *gG)
{
    if (c->storage == LBM_STORE_F32)
        return c->q == 19 ? run<19, float, 64, 4, LS>(c, state, lam_in, lam_out, dtau, gG)
                          : run<27, float, 32, 8, LS>(c, state, lam_in, lam_out, dtau, gG);
    if (c->storage == LBM_STORE_F64)
        return c->q == 19 ? run<19, double, 32, 8, LS>(c, state, lam_in, lam_out, dtau, gG)
                          : run<27, double, 32, 8, LS>(c, state, lam_in, lam_out, dtau, gG);
    return hipErrorNotSupported;
}

} // namespace

hipError_t launch_cg_adjoint_step(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out,
                                  double *dtau_accum, bool stored, void *gG_scratch)
{
    if (!gG_scratch) gG_scratch = c->scratch_adj;
    if (c->species != 2 || !gG_scratch) return hipErrorNotSupported;
    return stored ? dispatch<true>(c, state, lam_in, lam_out, dtau_accum, gG_scratch)
                  : dispatch<false>(c, state, lam_in, lam_out, dtau_accum, gG_scratch);
}

} // namespace lbm
