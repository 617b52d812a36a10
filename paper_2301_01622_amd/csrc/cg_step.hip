// Fused moment-only time step for two components (colour-gradient model).
//
// The paper carries two species on one flow field (Sec. III.A): per species
// only a density is stored, the density gradient is taken on the streamed
// (pre-collision) state, and the perturbation and recolouring operators act
// on the populations of Eq. 8.  Stored state per node (11 arrays): the
// mixture deviation dr = rho - 1, rho1, j, S = P - rho c_s^2 I.
//
// Per source node y (tile plus one-node halo):
//   phi   = (rho1 - rho2)/rho on a radius-2 footprint, kept in LDS for the
//           three planes z-1, z, z+1 (computed one plane ahead);
//   G     = (1/c_s^2) sum_i w_i c_i phi(y + c_i),  D = sqrt(|G|^2 + 1e-6),  n = G/D;
//   S'    = (1 - omega) S + omega j j/rho + (A/9)(G G - |G|^2 I)/D  (collision
//           plus the second moment of the perturbation operator);
//   h~_i  = w_i [T + 3 c_i.j + 4.5 c_i c_i : S'],  T = dr - 1.5 tr S';
//   f1_i  = (rho1/rho)(w_i + h~_i) + beta (rho1 rho2/rho) w_i (c_i.n)/|c_i|.
// Both h~_i and f1_i go through LDS; each interior node pulls them from
// x - c_i, sums the mixture moments from h~ and rho1 from f1.  The structure
// (z-marching tiles, three accumulator planes, two-plane prefetch,
// XCD-aware tile order) is that of the one-component kernel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"
#include "moment_math.hpp"
#include "storage.hpp"
#include "tile_common.hpp"

namespace lbm {
namespace {

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

template <class R>
struct CgAcc {
    MomentAcc<R> m;
    R rho1;
    __device__ __forceinline__ void zero()
    {
        m.zero();
        rho1 = R(0);
    }
};

template <int Q>
__host__ __device__ constexpr double inv_speed(int cx, int cy, int cz)
{
    return (cx * cx + cy * cy + cz * cz) == 1 ? 1.0 : (cx * cx + cy * cy + cz * cz) == 2 ? 0.70710678118654752440
                                                                                           : 0.57735026918962576451;
}

// FORCE: a body force (three arrays of N values, x fastest) enters the
// mixture collision with Guo's forcing: u* = (j + F/2)/rho in the
// equilibrium, (1 - omega/2)(u* F + F u*) added to the collided S, j + F
// streamed; the phase field phi = 2 rho1/rho - 1 of the stored output is
// written to phi_out (N values, x fastest) for the next step's force.
template <int Q, class R, int TX, int TY, bool FORCE>
__global__ __launch_bounds__(TX *TY) void k_cg_tile(const R *__restrict__ in, R *__restrict__ out, TileGrid g,
                                                    R omega, R A9, R beta, const R *__restrict__ frc,
                                                    R *__restrict__ phi_out)
{
    constexpr int NT = TX * TY;
    constexpr int SX = TX + 2, SY = TY + 2, SN = SX * SY;  // source region (radius 1)
    constexpr int FX = TX + 4, FY = TY + 4, FN = FX * FY;  // phase-field region (radius 2)
    constexpr int RING = SN - NT;                          // radius-1 halo nodes
    constexpr int OUTER = FN - SN;                         // radius-2 ring (phi only)
    static_assert(RING <= NT && OUTER <= NT, "halo rings must fit one pass");
    constexpr int NS = kLdsSlots<Q>;
    __shared__ R lds_h[NS * SN];   // shifted mixture populations
    __shared__ R lds_f[NS * SN];   // species-1 populations
    __shared__ R lds_phi[3 * FN];  // phase field of three planes

    const int b = xcd_tile_id();
    const int tx = b % g.tiles_x;
    const int ty = (b / g.tiles_x) % g.tiles_y;
    const int chunk = b / (g.tiles_x * g.tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = chunk * g.zchunk;
    const int z_end = min(z0 + g.zchunk, g.nz);
    const int64_t plane = g.lay.plane;  // stored elements per z-plane

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const bool active = (x0 + lx < g.nx) && (y0 + ly < g.ny);
    const int h0 = (ly + 1) * SX + (lx + 1);

    // Radius-1 ring node of this thread (source region coordinates).
    const bool has_ring = tid < RING;
    int hr;
    {
        const int m = tid;
        int hx, hy;
        if (m < SX) { hx = m; hy = 0; }
        else if (m < 2 * SX) { hx = m - SX; hy = SY - 1; }
        else if (m < 2 * SX + TY) { hx = 0; hy = 1 + (m - 2 * SX); }
        else { hx = SX - 1; hy = 1 + (m - 2 * SX - TY); }
        hr = hy * SX + hx;
    }
    // Radius-2 ring node of this thread (phase-field region coordinates).
    const bool has_outer = tid < OUTER;
    int ko;
    {
        const int m = tid;
        int kx, ky;
        if (m < FX) { kx = m; ky = 0; }
        else if (m < 2 * FX) { kx = m - FX; ky = FY - 1; }
        else if (m < 2 * FX + SY) { kx = 0; ky = 1 + (m - 2 * FX); }
        else { kx = FX - 1; ky = 1 + (m - 2 * FX - SY); }
        ko = ky * FX + kx;
    }
    auto src_to_phi = [](int h) { return (h / SX + 1) * FX + (h % SX + 1); };
    auto xy_src = [&](int h) -> int64_t {
        return g.lay.xy(wrap_coord(x0 - 1 + h % SX, g.nx), wrap_coord(y0 - 1 + h / SX, g.ny));
    };
    const int64_t own_xy = xy_src(h0);
    const int64_t ring_xy = has_ring ? xy_src(hr) : 0;
    // Offsets of the force arrays (public layout) of the two source nodes.
    auto lin_src = [&](int h) -> int64_t {
        return (int64_t)wrap_coord(x0 - 1 + h % SX, g.nx) + (int64_t)g.nx * wrap_coord(y0 - 1 + h / SX, g.ny);
    };
    const int64_t own_lin = FORCE ? lin_src(h0) : 0;
    const int64_t ring_lin = FORCE && has_ring ? lin_src(hr) : 0;
    const int64_t plane_lin = (int64_t)g.nx * g.ny;
    const int64_t outer_xy =
        has_outer ? g.lay.xy(wrap_coord(x0 - 2 + ko % FX, g.nx), wrap_coord(y0 - 2 + ko / FX, g.ny))
                  : 0;
    const int k_own = src_to_phi(h0), k_ring = src_to_phi(hr);

    using M11 = Moments<R, 11>;
    struct PlaneRegs {
        M11 own, ring;
        R outer_dr, outer_r1;
        R fox, foy, foz, frx, fry, frz;  // force at the two source nodes (FORCE)
    };
    PlaneRegs pa, pb;
    auto zwrap = [&](int p) { return p < 0 ? p + g.nz : (p >= g.nz ? p - g.nz : p); };
    auto fetch = [&](int p, PlaneRegs &r) {
        const int64_t zo = (int64_t)zwrap(p) * plane;
        load_moments<R, 11>(in, kBlock, own_xy + zo, r.own);
        if (has_ring) load_moments<R, 11>(in, kBlock, ring_xy + zo, r.ring);
        if (has_outer) {
            r.outer_dr = in[outer_xy + zo];
            r.outer_r1 = in[kBlock + outer_xy + zo];
        }
        if (FORCE) {
            const int64_t zl = (int64_t)zwrap(p) * plane_lin;
            r.fox = frc[own_lin + zl];
            r.foy = frc[g.N + own_lin + zl];
            r.foz = frc[2 * g.N + own_lin + zl];
            if (has_ring) {
                r.frx = frc[ring_lin + zl];
                r.fry = frc[g.N + ring_lin + zl];
                r.frz = frc[2 * g.N + ring_lin + zl];
            }
        }
    };
    auto phi_of = [](R dr, R r1) { return fma_(R(2) * r1, reciprocal<R>(R(1) + dr), R(-1)); };
    auto slot_of = [&](int p) { return (p - z0 + 2) % 3; };
    auto write_phi = [&](int p, const PlaneRegs &r) {
        R *ph = lds_phi + slot_of(p) * FN;
        ph[k_own] = phi_of(r.own.v[0], r.own.v[1]);
        if (has_ring) ph[k_ring] = phi_of(r.ring.v[0], r.ring.v[1]);
        if (has_outer) ph[ko] = phi_of(r.outer_dr, r.outer_r1);
    };

    CgAcc<R> acc[3];
    acc[0].zero();
    acc[1].zero();
    acc[2].zero();

    // Collides one source node (region slot h) and publishes h~ and f1.
    auto publish = [&](int p, const M11 &v, int h, R *own_h, R *own_f, R fx, R fy, R fz) {
        const int kc = src_to_phi(h);
        const R *phm = lds_phi + slot_of(p - 1) * FN;
        const R *ph0 = lds_phi + slot_of(p) * FN;
        const R *php = lds_phi + slot_of(p + 1) * FN;
        // G = 3 sum_i w_i c_i phi(y + c_i): the signed phi values are summed
        // per weight class (faces, edges, corners) and scaled once per class.
        R gf[3] = {R(0), R(0), R(0)}, ge[3] = {R(0), R(0), R(0)}, gc[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                for (int cx = -1; cx <= 1; ++cx) {
                    if ((cx == 0 && cy == 0 && cz == 0) || !has_dir<Q>(cx, cy, cz)) continue;
                    const R *ph = cz < 0 ? phm : (cz == 0 ? ph0 : php);
                    const R f = ph[kc + cy * FX + cx];
                    const int cls = cx * cx + cy * cy + cz * cz;
                    R *acc_c = cls == 1 ? gf : (cls == 2 ? ge : gc);
                    if (cx != 0) acc_c[0] = cx > 0 ? acc_c[0] + f : acc_c[0] - f;
                    if (cy != 0) acc_c[1] = cy > 0 ? acc_c[1] + f : acc_c[1] - f;
                    if (cz != 0) acc_c[2] = cz > 0 ? acc_c[2] + f : acc_c[2] - f;
                }
        constexpr double w3f = 3.0 * weight<Q>(1, 0, 0), w3e = 3.0 * weight<Q>(1, 1, 0), w3c = 3.0 * weight<Q>(1, 1, 1);
        R Gv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Gv[a] = fma_(R(w3e), ge[a], R(w3f) * gf[a]);
            if (Q == 27) Gv[a] = fma_(R(w3c), gc[a], Gv[a]);
        }
        const R Gx = Gv[0], Gy = Gv[1], Gz = Gv[2];
        const R G2 = fma_(Gx, Gx, fma_(Gy, Gy, Gz * Gz));
        const R invD = rsqrt_<R>(G2 + R(kEpsG * kEpsG));
        const R nx = Gx * invD, ny = Gy * invD, nz = Gz * invD;

        const R dr = v.v[0], r1 = v.v[1];
        Collided<R> c;
        if (FORCE) {
            // Guo's forcing: equilibrium at j* = j + F/2, source (1 - omega/2)(u* F + F u*).
            const R jsx = fma_(R(0.5), fx, v.v[2]), jsy = fma_(R(0.5), fy, v.v[3]), jsz = fma_(R(0.5), fz, v.v[4]);
            c = collide<R>(dr, jsx, jsy, jsz, v.v[5], v.v[6], v.v[7], v.v[8], v.v[9], v.v[10], omega);
            const R k = (R(1) - R(0.5) * omega) * reciprocal<R>(R(1) + dr);
            const R kx = k * jsx, ky = k * jsy, kz = k * jsz;
            c.sxx = fma_(R(2) * kx, fx, c.sxx);
            c.syy = fma_(R(2) * ky, fy, c.syy);
            c.szz = fma_(R(2) * kz, fz, c.szz);
            c.sxy = fma_(kx, fy, fma_(ky, fx, c.sxy));
            c.sxz = fma_(kx, fz, fma_(kz, fx, c.sxz));
            c.syz = fma_(ky, fz, fma_(kz, fy, c.syz));
            c.jx = v.v[2] + fx;
            c.jy = v.v[3] + fy;
            c.jz = v.v[4] + fz;
        } else {
            c = collide<R>(dr, v.v[2], v.v[3], v.v[4], v.v[5], v.v[6], v.v[7], v.v[8], v.v[9], v.v[10], omega);
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

        const R inv_rho = reciprocal<R>(R(1) + dr);
        const R a = r1 * inv_rho;                             // rho1/rho
        const R B = beta * (a * (R(1) + dr - r1));            // beta rho1 rho2/rho
        Layer<R> L[3];
        reconstruct_layer<Q, -1, R>(c, L[0]);
        reconstruct_layer<Q, 0, R>(c, L[1]);
        reconstruct_layer<Q, 1, R>(c, L[2]);
        // Moving directions; the rest population takes what is left of rho1,
        // so that each node emits exactly its species-1 mass (the identity
        // sum_i f1_i = rho1 holds in exact arithmetic: the weights sum to one
        // and the recolouring terms cancel in +-c pairs).
        // f1_i = (rho1/rho) (w_i + h~_i) + B w_i (c_i.n)/|c_i|, written as
        // fma(B w_i/|c_i|, c_i.n, fma(rho1/rho, h~_i, (rho1/rho) w_i)) with the
        // per-class products and the in-plane sums n_a +- n_b formed once.
        constexpr double wf = weight<Q>(1, 0, 0), we = weight<Q>(1, 1, 0), wc = weight<Q>(1, 1, 1);
        const R awf = a * R(wf), awe = a * R(we), awc = a * R(wc);
        const R bwf = B * R(wf), bwe = B * R(we * inv_speed<Q>(1, 1, 0)), bwc = B * R(wc * inv_speed<Q>(1, 1, 1));
        const R sxy = nx + ny, dxy = nx - ny, sxz = nx + nz, dxz = nx - nz, syz = ny + nz, dyz = ny - nz;
        R f1_moving = R(0);
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
            for (int sl = 0; sl < 9; ++sl) {
                const int cx = sl % 3 - 1, cy = sl / 3 - 1;
                if (!has_dir<Q>(cx, cy, cz) || (cx == 0 && cy == 0 && cz == 0)) continue;
                const R hv = L[cz + 1].v[sl];
                const int cls = cx * cx + cy * cy + cz * cz;
                R cn;
                if (cls == 1) {
                    cn = cx ? (cx > 0 ? nx : -nx) : cy ? (cy > 0 ? ny : -ny) : (cz > 0 ? nz : -nz);
                } else if (cls == 2) {
                    if (cz == 0) cn = cx == cy ? (cx > 0 ? sxy : -sxy) : (cx > 0 ? dxy : -dxy);
                    else if (cy == 0) cn = cx == cz ? (cx > 0 ? sxz : -sxz) : (cx > 0 ? dxz : -dxz);
                    else cn = cy == cz ? (cy > 0 ? syz : -syz) : (cy > 0 ? dyz : -dyz);
                } else {
                    const R t = cy == cx ? sxy : dxy;  // cx nx + cy ny, up to the sign of cx
                    const R txy = cx > 0 ? t : -t;
                    cn = cz > 0 ? txy + nz : txy - nz;
                }
                const R aw = cls == 1 ? awf : (cls == 2 ? awe : awc);
                const R bw = cls == 1 ? bwf : (cls == 2 ? bwe : bwc);
                const R f1 = fma_(bw, cn, fma_(a, hv, aw));
                f1_moving += f1;
                const int s = lds_slot<Q>(cz, sl);
                if (s >= 0) {
                    lds_h[s * SN + h] = hv;
                    lds_f[s * SN + h] = f1;
                } else if (own_h) {  // own column (0, 0, +-1)
                    own_h[cz + 1] = hv;
                    own_f[cz + 1] = f1;
                }
            }
        if (own_h) {
            own_h[1] = L[1].v[4];
            own_f[1] = r1 - f1_moving;
        }
    };

    auto pull_layer = [&](auto czc, R oh, R of) {
        constexpr int CZ = decltype(czc)::value;
        Layer<R> fh;
        R r1 = of;
#pragma unroll
        for (int sl = 0; sl < 9; ++sl) {
            const int cx = sl % 3 - 1, cy = sl / 3 - 1;
            if (sl == 4) {
                fh.v[sl] = oh;
            } else if (lds_slot<Q>(CZ, sl) >= 0) {
                const int idx = lds_slot<Q>(CZ, sl) * SN + h0 - cy * SX - cx;
                fh.v[sl] = lds_h[idx];
                r1 += lds_f[idx];
            }
        }
        accumulate_layer<Q, CZ, R>(acc[CZ + 1].m, fh);
        acc[CZ + 1].rho1 += r1;
    };

    auto plane_step = [&](int p, PlaneRegs &cur, PlaneRegs &nxt) {
        write_phi(p + 1, nxt);
        __syncthreads();
        R oh[3], of[3];
        publish(p, cur.own, h0, oh, of, cur.fox, cur.foy, cur.foz);
        if (has_ring) publish(p, cur.ring, hr, nullptr, nullptr, cur.frx, cur.fry, cur.frz);
        __syncthreads();
        if (p + 2 <= z_end + 1) fetch(p + 2, cur);
        pull_layer(std::integral_constant<int, -1>(), oh[0], of[0]);
        pull_layer(std::integral_constant<int, 0>(), oh[1], of[1]);
        pull_layer(std::integral_constant<int, 1>(), oh[2], of[2]);

        const int d = p - 1;
        if (d >= z0 && active) {
            const int64_t o = g.lay.xy(x0 + lx, y0 + ly) + (int64_t)d * plane;
            const MomentAcc<R> &a = acc[0].m;
            const R m3 = R(-1.0 / 3.0);
            store_out(out + o, a.r);
            store_out(out + kBlock + o, acc[0].rho1);
            store_out(out + 2 * kBlock + o, a.jx);
            store_out(out + 3 * kBlock + o, a.jy);
            store_out(out + 4 * kBlock + o, a.jz);
            store_out(out + 5 * kBlock + o, fma_(m3, a.r, a.mxx));
            store_out(out + 6 * kBlock + o, fma_(m3, a.r, a.myy));
            store_out(out + 7 * kBlock + o, fma_(m3, a.r, a.mzz));
            store_out(out + 8 * kBlock + o, a.mxy);
            store_out(out + 9 * kBlock + o, a.mxz);
            store_out(out + 10 * kBlock + o, a.myz);
            if (FORCE) phi_out[(x0 + lx) + (int64_t)g.nx * ((y0 + ly) + (int64_t)g.ny * d)] = phi_of(a.r, acc[0].rho1);
        }
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2].zero();
    };

    // Prologue: phase field of planes z0-2 and z0-1, moments of z0-1 and z0.
    fetch(z0 - 2, pa);
    write_phi(z0 - 2, pa);
    fetch(z0 - 1, pa);
    fetch(z0, pb);
    write_phi(z0 - 1, pa);
    for (int p = z0 - 1; p <= z_end; p += 2) {
        plane_step(p, pa, pb);
        if (p + 1 <= z_end) plane_step(p + 1, pb, pa);
    }
}

template <int Q, class R, int TX, int TY, int WG_PER_CU>
hipError_t run(const lbm_ctx *c, const void *in, void *out, bool phi_cached)
{
    TileGrid g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.N = c->N;
    g.lay = c->lay;
    g.tiles_x = (c->nx + TX - 1) / TX;
    g.tiles_y = (c->ny + TY - 1) / TY;
    g.zchunk = choose_zchunk(c->nz, g.tiles_x * g.tiles_y, 256 * WG_PER_CU);
    g.chunks = (c->nz + g.zchunk - 1) / g.zchunk;
    const int64_t blocks = (int64_t)g.tiles_x * g.tiles_y * g.chunks;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (c->nc_A != 0.0) {
        // Near-contact force of this state first (into the context's scratch:
        // F, then the phase field, reused when the previous step wrote it).
        R *phi = static_cast<R *>(c->scratch_nc) + 3 * c->N;
        hipError_t e = phi_cached ? launch_nc_force(c, nullptr, phi) : launch_nc_force(c, in, nullptr);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cg_tile<Q, R, TX, TY, true>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                           static_cast<const R *>(in), static_cast<R *>(out), g, (R)c->omega, (R)(c->A / 9.0),
                           (R)c->beta, static_cast<const R *>(c->scratch_nc), phi);
    } else {
        hipLaunchKernelGGL((k_cg_tile<Q, R, TX, TY, false>), dim3((unsigned)blocks), dim3(TX * TY), 0, c->stream,
                           static_cast<const R *>(in), static_cast<R *>(out), g, (R)c->omega, (R)(c->A / 9.0),
                           (R)c->beta, nullptr, nullptr);
    }
    return hipGetLastError();
}

} // namespace

// D3Q19 FP32 tiles: 64 x 4 nodes (full 64-wide rows of the stored blocks),
// z-chunks sized for two resident workgroups per CU (on 512 x 256 x 256 each
// workgroup marches the whole column).  Measured against 32 x 8, 64 x 8,
// 32 x 16 and 128 x 4 tiles and other chunkings; the shape is a compile-time
// choice (LBM_CG_TX, LBM_CG_TY, LBM_CG_WG).
#ifndef LBM_CG_TX
#define LBM_CG_TX 64
#define LBM_CG_TY 4
#define LBM_CG_WG 2
#endif

hipError_t launch_cg_step(const lbm_ctx *c, const void *in, void *out, bool phi_cached)
{
    if (c->species != 2) return hipErrorNotSupported;
    if (c->storage == LBM_STORE_F32)
        return c->q == 19 ? run<19, float, LBM_CG_TX, LBM_CG_TY, LBM_CG_WG>(c, in, out, phi_cached)
                          : run<27, float, 32, 8, 2>(c, in, out, phi_cached);
    if (c->storage == LBM_STORE_F64)
        return c->q == 19 ? run<19, double, 32, 4, 2>(c, in, out, phi_cached)
                          : run<27, double, 32, 4, 2>(c, in, out, phi_cached);
    return hipErrorInvalidValue;
}

} // namespace lbm
