// Library-internal context and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "layout.hpp"
#include "lbm.h"

struct lbm_ctx {
    int nx = 0, ny = 0, nz = 0;
    int64_t N = 0;
    int q = 19, species = 1, scheme = LBM_SCHEME_MOMENT, storage = LBM_STORE_F32;
    double tau = 1.0, omega = 1.0, beta = 0.7, sigma = 0.0, A = 0.0, s_pi = 1.0;
    hipStream_t stream = nullptr;
    int device = 0;
    int check_every = 0;
    int split = 0;    // moment scheme run as the split approach (collision pass + streaming pass)
    int sweep = 1;    // time steps per pass over the state (1, or 2: two-step sweeps)
    double nc_A = 0.0;  // near-contact force strength (two species; 0 = off)
    int nc_hmax = 0;    // near-contact probe range (nodes)
    void *scratch_nc = nullptr;  // near-contact force (3 N reals), then the moment scheme's phase field (N)
    const void *phi_of = nullptr;  // state whose phase field that scratch holds (moment scheme), or none
    int nfields = 0;  // stored arrays per state copy
    size_t elem = 4;  // bytes per stored element
    int64_t state_elems = 0;  // elements per state copy (blocked moment layout or q x N populations)
    lbm::MomentLayout lay{};  // stored layout of the moment scheme
    lbm::MomentLayout lay3{}; // 3-field blocked layout of the two-species adjoint's scratch
    void *state[2] = {nullptr, nullptr};
    int cur = 0;      // state[cur] holds the current time level
    double *partials = nullptr;  // FP64 reduction partials (kReduceBlocks x 5)
    double *red_out = nullptr;   // 5 device doubles
    float *scratch_phi = nullptr; // phase field of the two-species population scheme
    void *scratch_adj = nullptr;  // co-state of the colour gradient (3 fields, layout lay3), two-species adjoint
    void *scratch_split = nullptr; // split two-species step: phase field (N) and interface normal (3 N)
    void *adj_work = nullptr;     // lbm_adjoint_step: one stored state and two stored co-states
    double *adj_dtau = nullptr;   // lbm_adjoint_step: its dL/dtau term (one device double)
    bool owns_state = true;       // false: the state copies are caller buffers (lbm_opts.state_buffers)
    int64_t steps = 0;
    mutable std::string err;
};

namespace lbm {

constexpr int kReduceBlocks = 1024;

// Moment scheme.  collided: `in` holds post-collision moments (split
// approach), the step only reconstructs, pulls and sums.
hipError_t launch_moment_step(const lbm_ctx *c, const void *in, void *out, bool collided = false);

// Collision pass of the split approach, in place on the stored state.
hipError_t launch_moment_collide(const lbm_ctx *c, void *state);

// Two moment steps in one pass over the state (one species, fused step,
// FP32/FP16/BF16 storage); equal to two launch_moment_step calls bit for bit.
// mid (optional): receives the state after the first step.
bool moment_sweep2_supported(const lbm_ctx *c);
hipError_t launch_moment_sweep2(const lbm_ctx *c, const void *in, void *out, void *mid = nullptr);

// Two adjoint steps (co-states in the stored layout): lam_out =
// J(state_t0)^T J(state_t1)^T lam_in, state_t1 being one step after state_t0.
hipError_t launch_adjoint_sweep2(const lbm_ctx *c, const void *state_t1, const void *state_t0, const void *lam_in,
                                 void *lam_out, double *dtau_accum);

// Moment scheme, two species (colour gradient).
// Two-component moment step.  With the near-contact force the step also
// writes the phase field of its output into the scratch after the force;
// phi_cached says that the scratch already holds the phase field of `in`.
// normal (split schedule): `in` holds post-collision moments and `normal`
// the interface normal (three arrays of N reals); the step only streams.
hipError_t launch_cg_step(const lbm_ctx *c, const void *in, void *out, bool phi_cached = false,
                          const void *normal = nullptr);

// Split schedule of the two-component step (Sec. III.A): a phase-field
// pass, a collision pass that relaxes the stored moments in place (with the
// perturbation, and Guo's forcing of the near-contact force) and writes the
// interface normal, then the streaming pass.  Scratch: c->scratch_split
// (4 N reals: phase field, normal).  Equal to the fused step bit for bit.
hipError_t launch_cg_split_step(const lbm_ctx *c, void *in, void *out);

// Discrete adjoint of the one-species moment step; co-states in the public
// layout, or in the stored (blocked) layout of the state if `stored`.
hipError_t launch_adjoint_step(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out,
                               double *dtau_accum, bool stored);

// Discrete adjoint of the two-species (colour-gradient) moment step; keeps
// the co-state of the colour gradient (3 fields in the blocked layout lay3,
// written in full before it is read) in gG_scratch, or in c->scratch_adj if
// that is NULL.
hipError_t launch_cg_adjoint_step(const lbm_ctx *c, const void *state, const void *lam_in, void *lam_out,
                                  double *dtau_accum, bool stored, void *gG_scratch = nullptr);

// Co-state between the public layout (nfields fields, field k at
// base + k*stride, elements of pub_dtype; stride <= 0: N, pub_dtype < 0: the
// kernels' real type) and the stored blocked layout (state_elems elements of
// the kernels' real type).
hipError_t launch_costate_convert(const lbm_ctx *c, const void *src, void *dst, bool to_stored, int64_t stride = 0,
                                  int pub_dtype = -1);

// Near-contact force of the two-species schemes into c->scratch_nc (three
// arrays of N), from the phase field `phi` (N values, population scheme) or,
// if phi is NULL, from the moment state `moments`.  The scratch must start
// zeroed (nc_scratch_bytes bytes): per-block flags record where the force
// arrays may hold non-zero values.  A block is kNcBlockX x kNcBlockY nodes of
// one plane, block (bx, by) of plane z has index bx + gx (by + gy z) (gx, gy:
// blocks per row and column), and nc_blocks(c) of them follow the sign
// summary at nc_block_flags(c): after each force pass, a block whose flag is
// zero holds zeros in all three force arrays.
constexpr int kNcBlockX = 64, kNcBlockY = 4;
hipError_t launch_nc_force(const lbm_ctx *c, const void *moments, const void *phi);
int64_t nc_blocks(const lbm_ctx *c);
size_t nc_scratch_bytes(const lbm_ctx *c);
uint8_t *nc_block_flags(const lbm_ctx *c);

// Population scheme in place (AA pattern) on the single array `state`; odd:
// the state has gone through an odd number of steps.
hipError_t launch_population_aa_step(const lbm_ctx *c, void *state, bool odd);

// Population scheme.
hipError_t launch_population_step(const lbm_ctx *c, const void *in, void *out);

// Conversions between the public moment layout (dtype F32/F64, device
// pointer, given field stride) and the stored state of either scheme.
hipError_t launch_set_moments(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *state);
hipError_t launch_get_moments(const lbm_ctx *c, const void *state, void *dst, int64_t stride, int dtype);
hipError_t launch_set_equilibrium(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *state);

// Equilibrium moments of primitive fields (rho^k, u) into a public-layout
// buffer (field stride dstride, element type ddtype), and the transpose of
// that map's Jacobian at `prim` applied to a moment gradient `grad`.
hipError_t launch_equilibrium(const lbm_ctx *c, const void *src, int64_t stride, int dtype, void *dst,
                              int64_t dstride, int ddtype);
hipError_t launch_equilibrium_adjoint(const lbm_ctx *c, const void *prim, int64_t pstride, int pdtype,
                                      const void *grad, int64_t gstride, int gdtype, void *out, int64_t ostride,
                                      int odtype);

// Streaming device-to-device copy of `bytes` bytes (16-byte vector accesses).
hipError_t launch_copy(const lbm_ctx *c, const void *src, void *dst, int64_t bytes);

// FP64 totals of the stored state into c->red_out (device, 5 doubles):
// sum of delta_rho (one species) or rho1, sum of delta_rho (two species)
// or 0, sum of j.  The host adds N where the state stores deviations.
hipError_t launch_reduce(const lbm_ctx *c, const void *state);

} // namespace lbm
