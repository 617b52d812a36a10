/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann library without populations.
 *
 * The library advances a lattice Boltzmann fluid whose nodes store only the
 * hydrodynamic moments H = [rho, rho u_a, P_ab] (Eqs. 1-3 of Tiribocchi et
 * al., "Lightweight Lattice Boltzmann"), never the populations.  Every time
 * step rebuilds the populations of each node from its moments with the
 * second-order Hermite reconstruction (Eq. 4: equilibrium part Eq. 5 plus
 * non-equilibrium part Eq. 6, ghosts dropped), relaxes them with BGK
 * (Eqs. 7-8), streams them by pulling from the neighbours (Eq. 9) and stores
 * the moments of the streamed set (Eqs. 1-3) in a second copy of the arrays
 * (the flip-flop pair of Sec. III.A).  For one species the library by
 * default carries each tile of the box through two consecutive steps per
 * pass over the state (lbm_opts.steps_per_sweep), with the same results as
 * two single steps.  Two-component fluids follow the colour-gradient model
 * the paper uses (Sec. III.A): one density per species on a shared momentum
 * and pressure tensor, with perturbation and recolouring applied after the
 * collision, optionally with the near-contact force of the LBNCI extension
 * (Sec. III.B, lbm_opts.nc_A).
 *
 * For comparison the same context can instead run a conventional
 * population-storing BGK scheme (LBM_SCHEME_POPULATION, two copies, or
 * LBM_SCHEME_POPULATION_AA, in place), the "LB with populations" of Sec. IV.A,
 * or the moment scheme as the paper's split approach (lbm_opts.split).
 *
 * Conventions shared by every entry point
 *   - Box: nx*ny*nz nodes, fully periodic, node index n = x + nx*(y + ny*z).
 *   - Lattice: D3Q19 (the paper's) or D3Q27, c_s^2 = 1/3, nu = c_s^2 (tau - 1/2).
 *   - Public moment layout (lbm_fields): structure of arrays, field k starts
 *     at base + k*field_stride elements, each field holds N = nx*ny*nz
 *     contiguous values.  Field order:
 *       one species : rho, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz   (10)
 *       two species : rho1, rho2, jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz (11)
 *     with j = rho u the momentum density and P the full second moment.
 *     The moments are the post-streaming (pre-collision) ones.
 *   - All calls are asynchronous on the context's HIP stream unless stated.
 *     A context is not thread-safe; use one per stream.
 *   - Errors: every int-returning call returns LBM_OK (0) or a negative
 *     LBM_E* code; lbm_last_error() then holds a message.  No call aborts the
 *     process and no C++ exception crosses this interface.
 *   - Ownership: the library owns the context and every buffer it allocates;
 *     buffers passed in lbm_fields stay owned by the caller.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ----------------------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* bad argument (size, lattice, tau <= 1/2, ...) */
#define LBM_ENOMEM (-2)    /* device allocation failed */
#define LBM_EDEVICE (-3)   /* a HIP call failed; text in lbm_last_error */
#define LBM_EUNSTABLE (-4) /* a global FP64 check found a non-finite mass or momentum */
#define LBM_ESTATE (-5)    /* call not valid for this context (scheme, species, ...) */

/* ---- schemes and storage formats ------------------------------------------------- */
#define LBM_SCHEME_MOMENT 0     /* the paper's method: moments only (default) */
#define LBM_SCHEME_POPULATION 1 /* population-storing BGK, A-B buffers (baseline); two species:
                                   colour-gradient LB with 2q stored populations, FP32 */
#define LBM_SCHEME_POPULATION_AA 2 /* population-storing BGK in place (AA pattern: one copy of the
                                      q arrays, steps alternate between a neighbour-access and a
                                      node-local update); one species, FP32 or FP64; the stronger
                                      memory baseline.  lbm_save_state / lbm_load_state /
                                      lbm_step_state and the adjoint return LBM_ESTATE */

/* Device storage of the moment state.  All formats store deviations from the
 * rest state rho = 1, u = 0: delta_rho = rho - 1, j, and
 * S = (P - rho c_s^2 I) * s_pi; two-component states store delta_rho of the
 * mixture and rho1.  Arithmetic is FP64 for LBM_STORE_F64 and FP32 otherwise. */
#define LBM_STORE_F64 0
#define LBM_STORE_F32 1
#define LBM_STORE_F16 2  /* IEEE binary16, round to nearest even */
#define LBM_STORE_BF16 3 /* bfloat16, round to nearest even */

/* Element types of caller buffers. */
#define LBM_DTYPE_F64 0
#define LBM_DTYPE_F32 1

typedef struct lbm_ctx lbm_ctx;

typedef struct {
    int nx, ny, nz; /* each >= 3 */
} lbm_grid;

typedef struct {
    int scheme;      /* LBM_SCHEME_*; default LBM_SCHEME_MOMENT */
    int storage;     /* LBM_STORE_*; default LBM_STORE_F32 (population scheme: F32 or F64) */
    double beta;     /* recolouring strength, two species; default 0.7 */
    double sigma;    /* surface tension, two species; default 0.01 (A = 9 sigma / (2 tau)) */
    double s_pi;     /* scale of the stored S; 0 = default (1024 for F16, 1 otherwise).  A
                        power of two for one species with F16/BF16 moment storage; 0 or 1
                        for every other context (else LBM_EINVAL) */
    void *stream;    /* hipStream_t to run on; NULL = the null stream */
    int device;      /* HIP device ordinal; -1 = current device */
    int check_every; /* lbm_step runs the FP64 check every this many steps; 0 = never */
    int split;       /* 0 (default): fused step, one kernel.  1: the paper's split approach
                        (Sec. III.A), for comparison: a collision pass relaxes the stored moments
                        in place (rho, j, S) -> (rho, j, S'), then the streaming pass
                        reconstructs, pulls and sums; two species add a phase-field pass
                        before the collision pass, which also applies the perturbation (and
                        the near-contact force) and writes the interface normal for the
                        streaming pass's recolouring (scratch of 4 N reals).  Moment scheme
                        only (else LBM_EINVAL); results equal the fused step's bit for bit
                        with FP32/FP64 storage (16-bit storage rounds the stored S'); stored
                        values moved per node: 36 instead of 20 (one species), 49 (52 with
                        the near-contact force) instead of 22 (two species); lbm_step_state
                        gives LBM_ESTATE */
    int steps_per_sweep; /* time steps lbm_step applies per pass over the state: 1, or 2 (two
                        steps carried through each tile in one pass, the state read and written
                        once per two steps; results equal single steps bit for bit).  2 needs
                        one species, the moment scheme, the fused step, FP32/FP16/BF16
                        storage and one stored xy-plane below 2 GiB (else LBM_EINVAL).  0 (default): 2 where available, else 1.
                        lbm_step falls back to single steps for an odd remainder and where
                        a check_every health check falls between the two steps */
    double nc_A;     /* near-contact force of the LBNCI extension (Sec. III.B), two species:
                        F = -A_h n delta_I, read as F = (nc_A/2) G at nodes from which a film
                        of species 2 is crossed into another drop within nc_hmax nodes along
                        the lattice direction closest to the outward normal, 0 elsewhere
                        (G the colour gradient); added to the mixture collision with Guo's
                        forcing.  0 (default) = off.  Non-zero needs two species,
                        1 <= nc_hmax <= 32, nz <= 65535 and ny <= 262140 (else
                        LBM_EINVAL); the context then holds a
                        scratch of 3 N reals (moment scheme 4 N) and the adjoint entry
                        points give LBM_ESTATE */
    int nc_hmax;     /* probe range of the near-contact force, nodes */
    void *state_buffers[2]; /* optional caller-owned device buffers for the two state copies
                        (flip-flop pair; the in-place population scheme uses only [0]), e.g.
                        allocated by the caller's framework.  NULL (default): the library
                        allocates them.  Each must hold state_buffer_bytes >=
                        lbm_state_bytes_for() bytes on the context's device and stay valid
                        until lbm_destroy; the library overwrites them (the fluid starts at
                        rest) and never frees them.  Both NULL or both set (LBM_EINVAL) */
    int64_t state_buffer_bytes; /* size of each buffer in state_buffers */
} lbm_opts;

/* Caller-owned moment buffers, see the layout above. */
typedef struct {
    void *base;           /* first element of field 0 */
    int64_t field_stride; /* elements between the starts of consecutive fields (>= N) */
    int dtype;            /* LBM_DTYPE_F32 or LBM_DTYPE_F64 */
    int on_device;        /* 1: device memory of the context's device; 0: host memory */
} lbm_fields;

/* Fills *opts with the defaults listed above.  NULL-safe. */
void lbm_default_opts(lbm_opts *opts);

/* Creates a context: validates the arguments, allocates the two state copies
 * (flip-flop, Sec. III.A) on the device and initialises the fluid at rest
 * (rho = 1, u = 0, P = c_s^2 I; with two species, species 2 fills the box).
 *   grid    : box size, every side >= 3
 *   lattice : 19 or 27
 *   tau     : BGK relaxation time (Eq. 7, omega = 1/tau), > 1/2
 *   species : 1, or 2 for the colour-gradient mixture (moment scheme with
 *             FP32/FP64 storage and one stored xy-plane of the 11 fields below
 *             2 GiB, or population scheme with FP32 storage).  Two species: phase field
 *             phi = (rho1 - rho2)/rho, colour gradient
 *             G = (1/c_s^2) sum_i w_i c_i phi(x + c_i), perturbation with second
 *             moment (A/9)(G G - |G|^2 I)/D, A = 9 sigma/(2 tau), recolouring
 *             beta (rho1 rho2/rho) w_i (c_i.n)/|c_i| (operators the paper names
 *             in Sec. III.A; sigma = 2 A tau / 9 is the surface tension of the
 *             interfacial force F_surf of Sec. III.B), n = G/D, with the
 *             smoothed norm D = sqrt(|G|^2 + 1e-6)
 *   opts    : NULL for the defaults
 * On success *out holds the context; on failure *out is NULL.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE. */
int lbm_create(lbm_ctx **out, lbm_grid grid, int lattice, double tau, int species, const lbm_opts *opts);

/* Frees the context and everything the library allocated.  NULL-safe.
 * Synchronises the stream first. */
int lbm_destroy(lbm_ctx *ctx);

/* Replaces the state by the given moments (public layout above; the moments
 * are post-streaming ones).  For the population scheme the populations are
 * rebuilt from them with Eq. 4.  Host buffers are copied before return.
 * Errors: LBM_EINVAL (NULL, bad dtype or stride), LBM_EDEVICE. */
int lbm_set_moments(lbm_ctx *ctx, const lbm_fields *in);

/* Writes the current moments (Eqs. 1-3 of the post-streaming set) to a
 * caller buffer in the public layout.  Synchronises the stream when the
 * destination is host memory.  Errors: LBM_EINVAL, LBM_EDEVICE. */
int lbm_get_moments(const lbm_ctx *ctx, lbm_fields *out);

/* The equilibrium moments of primitive fields, written to a caller buffer
 * (the context's state is not touched): the map from an initial density and
 * velocity field to an initial state with zero non-equilibrium part,
 * rho^k, j = rho u, P = rho c_s^2 I + rho u u (the moments of the
 * equilibrium populations of Eq. 5).
 *   primitive : rho (one species) or rho1, rho2 (two species), then ux, uy,
 *               uz; lbm_fields layout, F32 or F64, host or device
 *   moments   : receives the public moment fields (10 or 11), F32 or F64,
 *               host or device
 * Arithmetic in FP64, one rounding at the store.  Asynchronous for device
 * buffers; with a host buffer the call synchronises the stream.
 * Errors: LBM_EINVAL (NULL, bad dtype or stride), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_equilibrium_moments(lbm_ctx *ctx, const lbm_fields *primitive, lbm_fields *moments);

/* Transpose of the Jacobian of lbm_equilibrium_moments at `primitive`,
 * applied to a gradient with respect to the moments: the chain from dL/dM(0)
 * to dL/drho^k and dL/du of the initial fields.  With g_j and g_P the
 * gradients of j and of the six stored P components (an off-diagonal stored
 * component counts once),
 *   dL/drho^k = g_rho^k + u.g_j + sum_ab g_P_ab (u_a u_b + delta_ab c_s^2),
 *   dL/du_c   = rho g_j_c + rho sum_ab g_P_ab (delta_ac u_b + u_a delta_bc).
 *   primitive      : as for lbm_equilibrium_moments
 *   grad_moments   : public moment layout (10 or 11 fields)
 *   grad_primitive : receives species + 3 fields in the primitive layout
 * F32 or F64, host or device each; FP64 arithmetic.  Asynchronous for device
 * buffers; with a host buffer the call synchronises the stream.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE. */
int lbm_equilibrium_moments_adjoint(lbm_ctx *ctx, const lbm_fields *primitive, const lbm_fields *grad_moments,
                                    lbm_fields *grad_primitive);

/* Sets an equilibrium state from primitive fields: the buffer holds
 * rho (one species) or rho1, rho2 (two species) followed by ux, uy, uz; the
 * moments become rho^k, j = rho u and P = rho c_s^2 I + rho u u (the second
 * moment of Eq. 5), i.e. a zero non-equilibrium part.
 * Errors: LBM_EINVAL, LBM_EDEVICE. */
int lbm_set_equilibrium(lbm_ctx *ctx, const lbm_fields *primitive);

/* Advances n >= 0 time steps (one fused kernel launch per step for the moment
 * scheme).  Asynchronous unless check_every > 0, in which case the FP64 check
 * of lbm_reduce runs every check_every steps and the call returns
 * LBM_EUNSTABLE at the first non-finite total.  Errors: LBM_EINVAL,
 * LBM_EDEVICE, LBM_EUNSTABLE. */
int lbm_step(lbm_ctx *ctx, int n);

/* Global totals in FP64, summed on the device in a fixed order:
 * out[0] = sum rho (species 1 for two species), out[1] = sum rho2 (0 for one
 * species), out[2..4] = sum j.  Synchronises the stream.
 * Returns LBM_EUNSTABLE if any total is not finite. */
int lbm_reduce(lbm_ctx *ctx, double out[5]);

/* Bytes of device memory the context holds for its state (both copies with
 * the padding of the blocked layout, plus the phase-field scratch array of
 * the two-species population scheme and the colour-gradient co-state buffer
 * of the two-species adjoint) and the bytes one time step moves at minimum
 * (every stored value of every node read once and written once).  Either
 * pointer may be NULL. */
int lbm_memory_info(const lbm_ctx *ctx, int64_t *state_bytes, int64_t *step_bytes);

/* Bytes of one state copy that lbm_create(grid, lattice, tau, species, opts)
 * would use (the size each of lbm_opts.state_buffers must have), without
 * creating a context.  Errors: LBM_EINVAL (NULL bytes, or a setup
 * lbm_create refuses). */
int lbm_state_bytes_for(lbm_grid grid, int lattice, int species, const lbm_opts *opts, int64_t *bytes);

/* Size in bytes of one time level of the stored state (the buffer that
 * lbm_save_state fills).  The moment scheme stores its fields in an internal
 * blocked layout (the fields of each 64 x 16 block of an xy-plane are
 * contiguous; nx and ny are rounded up to multiples of 64 and 16), so this is
 * at least nfields x N x element size; the population scheme stores q (or 2q)
 * arrays of N values.  Errors: LBM_EINVAL. */
int lbm_state_bytes(const lbm_ctx *ctx, int64_t *bytes);

/* Copies the current time level of the stored state, in its storage format,
 * to / from a caller-owned device buffer of lbm_state_bytes() bytes with the
 * library's streaming copy kernel (used for the adjoint's checkpoints).
 * Asynchronous on the context's stream; a restored state continues bit for
 * bit like the saved one.  Errors: LBM_EINVAL (NULL), LBM_EDEVICE. */
int lbm_save_state(lbm_ctx *ctx, void *dst_device);
int lbm_load_state(lbm_ctx *ctx, const void *src_device);

/* One time step from a saved state to another buffer, both in the format of
 * lbm_save_state (device, lbm_state_bytes() bytes each, must not overlap);
 * the context's own state is not touched.  Used to recompute the states of
 * a checkpointed segment straight into the adjoint's buffers.
 * Errors: LBM_EINVAL, LBM_ESTATE (population scheme), LBM_EDEVICE. */
int lbm_step_state(lbm_ctx *ctx, const void *src_state, void *dst_state);

/* Two time steps from a saved state in one pass (the two-step sweep of
 * lbm_step): mid_state receives the state after the first step, dst_state the
 * state after the second, both bit for bit as two lbm_step_state calls would
 * give them.  Three device buffers of lbm_state_bytes() bytes, pairwise
 * distinct, must not overlap; the context's own state is not touched.
 * Recomputes two states of a checkpointed segment for the cost of about one.
 * Errors: LBM_EINVAL (NULL or aliased), LBM_ESTATE (not one species with
 * the fused moment step and FP32/FP16/BF16 storage), LBM_EDEVICE. */
int lbm_step_state2(lbm_ctx *ctx, const void *src_state, void *mid_state, void *dst_state);

/* One reverse step of the discrete adjoint of the moment scheme: the exact
 * transpose of the Jacobian of one step (one species: Eqs. 4-9 and 1-3; two
 * species: the colour-gradient step of Sec. III.A with the perturbation and
 * recolouring operators of Sec. III.B, smoothed normal, A held at 9 sigma/(2 tau)).
 *   state_t    : the state M(t) the forward step starts from, public moment
 *                layout (10 or 11 fields); it is first converted to the
 *                storage format exactly as lbm_set_moments would store it,
 *                and the step is linearised at that stored state
 *   lam_next   : co-state of M(t+1), public moment layout
 *   lam_out    : receives the co-state of M(t), public moment layout; must
 *                not be the same buffer as lam_next
 *   dtau_accum : host pointer to one double, or NULL; the step's dL/dtau
 *                (sum over nodes in FP64, fixed order; two species: at fixed
 *                sigma, so A varies with tau) is added to it
 * Each buffer may be host or device memory, F32 or F64; the kernels compute
 * in FP64 for LBM_STORE_F64 contexts and FP32 otherwise, and co-states are
 * converted to that type on the way in and rounded to the caller's type on
 * the way out.  A stored off-diagonal P component stands for P_ab and P_ba
 * together, so its co-state is the derivative with respect to that one
 * stored value.  The context's own state is not touched.  The first call
 * allocates a work area the context keeps (one stored state, two stored
 * co-states; two species also a buffer of 3 N reals for the co-state of the
 * colour gradient).  The call synchronises the stream when dtau_accum is
 * non-NULL or a buffer is in host memory.  Two species: FP32 or FP64 storage
 * only.  A checkpointed rollout instead keeps its states in the stored
 * format and its co-states in the stored layout (lbm_adjoint_step_stored).
 * Errors: LBM_EINVAL (NULL, bad dtype or stride, lam_out == lam_next),
 * LBM_ESTATE (population scheme, near-contact force, or two species with
 * FP16/BF16 storage), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_adjoint_step(lbm_ctx *ctx, const lbm_fields *state_t, const lbm_fields *lam_next, lbm_fields *lam_out,
                     double *dtau_accum);

/* The same reverse step on the library's own formats, for checkpointed
 * rollouts: state_t is a device buffer in the format of lbm_save_state;
 * lam_next and lam_out are device buffers of lbm_costate_bytes() bytes in the
 * stored (blocked) layout of the state, with the kernels' real type (FP64 for
 * LBM_STORE_F64, else FP32); dtau_accum is a device pointer to one double or
 * NULL, added to on the stream.  A rollout keeps its co-state in this layout
 * between steps and converts it only at the ends (lbm_costate_to_stored /
 * _from_stored); the results equal those of lbm_adjoint_step from the same
 * stored state bit for bit.  Slots of the layout that belong to no node are
 * neither read nor written.  Asynchronous; the two-species co-state buffer
 * is allocated on the first call as for lbm_adjoint_step.
 * Errors: LBM_EINVAL (NULL, or lam_next == lam_out), LBM_ESTATE, LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_adjoint_step_stored(lbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out,
                            double *dtau_accum);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reverse step as lbm_adjoint_step_stored, same arguments and results bit for
 * bit, calling no hipMalloc, hipFree or allocating library routine.  The
 * two-species step keeps the co-state of the colour gradient (3 N reals, in
 * the blocked layout) in a static device array of 64 MiB instead of the
 * context's lazily allocated buffer; each device the library runs on holds
 * that array from the first lbm_create on it until the process ends.  Every
 * call on one device shares its array: calls that overlap on one device (on
 * different streams or host threads) race, and must be ordered by the
 * caller.  The array is written in full before it is read within each call,
 * so nothing carries over between calls.  One species needs no scratch.
 * Errors: LBM_EINVAL (NULL or aliased buffers, or a two-species box whose
 * colour-gradient co-state exceeds 64 MiB: above about 5.6 M nodes in FP32,
 * 2.8 M in FP64, e.g. 128^3 fits both), LBM_ESTATE (as lbm_adjoint_step_stored),
 * LBM_EDEVICE. */
int lbm_adjoint_step_stored_noalloc(lbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out,
                                    double *dtau_accum);

/* Two reverse steps in one pass, co-states in the stored layout:
 * lam_out = J(state_t0)^T J(state_t1)^T lam_next, where state_t1 is the state
 * one step after state_t0 (both in the format of lbm_save_state), i.e. the
 * same as lbm_adjoint_step_stored(state_t1, lam_next, tmp) followed by
 * lbm_adjoint_step_stored(state_t0, tmp, lam_out), bit for bit in lam_out.
 * dtau_accum (device double or NULL) receives the sum of both steps'
 * contributions (equal to the two single steps' up to FP64 rounding of the
 * grouping).  One species, fused moment step, FP32/FP16/BF16 storage.
 * Errors: LBM_EINVAL (NULL, or lam_next aliasing lam_out), LBM_ESTATE,
 * LBM_EDEVICE. */
int lbm_adjoint_step2_stored(lbm_ctx *ctx, const void *state_t1, const void *state_t0, const void *lam_next,
                             void *lam_out, double *dtau_accum);

/* Size in bytes of one co-state in the stored layout (moment scheme).
 * Errors: LBM_EINVAL, LBM_ESTATE (population scheme). */
int lbm_costate_bytes(const lbm_ctx *ctx, int64_t *bytes);

/* Co-state conversion between the public layout (nfields arrays of N reals,
 * x fastest) and the stored layout (lbm_costate_bytes() bytes); both device
 * buffers, must not overlap.  Asynchronous on the context's stream.
 * Errors: LBM_EINVAL (NULL or aliased), LBM_ESTATE (population scheme),
 * LBM_EDEVICE. */
int lbm_costate_to_stored(lbm_ctx *ctx, const void *public_dev, void *stored_dev);
int lbm_costate_from_stored(lbm_ctx *ctx, const void *stored_dev, void *public_dev);

/* Number of time steps advanced since creation or the last set_* call. */
int64_t lbm_steps_done(const lbm_ctx *ctx);

/* Time steps lbm_step carries through each tile per pass over the state for
 * this context (1 or 2, as resolved from lbm_opts.steps_per_sweep at
 * creation); 2 also means lbm_step_state2 and lbm_adjoint_step2_stored are
 * available.  -1 for NULL. */
int lbm_steps_per_sweep(const lbm_ctx *ctx);

/* Static description of an error code; never NULL. */
const char *lbm_strerror(int code);

/* Message of the last failed call on this context ("" if none); never NULL,
 * valid until the next call on the context.  NULL-safe. */
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
