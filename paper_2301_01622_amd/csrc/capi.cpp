// C ABI of the library (declared and documented in include/lbm.h).
//
// Host-side only: argument validation, device buffers, stream binding and
// error reporting.  Every step of the method runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>

#include "internal.hpp"

// Static device scratch of lbm_adjoint_step_stored_noalloc: the co-state of
// the colour gradient of the two-species reverse step (3 fields in the
// blocked layout, FP32 or FP64).  Every device the library runs on holds its
// own copy until the process ends.  In host code the name is only a handle
// for hipGetSymbolAddress; kernels receive the device address resolved once
// per device at context creation (scratch_ptr).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (the current device), resolved on the
// first call for that device.  Returns hipSuccess and sets *ptr.
hipError_t scratch_ptr(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

int fail(const lbm_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(const lbm_ctx *c, hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(c, LBM_ENOMEM, m);
    return fail(c, LBM_EDEVICE, m);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t storage_bytes(int storage)
{
    switch (storage) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    case LBM_STORE_F16:
    case LBM_STORE_BF16: return 2;
    default: return 0;
    }
}

int check_fields(const lbm_ctx *c, const lbm_fields *f, int nfields)
{
    if (!f || !f->base) return fail(c, LBM_EINVAL, "fields: NULL buffer");
    if (f->dtype != LBM_DTYPE_F32 && f->dtype != LBM_DTYPE_F64) return fail(c, LBM_EINVAL, "fields: bad dtype");
    if (f->field_stride < c->N) return fail(c, LBM_EINVAL, "fields: field_stride < number of nodes");
    (void)nfields;
    return LBM_OK;
}

// Copies a caller buffer to a fresh device buffer when it is on the host.
// *dev receives a device pointer with the same layout; *owned is set when the
// caller must free it.
int stage_in(const lbm_ctx *c, const lbm_fields *f, int nfields, const void **dev, void **owned)
{
    *owned = nullptr;
    if (f->on_device) {
        *dev = f->base;
        return LBM_OK;
    }
    const size_t bytes = (size_t)(f->dtype == LBM_DTYPE_F64 ? 8 : 4) * (size_t)f->field_stride * (size_t)nfields;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(staging)");
    e = hipMemcpyAsync(d, f->base, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(c, e, "hipMemcpyAsync(host->device)");
    }
    *dev = d;
    *owned = d;
    return LBM_OK;
}

int public_fields(const lbm_ctx *c) { return c->species == 1 ? 10 : 11; }

size_t dtype_bytes(int dtype) { return dtype == LBM_DTYPE_F64 ? 8 : 4; }

// Device view of a caller output buffer: the buffer itself when it is device
// memory, else a fresh device buffer of the same layout (*owned) that
// finish_out copies to the host buffer.
int stage_out(const lbm_ctx *c, const lbm_fields *f, int nfields, void **dev, void **owned)
{
    *owned = nullptr;
    if (f->on_device) {
        *dev = f->base;
        return LBM_OK;
    }
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, dtype_bytes(f->dtype) * (size_t)f->field_stride * (size_t)nfields);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(staging)");
    *dev = d;
    *owned = d;
    return LBM_OK;
}

// Completes a staged output (copy to the host, synchronise) and frees the
// staging buffers; e is the status of the launches so far.
hipError_t finish_io(const lbm_ctx *c, hipError_t e, const lbm_fields *out, int nfields, void *out_owned,
                     void *in_owned_a, void *in_owned_b = nullptr)
{
    if (e == hipSuccess && out_owned)
        e = hipMemcpyAsync(out->base, out_owned, dtype_bytes(out->dtype) * (size_t)out->field_stride * (size_t)nfields,
                           hipMemcpyDeviceToHost, c->stream);
    if (out_owned || in_owned_a || in_owned_b) {
        hipError_t e2 = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = e2;
    }
    if (out_owned) (void)hipFree(out_owned);
    if (in_owned_a) (void)hipFree(in_owned_a);
    if (in_owned_b) (void)hipFree(in_owned_b);
    return e;
}

// Stored arrays per state copy, bytes per stored element and elements per
// copy (blocked moment layout, or q x N populations) for a validated setup.
struct StatePlan {
    int nfields;
    size_t elem;
    int64_t elems;
    int copies;
};

StatePlan state_plan(lbm_grid g, int lattice, int species, const lbm_opts &o)
{
    StatePlan p;
    p.nfields = o.scheme == LBM_SCHEME_MOMENT ? (species == 1 ? 10 : 11) : lattice * species;
    p.elem = storage_bytes(o.storage);
    p.elems = o.scheme == LBM_SCHEME_MOMENT ? lbm::moment_layout(g.nx, g.ny, p.nfields).plane * g.nz
                                            : (int64_t)p.nfields * g.nx * g.ny * g.nz;
    p.copies = o.scheme == LBM_SCHEME_POPULATION_AA ? 1 : 2;
    return p;
}

} // namespace

extern "C" {

void lbm_default_opts(lbm_opts *o)
{
    if (!o) return;
    o->scheme = LBM_SCHEME_MOMENT;
    o->storage = LBM_STORE_F32;
    o->beta = 0.7;
    o->sigma = 0.01;
    o->s_pi = 0.0;
    o->stream = nullptr;
    o->device = -1;
    o->check_every = 0;
    o->split = 0;
    o->steps_per_sweep = 0;
    o->nc_A = 0.0;
    o->nc_hmax = 0;
    o->state_buffers[0] = nullptr;
    o->state_buffers[1] = nullptr;
    o->state_buffer_bytes = 0;
}

const char *lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of device memory";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_EUNSTABLE: return "non-finite global mass or momentum (unstable run)";
    case LBM_ESTATE: return "operation not valid for this context";
    default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

// Validates a setup (every rule of lbm_create except tau and the external
// state buffers); *sweep receives the resolved steps per sweep.
static int validate(lbm_grid grid, int lattice, int species, const lbm_opts &o, int *sweep)
{
    if (grid.nx < 3 || grid.ny < 3 || grid.nz < 3) return LBM_EINVAL;
    if (lattice != 19 && lattice != 27) return LBM_EINVAL;
    if (species != 1 && species != 2) return LBM_EINVAL;
    if (o.scheme != LBM_SCHEME_MOMENT && o.scheme != LBM_SCHEME_POPULATION && o.scheme != LBM_SCHEME_POPULATION_AA)
        return LBM_EINVAL;
    if (o.split != 0 && (o.split != 1 || o.scheme != LBM_SCHEME_MOMENT)) return LBM_EINVAL;
    if (o.scheme == LBM_SCHEME_POPULATION_AA &&
        (species != 1 || (o.storage != LBM_STORE_F32 && o.storage != LBM_STORE_F64)))
        return LBM_EINVAL;
    if (storage_bytes(o.storage) == 0) return LBM_EINVAL;
    if (o.check_every < 0) return LBM_EINVAL;
    if (o.scheme == LBM_SCHEME_POPULATION && o.storage != LBM_STORE_F32 && o.storage != LBM_STORE_F64)
        return LBM_EINVAL;
    if (species == 2 && o.storage != LBM_STORE_F32 && o.storage != LBM_STORE_F64) return LBM_EINVAL;
    if (species == 2 && (!(o.beta >= 0.0) || !(o.sigma >= 0.0))) return LBM_EINVAL;
    if (!(o.s_pi >= 0.0) || !std::isfinite(o.s_pi)) return LBM_EINVAL;
    // The scale of the stored S is applied only where S is stored in 16 bits
    // (one species, moment scheme); elsewhere it must stay 1.  A power of two
    // keeps the scaling exact.
    if (o.s_pi != 0.0) {
        const bool scaled = o.scheme == LBM_SCHEME_MOMENT && species == 1 &&
                            (o.storage == LBM_STORE_F16 || o.storage == LBM_STORE_BF16);
        int e2 = 0;
        if (scaled ? std::frexp(o.s_pi, &e2) != 0.5 : o.s_pi != 1.0) return LBM_EINVAL;
    }
    if (species == 2 && o.scheme == LBM_SCHEME_POPULATION && o.storage != LBM_STORE_F32) return LBM_EINVAL;
    // The two-component moment step addresses one stored z-plane (11 fields)
    // per buffer descriptor: at most 2 GiB.
    if (species == 2 && o.scheme == LBM_SCHEME_MOMENT &&
        lbm::moment_layout(grid.nx, grid.ny, 11).plane * (int64_t)storage_bytes(o.storage) >= ((int64_t)1 << 31))
        return LBM_EINVAL;

    // Near-contact force: two species only, finite strength, 1..32 probes;
    // its per-node passes launch one block row per z-plane and 4 rows of y
    // per block, within the grid's 65535 limit.
    if (o.nc_A != 0.0 && (species != 2 || !std::isfinite(o.nc_A) || o.nc_hmax < 1 || o.nc_hmax > 32 ||
                          grid.nz > 65535 || (grid.ny + 3) / 4 > 65535))
        return LBM_EINVAL;
    // Two-step sweeps: one species, fused moment step, not FP64 storage.
    // The sweep addresses one z-plane (at most 2 GiB) per buffer descriptor.
    const bool sweep2_ok = o.scheme == LBM_SCHEME_MOMENT && species == 1 && o.split == 0 &&
                           o.storage != LBM_STORE_F64 &&
                           lbm::moment_layout(grid.nx, grid.ny, 10).plane * (int64_t)storage_bytes(o.storage) <
                               ((int64_t)1 << 31);
    if (o.steps_per_sweep < 0 || o.steps_per_sweep > 2 || (o.steps_per_sweep == 2 && !sweep2_ok)) return LBM_EINVAL;
    *sweep = o.steps_per_sweep == 0 ? (sweep2_ok ? 2 : 1) : o.steps_per_sweep;
    return LBM_OK;
}

int lbm_create(lbm_ctx **out, lbm_grid grid, int lattice, double tau, int species, const lbm_opts *opts)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_opts o;
    lbm_default_opts(&o);
    if (opts) o = *opts;
    if (!(tau > 0.5) || !std::isfinite(tau)) return LBM_EINVAL;
    int sweep = 1;
    if (validate(grid, lattice, species, o, &sweep) != LBM_OK) return LBM_EINVAL;
    const StatePlan plan = state_plan(grid, lattice, species, o);
    // Caller-owned state copies: both given (one for the in-place scheme),
    // each large enough, or none.
    const bool external = o.state_buffers[0] || o.state_buffers[1];
    if (external) {
        const bool pair_ok = plan.copies == 1 || (o.state_buffers[1] && o.state_buffers[1] != o.state_buffers[0]);
        if (!o.state_buffers[0] || !pair_ok || o.state_buffer_bytes < (int64_t)plan.elem * plan.elems)
            return LBM_EINVAL;
    }
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->nx = grid.nx;
    c->ny = grid.ny;
    c->nz = grid.nz;
    c->N = (int64_t)grid.nx * grid.ny * grid.nz;
    c->q = lattice;
    c->species = species;
    c->scheme = o.scheme;
    c->storage = o.storage;
    c->tau = tau;
    c->omega = 1.0 / tau;
    c->beta = o.beta;
    c->sigma = o.sigma;
    c->A = 9.0 * o.sigma / (2.0 * tau);
    c->s_pi = o.s_pi > 0.0 ? o.s_pi : (o.storage == LBM_STORE_F16 ? 1024.0 : 1.0);
    c->stream = static_cast<hipStream_t>(o.stream);
    c->check_every = o.check_every;
    c->split = o.split;
    c->sweep = sweep;
    c->nc_A = o.nc_A;
    c->nc_hmax = o.nc_A != 0.0 ? o.nc_hmax : 0;
    c->elem = plan.elem;
    c->nfields = plan.nfields;
    c->lay = lbm::moment_layout(c->nx, c->ny, c->nfields);
    c->lay3 = lbm::moment_layout(c->nx, c->ny, 3);
    c->state_elems = plan.elems;

    if (o.device >= 0) {
        c->device = o.device;
    } else if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBM_EDEVICE;
    }
    DeviceGuard g(c->device);
    // The static scratch of the allocation-free entry point, once per device.
    void *sp = nullptr;
    if (scratch_ptr(c->device, &sp) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return LBM_EDEVICE;
    }
    const size_t bytes = c->elem * (size_t)c->state_elems;
    const int copies = plan.copies;  // in place: one copy
    c->owns_state = !external;
    for (int k = 0; k < copies; ++k) {
        if (external) {
            c->state[k] = o.state_buffers[k];
            continue;
        }
        hipError_t e = hipMalloc(&c->state[k], bytes);
        if (e != hipSuccess) {
            lbm_destroy(c);
            return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
        }
    }
    if (c->scheme == LBM_SCHEME_POPULATION && species == 2 &&
        hipMalloc((void **)&c->scratch_phi, sizeof(float) * (size_t)c->N) != hipSuccess) {
        lbm_destroy(c);
        return LBM_ENOMEM;
    }
    // Near-contact force (3 N), for the moment scheme its phase field (N), and
    // two bytes per force block; zeroed (the force passes rewrite only blocks
    // whose flags say they may hold non-zero values).
    if (c->nc_A != 0.0) {
        if (hipMalloc(&c->scratch_nc, lbm::nc_scratch_bytes(c)) != hipSuccess) {
            c->scratch_nc = nullptr;
            lbm_destroy(c);
            return LBM_ENOMEM;
        }
        if (hipMemsetAsync(c->scratch_nc, 0, lbm::nc_scratch_bytes(c), c->stream) != hipSuccess) {
            lbm_destroy(c);
            return LBM_EDEVICE;
        }
    }
    // Split two-species step: phase field (N) and interface normal (3 N).
    if (c->split && species == 2 && hipMalloc(&c->scratch_split, c->elem * 4 * (size_t)c->N) != hipSuccess) {
        c->scratch_split = nullptr;
        lbm_destroy(c);
        return LBM_ENOMEM;
    }
    if (hipMalloc((void **)&c->partials, sizeof(double) * 5 * lbm::kReduceBlocks) != hipSuccess ||
        hipMalloc((void **)&c->red_out, sizeof(double) * 5) != hipSuccess) {
        lbm_destroy(c);
        return LBM_ENOMEM;
    }
    // Fluid at rest: every stored deviation is zero (for two species rho1 = 0:
    // species 2 fills the box).
    for (int k = 0; k < copies; ++k) {
        if (hipMemsetAsync(c->state[k], 0, bytes, c->stream) != hipSuccess) {
            lbm_destroy(c);
            return LBM_EDEVICE;
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        lbm_destroy(c);
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *c)
{
    if (!c) return LBM_OK;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k)
        if (c->state[k] && c->owns_state) (void)hipFree(c->state[k]);
    if (c->adj_work) (void)hipFree(c->adj_work);
    if (c->adj_dtau) (void)hipFree(c->adj_dtau);
    if (c->partials) (void)hipFree(c->partials);
    if (c->red_out) (void)hipFree(c->red_out);
    if (c->scratch_phi) (void)hipFree(c->scratch_phi);
    if (c->scratch_nc) (void)hipFree(c->scratch_nc);
    if (c->scratch_adj) (void)hipFree(c->scratch_adj);
    delete c;
    return LBM_OK;
}

int lbm_set_moments(lbm_ctx *c, const lbm_fields *in)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int nf = public_fields(c);
    int rc = check_fields(c, in, nf);
    if (rc) return rc;
    DeviceGuard g(c->device);
    const void *dev = nullptr;
    void *owned = nullptr;
    if ((rc = stage_in(c, in, nf, &dev, &owned))) return rc;
    c->phi_of = nullptr;  // the state changes outside the step
    hipError_t e = lbm::launch_set_moments(c, dev, in->field_stride, in->dtype, c->state[c->cur]);
    if (owned) {
        hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(owned);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(c, e, "set_moments");
    c->steps = 0;
    return LBM_OK;
}

int lbm_set_equilibrium(lbm_ctx *c, const lbm_fields *prim)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int nf = c->species + 3;
    int rc = check_fields(c, prim, nf);
    if (rc) return rc;
    DeviceGuard g(c->device);
    const void *dev = nullptr;
    void *owned = nullptr;
    if ((rc = stage_in(c, prim, nf, &dev, &owned))) return rc;
    c->phi_of = nullptr;  // the state changes outside the step
    hipError_t e = lbm::launch_set_equilibrium(c, dev, prim->field_stride, prim->dtype, c->state[c->cur]);
    if (owned) {
        hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(owned);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(c, e, "set_equilibrium");
    c->steps = 0;
    return LBM_OK;
}

int lbm_get_moments(const lbm_ctx *c, lbm_fields *out)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int nf = public_fields(c);
    int rc = check_fields(c, out, nf);
    if (rc) return rc;
    DeviceGuard g(c->device);
    if (out->on_device) {
        hipError_t e = lbm::launch_get_moments(c, c->state[c->cur], out->base, out->field_stride, out->dtype);
        if (e != hipSuccess) return hip_fail(c, e, "get_moments");
        return LBM_OK;
    }
    const size_t bytes = (size_t)(out->dtype == LBM_DTYPE_F64 ? 8 : 4) * (size_t)out->field_stride * (size_t)nf;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(staging)");
    e = lbm::launch_get_moments(c, c->state[c->cur], d, out->field_stride, out->dtype);
    if (e == hipSuccess) e = hipMemcpyAsync(out->base, d, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(c, e, "get_moments(host)");
    return LBM_OK;
}

int lbm_reduce(lbm_ctx *c, double out[5])
{
    if (!c || !out) return LBM_EINVAL;
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = lbm::launch_reduce(c, c->state[c->cur]);
    double v[5];
    if (e == hipSuccess) e = hipMemcpyAsync(v, c->red_out, sizeof(v), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce");
    const double n = (double)c->N;
    // In place, after an odd number of steps the populations sit in the
    // reversed slots: the summed momentum changes sign.
    if (c->scheme == LBM_SCHEME_POPULATION_AA && (c->steps & 1))
        for (int a = 2; a < 5; ++a) v[a] = -v[a];
    if (c->species == 1) {
        out[0] = n + v[0];
        out[1] = 0.0;
    } else if (c->scheme == LBM_SCHEME_POPULATION) {
        out[0] = v[0];
        out[1] = v[1];
    } else {
        out[0] = v[0];
        out[1] = n + v[1] - v[0];
    }
    for (int a = 0; a < 3; ++a) out[2 + a] = v[2 + a];
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(out[k])) return fail(c, LBM_EUNSTABLE, "non-finite global total");
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int n)
{
    if (!c || n < 0) return fail(c, LBM_EINVAL, "lbm_step: bad argument");
    c->err.clear();
    DeviceGuard g(c->device);
    for (int t = 0; t < n;) {
        hipError_t e;
        int done = 1;
        // A two-step sweep unless a health check falls after its first step.
        const bool two = c->sweep == 2 && n - t >= 2 && !(c->check_every > 0 && (c->steps + 1) % c->check_every == 0);
        if (two) {
            e = lbm::launch_moment_sweep2(c, c->state[c->cur], c->state[1 - c->cur]);
            if (e == hipSuccess) c->cur = 1 - c->cur;
            done = 2;
        } else if (c->scheme == LBM_SCHEME_POPULATION_AA) {
            e = lbm::launch_population_aa_step(c, c->state[0], (c->steps & 1) != 0);
        } else {
            const void *in = c->state[c->cur];
            void *out = c->state[1 - c->cur];
            if (c->split && c->species == 2) {
                // Split approach: phase field, collision in place, streaming.
                e = lbm::launch_cg_split_step(c, c->state[c->cur], out);
            } else if (c->split) {
                // Split approach: relax the current state in place, then stream.
                e = lbm::launch_moment_collide(c, c->state[c->cur]);
                if (e == hipSuccess) e = lbm::launch_moment_step(c, in, out, true);
            } else {
                e = c->scheme == LBM_SCHEME_POPULATION ? lbm::launch_population_step(c, in, out)
                    : c->species == 2                  ? lbm::launch_cg_step(c, in, out, c->phi_of == in)
                                                       : lbm::launch_moment_step(c, in, out);
                // The near-contact scratch now holds the phase field of `out`.
                c->phi_of = e == hipSuccess && c->species == 2 && c->scheme == LBM_SCHEME_MOMENT && c->nc_A != 0.0
                                ? out
                                : nullptr;
            }
            if (e == hipSuccess) c->cur = 1 - c->cur;
        }
        if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
        c->steps += done;
        t += done;
        if (c->check_every > 0 && c->steps % c->check_every == 0) {
            double tot[5];
            int rc = lbm_reduce(c, tot);
            if (rc) return rc;
        }
    }
    return LBM_OK;
}

int lbm_memory_info(const lbm_ctx *c, int64_t *state_bytes, int64_t *step_bytes)
{
    if (!c) return LBM_EINVAL;
    const int64_t per_copy = (int64_t)c->elem * c->state_elems;
    const int64_t copies = c->scheme == LBM_SCHEME_POPULATION_AA ? 1 : 2;
    if (state_bytes)
        *state_bytes = copies * per_copy + (c->scratch_phi ? (int64_t)sizeof(float) * c->N : 0) +
                       (c->scratch_nc ? (int64_t)lbm::nc_scratch_bytes(c) : 0) +
                       (c->scratch_adj ? (int64_t)c->elem * c->lay3.plane * c->nz : 0) +
                       (c->scratch_split ? (int64_t)c->elem * 4 * c->N : 0);
    // Split approach, one species: the collision pass reads all stored fields
    // and writes S' (6 fields), the streaming pass reads and writes all of
    // them.  Two species: the phase pass reads dr and rho1 and writes phi (3),
    // the collision pass reads the 11 fields and phi and writes S' and n (21,
    // 24 with a force, which also rewrites j), the streaming pass reads the
    // 11 fields and n and writes 11 (25).
    const int64_t moved = !c->split ? 2 * (int64_t)c->nfields
                          : c->species == 1 ? 3 * (int64_t)c->nfields + 6
                                            : (c->nc_A != 0.0 ? 52 : 49);
    if (step_bytes) *step_bytes = moved * (int64_t)c->elem * c->N;
    return LBM_OK;
}

int lbm_state_bytes(const lbm_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = (int64_t)c->elem * c->state_elems;
    return LBM_OK;
}

int lbm_state_bytes_for(lbm_grid grid, int lattice, int species, const lbm_opts *opts, int64_t *bytes)
{
    if (!bytes) return LBM_EINVAL;
    lbm_opts o;
    lbm_default_opts(&o);
    if (opts) o = *opts;
    int sweep = 1;
    if (validate(grid, lattice, species, o, &sweep) != LBM_OK) return LBM_EINVAL;
    const StatePlan plan = state_plan(grid, lattice, species, o);
    *bytes = (int64_t)plan.elem * plan.elems;
    return LBM_OK;
}

int lbm_equilibrium_moments(lbm_ctx *c, const lbm_fields *primitive, lbm_fields *moments)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int np = c->species + 3, nm = public_fields(c);
    int rc = check_fields(c, primitive, np);
    if (!rc) rc = check_fields(c, moments, nm);
    if (rc) return rc;
    DeviceGuard g(c->device);
    const void *src = nullptr;
    void *in_owned = nullptr, *dst = nullptr, *out_owned = nullptr;
    if ((rc = stage_in(c, primitive, np, &src, &in_owned))) return rc;
    if ((rc = stage_out(c, moments, nm, &dst, &out_owned))) {
        if (in_owned) (void)hipFree(in_owned);
        return rc;
    }
    hipError_t e = lbm::launch_equilibrium(c, src, primitive->field_stride, primitive->dtype, dst,
                                           moments->field_stride, moments->dtype);
    e = finish_io(c, e, moments, nm, out_owned, in_owned);
    if (e != hipSuccess) return hip_fail(c, e, "equilibrium_moments");
    return LBM_OK;
}

int lbm_equilibrium_moments_adjoint(lbm_ctx *c, const lbm_fields *primitive, const lbm_fields *grad_moments,
                                    lbm_fields *grad_primitive)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int np = c->species + 3, nm = public_fields(c);
    int rc = check_fields(c, primitive, np);
    if (!rc) rc = check_fields(c, grad_moments, nm);
    if (!rc) rc = check_fields(c, grad_primitive, np);
    if (rc) return rc;
    DeviceGuard g(c->device);
    const void *prim = nullptr, *grad = nullptr;
    void *p_owned = nullptr, *g_owned = nullptr, *dst = nullptr, *out_owned = nullptr;
    if ((rc = stage_in(c, primitive, np, &prim, &p_owned))) return rc;
    if ((rc = stage_in(c, grad_moments, nm, &grad, &g_owned)) ||
        (rc = stage_out(c, grad_primitive, np, &dst, &out_owned))) {
        if (p_owned) (void)hipFree(p_owned);
        if (g_owned) (void)hipFree(g_owned);
        return rc;
    }
    hipError_t e = lbm::launch_equilibrium_adjoint(c, prim, primitive->field_stride, primitive->dtype, grad,
                                                   grad_moments->field_stride, grad_moments->dtype, dst,
                                                   grad_primitive->field_stride, grad_primitive->dtype);
    e = finish_io(c, e, grad_primitive, np, out_owned, p_owned, g_owned);
    if (e != hipSuccess) return hip_fail(c, e, "equilibrium_moments_adjoint");
    return LBM_OK;
}

int lbm_save_state(lbm_ctx *c, void *dst)
{
    if (!c) return LBM_EINVAL;
    if (!dst) return fail(c, LBM_EINVAL, "save_state: NULL buffer");
    if (c->scheme == LBM_SCHEME_POPULATION_AA) return fail(c, LBM_ESTATE, "save_state: not for the in-place scheme");
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = lbm::launch_copy(c, c->state[c->cur], dst, (int64_t)c->elem * c->state_elems);
    if (e != hipSuccess) return hip_fail(c, e, "save_state");
    return LBM_OK;
}

int lbm_load_state(lbm_ctx *c, const void *src)
{
    if (!c) return LBM_EINVAL;
    if (!src) return fail(c, LBM_EINVAL, "load_state: NULL buffer");
    if (c->scheme == LBM_SCHEME_POPULATION_AA) return fail(c, LBM_ESTATE, "load_state: not for the in-place scheme");
    c->err.clear();
    DeviceGuard g(c->device);
    c->phi_of = nullptr;  // the state changes outside the step
    hipError_t e = lbm::launch_copy(c, src, c->state[c->cur], (int64_t)c->elem * c->state_elems);
    if (e != hipSuccess) return hip_fail(c, e, "load_state");
    return LBM_OK;
}

int lbm_step_state(lbm_ctx *c, const void *src, void *dst)
{
    if (!c) return LBM_EINVAL;
    if (!src || !dst || src == dst) return fail(c, LBM_EINVAL, "step_state: NULL or identical buffers");
    if (c->scheme != LBM_SCHEME_MOMENT) return fail(c, LBM_ESTATE, "step_state: moment scheme only");
    if (c->split) return fail(c, LBM_ESTATE, "step_state: fused step only (split context)");
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = c->species == 2 ? lbm::launch_cg_step(c, src, dst) : lbm::launch_moment_step(c, src, dst);
    c->phi_of = nullptr;  // the scratch describes dst, not the context's state
    if (e != hipSuccess) return hip_fail(c, e, "step_state");
    return LBM_OK;
}

int lbm_step_state2(lbm_ctx *c, const void *src, void *mid, void *dst)
{
    if (!c) return LBM_EINVAL;
    if (!src || !mid || !dst || src == mid || src == dst || mid == dst)
        return fail(c, LBM_EINVAL, "step_state2: NULL or aliased buffers");
    if (!lbm::moment_sweep2_supported(c))
        return fail(c, LBM_ESTATE, "step_state2: one species, fused moment step, FP32/FP16/BF16 storage only");
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = lbm::launch_moment_sweep2(c, src, dst, mid);
    if (e != hipSuccess) return hip_fail(c, e, "step_state2");
    return LBM_OK;
}

int lbm_adjoint_step2_stored(lbm_ctx *c, const void *state_t1, const void *state_t0, const void *lam_next,
                             void *lam_out, double *dtau_accum)
{
    if (!c) return LBM_EINVAL;
    if (!state_t1 || !state_t0 || !lam_next || !lam_out || lam_next == lam_out)
        return fail(c, LBM_EINVAL, "adjoint_step2: NULL or aliased buffers");
    if (!lbm::moment_sweep2_supported(c))
        return fail(c, LBM_ESTATE, "adjoint_step2: one species, fused moment step, FP32/FP16/BF16 storage only");
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = lbm::launch_adjoint_sweep2(c, state_t1, state_t0, lam_next, lam_out, dtau_accum);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step2");
    return LBM_OK;
}

static size_t real_bytes(const lbm_ctx *c) { return c->storage == LBM_STORE_F64 ? 8 : 4; }

// Validation shared by the adjoint entry points, and (if allocate) the
// colour-gradient co-state buffer the two-species adjoint needs, allocated on
// first use.
static int adjoint_ready(lbm_ctx *c, bool allocate = true)
{
    if (c->scheme != LBM_SCHEME_MOMENT) return fail(c, LBM_ESTATE, "adjoint_step: moment scheme only");
    if (c->species == 2 && c->storage != LBM_STORE_F32 && c->storage != LBM_STORE_F64)
        return fail(c, LBM_ESTATE, "adjoint_step: two species need FP32 or FP64 storage");
    if (c->nc_A != 0.0) return fail(c, LBM_ESTATE, "adjoint_step: not with the near-contact force");
    if (allocate && c->species == 2 && !c->scratch_adj) {
        if (hipMalloc(&c->scratch_adj, c->elem * (size_t)(c->lay3.plane * c->nz)) != hipSuccess) {
            c->scratch_adj = nullptr;
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "adjoint_step: colour-gradient co-state buffer");
        }
    }
    return LBM_OK;
}

int lbm_adjoint_step(lbm_ctx *c, const lbm_fields *state_t, const lbm_fields *lam_next, lbm_fields *lam_out,
                     double *dtau_accum)
{
    if (!c) return LBM_EINVAL;
    c->err.clear();
    const int nf = public_fields(c);
    int rc = check_fields(c, state_t, nf);
    if (!rc) rc = check_fields(c, lam_next, nf);
    if (!rc) rc = check_fields(c, lam_out, nf);
    if (rc) return rc;
    if (lam_next->base == lam_out->base) return fail(c, LBM_EINVAL, "adjoint_step: lam_out aliases lam_next");
    DeviceGuard g(c->device);
    if ((rc = adjoint_ready(c))) return rc;
    // Work area kept by the context: the state in its stored format and the
    // two co-states in the stored layout, then one double for dL/dtau.
    const size_t st_bytes = (c->elem * (size_t)c->state_elems + 255) / 256 * 256;
    const size_t co_bytes = (real_bytes(c) * (size_t)c->state_elems + 255) / 256 * 256;
    if (!c->adj_work) {
        if (hipMalloc(&c->adj_work, st_bytes + 2 * co_bytes) != hipSuccess ||
            hipMalloc((void **)&c->adj_dtau, sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            if (c->adj_work) (void)hipFree(c->adj_work);
            c->adj_work = nullptr;
            c->adj_dtau = nullptr;
            return fail(c, LBM_ENOMEM, "adjoint_step: work area");
        }
    }
    char *w = static_cast<char *>(c->adj_work);
    void *st = w, *co_in = w + st_bytes, *co_out = w + st_bytes + co_bytes;
    const void *s_dev = nullptr, *l_dev = nullptr;
    void *s_owned = nullptr, *l_owned = nullptr, *o_dev = nullptr, *o_owned = nullptr;
    if ((rc = stage_in(c, state_t, nf, &s_dev, &s_owned))) return rc;
    if ((rc = stage_in(c, lam_next, nf, &l_dev, &l_owned)) || (rc = stage_out(c, lam_out, nf, &o_dev, &o_owned))) {
        if (s_owned) (void)hipFree(s_owned);
        if (l_owned) (void)hipFree(l_owned);
        return rc;
    }
    hipError_t e = lbm::launch_set_moments(c, s_dev, state_t->field_stride, state_t->dtype, st);
    if (e == hipSuccess) e = lbm::launch_costate_convert(c, l_dev, co_in, true, lam_next->field_stride, lam_next->dtype);
    if (e == hipSuccess && dtau_accum) e = hipMemsetAsync(c->adj_dtau, 0, sizeof(double), c->stream);
    if (e == hipSuccess)
        e = c->species == 2 ? lbm::launch_cg_adjoint_step(c, st, co_in, co_out, dtau_accum ? c->adj_dtau : nullptr, true)
                            : lbm::launch_adjoint_step(c, st, co_in, co_out, dtau_accum ? c->adj_dtau : nullptr, true);
    if (e == hipSuccess)
        e = lbm::launch_costate_convert(c, co_out, o_dev, false, lam_out->field_stride, lam_out->dtype);
    double d = 0.0;
    if (e == hipSuccess && dtau_accum) e = hipMemcpyAsync(&d, c->adj_dtau, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && dtau_accum && !o_owned && !s_owned && !l_owned) e = hipStreamSynchronize(c->stream);
    e = finish_io(c, e, lam_out, nf, o_owned, s_owned, l_owned);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    if (dtau_accum) *dtau_accum += d;
    return LBM_OK;
}

int lbm_adjoint_step_stored(lbm_ctx *c, const void *state, const void *lam_next, void *lam_out, double *dtau_accum)
{
    if (!c) return LBM_EINVAL;
    if (!state || !lam_next || !lam_out || lam_next == lam_out)
        return fail(c, LBM_EINVAL, "adjoint_step: NULL or aliased buffers");
    c->err.clear();
    DeviceGuard g(c->device);
    int rc = adjoint_ready(c);
    if (rc) return rc;
    hipError_t e = c->species == 2 ? lbm::launch_cg_adjoint_step(c, state, lam_next, lam_out, dtau_accum, true)
                                   : lbm::launch_adjoint_step(c, state, lam_next, lam_out, dtau_accum, true);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    return LBM_OK;
}
int lbm_adjoint_step_stored_noalloc(lbm_ctx *c, const void *state, const void *lam_next, void *lam_out,
                                    double *dtau_accum)
{
    if (!c) return LBM_EINVAL;
    if (!state || !lam_next || !lam_out || lam_next == lam_out)
        return fail(c, LBM_EINVAL, "adjoint_step_stored_noalloc: NULL or aliased buffers");
    c->err.clear();
    int rc = adjoint_ready(c, false);
    if (rc) return rc;
    DeviceGuard g(c->device);
    hipError_t e;
    if (c->species == 2) {
        const size_t need = c->elem * (size_t)(c->lay3.plane * c->nz);
        if (need > kScratchBytes)
            return fail(c, LBM_EINVAL,
                        "adjoint_step_stored_noalloc: the colour-gradient co-state needs " + std::to_string(need) +
                            " bytes, beyond the static scratch of " + std::to_string(kScratchBytes) + " bytes");
        void *sp = nullptr;
        if ((e = scratch_ptr(c->device, &sp)) != hipSuccess) return hip_fail(c, e, "adjoint_step_stored_noalloc");
        e = lbm::launch_cg_adjoint_step(c, state, lam_next, lam_out, dtau_accum, true, sp);
    } else {
        e = lbm::launch_adjoint_step(c, state, lam_next, lam_out, dtau_accum, true);
    }
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step_stored_noalloc");
    return LBM_OK;
}

int lbm_costate_bytes(const lbm_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return LBM_EINVAL;
    if (c->scheme != LBM_SCHEME_MOMENT) return fail(c, LBM_ESTATE, "costate_bytes: moment scheme only");
    *bytes = (int64_t)real_bytes(c) * c->state_elems;
    return LBM_OK;
}

static int costate_convert(lbm_ctx *c, const void *src, void *dst, bool to_stored)
{
    if (!c) return LBM_EINVAL;
    if (!src || !dst || src == dst) return fail(c, LBM_EINVAL, "costate conversion: NULL or aliased buffers");
    if (c->scheme != LBM_SCHEME_MOMENT) return fail(c, LBM_ESTATE, "costate conversion: moment scheme only");
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = lbm::launch_costate_convert(c, src, dst, to_stored);
    if (e != hipSuccess) return hip_fail(c, e, "costate conversion");
    return LBM_OK;
}

int lbm_costate_to_stored(lbm_ctx *c, const void *public_dev, void *stored_dev)
{
    return costate_convert(c, public_dev, stored_dev, true);
}

int lbm_costate_from_stored(lbm_ctx *c, const void *stored_dev, void *public_dev)
{
    return costate_convert(c, stored_dev, public_dev, false);
}

int64_t lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : -1; }

int lbm_steps_per_sweep(const lbm_ctx *c) { return c ? c->sweep : -1; }

} // extern "C"
