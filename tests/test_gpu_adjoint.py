"""GPU parity of the discrete adjoint (one species) against the oracle's
adjoint, K-independence of the checkpointed rollout, and a central
finite-difference check of the rollout gradient."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def mods():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_01622_amd import autograd as AG
    from paper_2301_01622_amd.lbm import LBM
    return LBM, AG


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("where", ["device", "host"])
def test_adjoint_step_matches_oracle(mods, oracle, q, storage, tol, where):
    """lbm_adjoint_step at the boundary: state M(t) and co-states as public
    moments, in device memory (the kernels' real type) or in host memory
    (FP64 numpy arrays), dL/dtau accumulated into a host double."""
    LBM, _ = mods
    shape = (19, 23, 37)
    _say(f"adjoint step {shape} D3Q{q} {storage} buffers on the {where}")
    M = I.random_moments(shape, seed=91)
    lam = np.random.default_rng(92).standard_normal(M.shape)
    tau = 0.66
    ref, dom = oracle.moment_adjoint_step(M, lam, q, tau)
    sim = LBM((37, 23, 19), q, tau, storage=storage)
    if where == "device":
        st = torch.from_numpy(M).cuda()
        ln = torch.from_numpy(lam).to(sim.real_dtype).cuda().contiguous()
        lo = torch.empty_like(ln)
    else:
        st, ln, lo = M, lam, np.empty_like(lam)
    dtau = sim.adjoint_step(st, ln, lo, dtau=1.0) - 1.0
    got = lo.double().cpu().numpy() if where == "device" else lo
    sim.close()
    e = _rel(got, ref)
    _say(f"  rel err {e:.3e}, dL/dtau gpu {dtau:.10e} oracle {-dom / tau ** 2:.10e}")
    assert e <= tol
    assert abs(dtau - (-dom / tau ** 2)) <= 10 * tol * abs(dom / tau ** 2)


def _loss_weights(shape, seed):
    return np.random.default_rng(seed).standard_normal((10,) + shape)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-4)])
def test_rollout_gradient_matches_oracle(mods, oracle, storage, tol):
    """L = sum(W * M(T)); dL/dM0 and dL/dtau through 13 steps, K = 5."""
    LBM, AG = mods
    q, shape, T, tau = 19, (12, 13, 17), 13, 0.7
    _say(f"rollout gradient {shape} {storage} T={T} K=5")
    M0 = I.random_moments(shape, seed=93, drho=0.01, dj=0.01, dp=0.003)
    W = _loss_weights(shape, 94)
    lam0, dL_dtau = oracle.moment_rollout_gradient(M0, W, q, tau, T)
    sim = LBM((17, 13, 12), q, tau, storage=storage)
    m0 = torch.from_numpy(M0).cuda().requires_grad_(True)
    t = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    MT = AG.rollout(sim, m0, t, T, K=5)
    (MT * torch.from_numpy(W).cuda()).sum().backward()
    g = m0.grad.cpu().numpy()
    gt = float(t.grad.cpu())
    sim.close()
    e = _rel(g, lam0)
    _say(f"  rel err dM0 {e:.3e}; dL/dtau gpu {gt:.8e} oracle {dL_dtau:.8e}")
    assert e <= tol
    assert abs(gt - dL_dtau) <= tol * abs(dL_dtau)


def test_rollout_independent_of_checkpoint_interval(mods):
    LBM, AG = mods
    shape, T, tau = (16, 16, 16), 24, 0.75
    M0 = I.random_moments(shape, seed=95, drho=0.01, dj=0.01, dp=0.003)
    W = torch.from_numpy(_loss_weights(shape, 96)).cuda()
    grads = []
    for K in (1, 5, 24):
        sim = LBM((16, 16, 16), 27, tau, storage="f32")
        m0 = torch.from_numpy(M0).cuda().requires_grad_(True)
        t = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
        (AG.rollout(sim, m0, t, T, K=K) * W).sum().backward()
        grads.append((m0.grad.cpu().numpy(), float(t.grad)))
        sim.close()
    for g, gt in grads[1:]:
        np.testing.assert_array_equal(g, grads[0][0])
        # Two-step adjoint passes group the per-step FP64 sums differently.
        assert abs(gt - grads[0][1]) <= 1e-12 * abs(grads[0][1])


def test_rollout_gradient_finite_differences(mods):
    """32^3 D3Q19 FP32, 60 steps, checkpoints every 20: gradient of the
    kinetic energy of a target region with respect to the initial velocity
    (along a seeded solenoidal direction) and to tau, against central
    differences with h = 1e-3 computed with the GPU forward step."""
    LBM, AG = mods
    n, T, K, tau = 32, 60, 20, 0.8
    _say("finite-difference check 32^3 D3Q19 f32 T=60 K=20")
    rho, u0 = I.random_solenoidal_box(n, seed=I.SEED_C5, umax=0.02)
    d = I.solenoidal((n, n, n), seed=I.SEED_C5 + 1, umax=1.0)
    mask = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    mask[8:24, 8:24, 8:24] = 1.0
    rho_t = torch.from_numpy(rho).cuda()

    def loss_of(u, t, grad=False):
        sim = LBM((n, n, n), 19, float(t), storage="f32")
        u = torch.from_numpy(u).cuda().requires_grad_(grad)
        tt = torch.tensor(float(t), dtype=torch.float64, device="cuda", requires_grad=grad)
        MT = AG.MomentLBRollout.apply(rho_t, u, tt, sim, T, K)
        L = (mask * (MT[1] ** 2 + MT[2] ** 2 + MT[3] ** 2) / MT[0]).sum()
        if grad:
            L.backward()
            out = (float(L), u.grad.cpu().numpy(), float(tt.grad))
        else:
            out = float(L)
        sim.close()
        return out

    L0, gu, gt = loss_of(u0, tau, grad=True)
    h = 1e-3
    fd_u = (loss_of(u0 + h * d, tau) - loss_of(u0 - h * d, tau)) / (2 * h)
    fd_t = (loss_of(u0, tau + h) - loss_of(u0, tau - h)) / (2 * h)
    ad_u = float(np.sum(gu * d))
    _say(f"  dL/du.d adjoint {ad_u:.6e} fd {fd_u:.6e};  dL/dtau adjoint {gt:.6e} fd {fd_t:.6e}")
    assert abs(ad_u - fd_u) <= 1e-2 * abs(fd_u)
    assert abs(gt - fd_t) <= 1e-2 * abs(fd_t)


@pytest.mark.parametrize("species", [1, 2])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_adjoint_step_stored_layout_bitwise(mods, oracle, species, storage):
    """Co-states in the stored (blocked) layout: conversion round trip and one
    reverse step equal, bit for bit, the public-layout step, on a ragged box
    whose x and y are not multiples of the 64 x 16 blocks."""
    LBM, _ = mods
    shape = (19, 23, 37)
    if species == 1:
        M = I.random_moments(shape, seed=95)
    else:
        nz, ny, nx = shape
        r1, r2, u = I.droplets(shape, centres=[(11.0, 10.0, 9.0), (26.0, 13.0, 9.0)], radius=5.0,
                               velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
        M = oracle.equilibrium_moments2(r1, r2, u)
    lam = np.random.default_rng(96).standard_normal(M.shape)
    sim = LBM((37, 23, 19), 19, 0.7, species=species, storage=storage, sigma=0.01, beta=0.7)
    Md = torch.from_numpy(M).cuda()
    sim.set_moments(Md)
    st = sim.new_checkpoint()
    sim.save_state(st)
    ln = torch.from_numpy(lam).to(sim.real_dtype).cuda().contiguous()
    lo = torch.empty_like(ln)
    d_pub = sim.adjoint_step(Md, ln, lo, dtau=0.0)
    s_in, s_out = sim.new_costate(), sim.new_costate()
    sim.costate_to_stored(ln, s_in)
    back = torch.empty_like(ln)
    sim.costate_from_stored(s_in, back)
    d_st = torch.zeros(1, dtype=torch.float64, device="cuda")
    sim.adjoint_step_stored(st, s_in, s_out, d_st)
    lo2 = torch.empty_like(ln)
    sim.costate_from_stored(s_out, lo2)
    torch.cuda.synchronize()
    sim.close()
    assert torch.equal(back, ln)
    assert torch.equal(lo2, lo)
    assert float(d_st) == d_pub


def test_adjoint_entry_points_reject_bad_calls(mods):
    """Error behaviour of the adjoint and co-state entry points: aliased or
    NULL buffers are LBM_EINVAL, the population scheme is LBM_ESTATE; nothing
    is launched in either case."""
    LBM, _ = mods
    from paper_2301_01622_amd import _lib
    lib = _lib.load()
    sim = LBM((20, 18, 16), 19, 0.7, storage="f32")
    st = sim.new_checkpoint()
    sim.save_state(st)
    lam = sim.new_costate()
    p = ctypes.c_void_p
    ctx = sim._ctx
    assert lib.lbm_adjoint_step_stored(ctx, p(st.data_ptr()), p(lam.data_ptr()), p(lam.data_ptr()), None) == \
        _lib.LBM_EINVAL
    pub = torch.zeros((10, 16, 18, 20), device="cuda")
    f = _lib.Fields(pub.data_ptr(), sim.n_nodes, _lib.DTYPE_F32, 1)
    g = _lib.Fields(lam.data_ptr(), sim.n_nodes, _lib.DTYPE_F32, 1)
    assert lib.lbm_adjoint_step(ctx, None, ctypes.byref(f), ctypes.byref(g), None) == _lib.LBM_EINVAL
    assert lib.lbm_adjoint_step(ctx, ctypes.byref(f), ctypes.byref(g), ctypes.byref(g), None) == _lib.LBM_EINVAL
    short = _lib.Fields(pub.data_ptr(), sim.n_nodes - 1, _lib.DTYPE_F32, 1)
    assert lib.lbm_adjoint_step(ctx, ctypes.byref(short), ctypes.byref(f), ctypes.byref(g), None) == \
        _lib.LBM_EINVAL
    assert lib.lbm_costate_to_stored(ctx, p(lam.data_ptr()), p(lam.data_ptr())) == _lib.LBM_EINVAL
    assert lib.lbm_costate_from_stored(ctx, None, p(lam.data_ptr())) == _lib.LBM_EINVAL
    assert lib.lbm_costate_bytes(ctx, None) == _lib.LBM_EINVAL
    sim.close()
    pop = LBM((20, 18, 16), 19, 0.7, storage="f32", scheme="population")
    b = ctypes.c_int64()
    assert lib.lbm_costate_bytes(pop._ctx, ctypes.byref(b)) == _lib.LBM_ESTATE
    buf = torch.zeros(16, device="cuda")
    buf2 = torch.zeros(16, device="cuda")
    pa = torch.zeros((10, 16, 18, 20), device="cuda")
    pb = torch.zeros((10, 16, 18, 20), device="cuda")
    pc = torch.zeros((10, 16, 18, 20), device="cuda")
    fa, fb, fc = (_lib.Fields(t.data_ptr(), pop.n_nodes, _lib.DTYPE_F32, 1) for t in (pa, pb, pc))
    assert lib.lbm_adjoint_step(pop._ctx, ctypes.byref(fa), ctypes.byref(fb), ctypes.byref(fc), None) == \
        _lib.LBM_ESTATE
    assert lib.lbm_costate_to_stored(pop._ctx, p(buf.data_ptr()), p(buf2.data_ptr())) == _lib.LBM_ESTATE
    assert "moment scheme" in lib.lbm_last_error(pop._ctx).decode()
    torch.cuda.synchronize()
    pop.close()
