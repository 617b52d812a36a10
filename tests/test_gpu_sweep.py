"""Two time steps per pass over the state (one species, fused step): the
sweep kernel carries each tile through two steps with the same per-node
arithmetic as the single step, so its results must equal single steps bit
for bit (16-bit storage included: the intermediate state is rounded to the
storage format as a stored state would be), and match the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _run(H, q, tau, steps, storage, sweep, check_every=0, chunks=(None,)):
    from paper_2301_01622_amd.lbm import LBM
    nf, nz, ny, nx = H.shape
    sim = LBM((nx, ny, nz), q, tau, storage=storage, steps_per_sweep=sweep, check_every=check_every)
    sim.set_moments(torch.from_numpy(H).cuda())
    for c in chunks:
        sim.step(steps if c is None else c)
    out = sim.get_moments(torch.float64).cpu().numpy()
    assert sim.steps_done == steps
    sim.close()
    return out


# (nx, ny, nz): several 32 x 16 tiles with ragged tails and two z-chunks;
# one tile wider than the box (x-halo wraps onto the tile); minimum box;
# a 256-wide box.
SHAPES = [(70, 37, 20), (17, 13, 11), (3, 3, 3), (256, 5, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_sweep_equals_single_steps(shape, q, storage):
    steps = 7  # three sweeps and one single step
    _say(f"two-step sweep {shape} D3Q{q} {storage} {steps} steps")
    H = I.random_moments(shape[::-1], seed=90 + q)
    a = _run(H, q, 0.62, steps, storage, 2)
    b = _run(H, q, 0.62, steps, storage, 1)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("q", [19, 27])
def test_sweep_matches_oracle(oracle, q):
    shape = (70, 37, 20)
    _say(f"two-step sweep {shape} D3Q{q} f32 8 steps vs oracle")
    H = I.random_moments(shape[::-1], seed=95 + q)
    got = _run(H, q, 0.7, 8, "f32", 2)
    ref = oracle.moment_run(H, q, 0.7, 8)
    assert np.abs(got - ref).max() <= 1e-6


def test_sweep_with_health_checks_and_split_calls():
    """check_every = 3 forces single steps where a check falls between the two
    steps of a sweep; calls of odd length leave single steps too; the result
    is the same."""
    H = I.random_moments((20, 37, 70), seed=97)
    ref = _run(H, 27, 0.6, 12, "f32", 1)
    np.testing.assert_array_equal(_run(H, 27, 0.6, 12, "f32", 2, check_every=3), ref)
    np.testing.assert_array_equal(_run(H, 27, 0.6, 12, "f32", 2, chunks=(1, 3, 5, 2, 1)), ref)


def test_sweep_full_size_sampled(oracle):
    """256^3 D3Q27 FP32 (the throughput workload), 2 steps as one sweep,
    against the oracle on sampled nodes (each from its 5^3 dependency cone)."""
    n, q, tau, steps = 256, 27, 0.6, 2
    rho, u = I.random_solenoidal_box(n, I.SEED_C2, umax=1e-3)
    H0 = oracle.equilibrium_moments(rho, u)
    from paper_2301_01622_amd.lbm import LBM
    sim = LBM((n, n, n), q, tau, storage="f32", steps_per_sweep=2)
    sim.set_moments(torch.from_numpy(H0).cuda())
    sim.step(steps)
    got = sim.get_moments(torch.float64).cpu().numpy()
    sim.close()
    rng = np.random.default_rng(5)
    nodes = [(0, 0, 0), (255, 255, 255), (128, 31, 32)] + [tuple(rng.integers(0, n, 3)) for _ in range(5)]
    r = steps
    for (z, y, x) in nodes:
        idx = [np.arange(c - r, c + r + 1) % n for c in (z, y, x)]
        cube = H0[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
        # The cone is not periodic: only its centre is exact after `steps` steps.
        ref = oracle.moment_run(np.ascontiguousarray(cube), q, tau, steps)[:, r, r, r]
        assert np.abs(got[:, z, y, x] - ref).max() <= 1e-6, (z, y, x)


# ---- two-step recompute and two-step adjoint (reverse mode) --------------------------

@pytest.mark.parametrize("shape", [(70, 37, 20), (17, 13, 11), (3, 3, 3)])
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_step_state2_and_adjoint2_equal_single_steps(shape, q, storage):
    from paper_2301_01622_amd.lbm import LBM
    _say(f"two-step recompute and adjoint {shape} D3Q{q} {storage}")
    H = I.random_moments(shape[::-1], seed=110 + q, drho=0.01, dj=0.01, dp=0.003)
    sim = LBM(shape, q, 0.66, storage=storage)
    sim.set_moments(torch.from_numpy(H).cuda())
    # Zeroed buffers: slots of the stored layout that hold no node stay zero.
    s0, s1, s2, m, d = (sim.new_checkpoint().zero_() for _ in range(5))
    sim.save_state(s0)
    sim.step_state(s0, s1)
    sim.step_state(s1, s2)
    sim.step_state2(s0, m, d)
    assert torch.equal(m, s1) and torch.equal(d, s2)

    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    pub = torch.randn((10,) + sim.shape, generator=g, device="cuda", dtype=torch.float32)
    lam, a, b = sim.new_costate(), sim.new_costate(), sim.new_costate()
    sim.costate_to_stored(pub, lam)
    t1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    sim.adjoint_step_stored(s1, lam, a, t1)
    sim.adjoint_step_stored(s0, a, b, t1)
    out = sim.new_costate()
    sim.adjoint_step2_stored(s1, s0, lam, out, t2)
    pa, pb = torch.empty_like(pub), torch.empty_like(pub)
    sim.costate_from_stored(b, pa)
    sim.costate_from_stored(out, pb)
    assert torch.equal(pa, pb)
    assert abs(float(t2) - float(t1)) <= 1e-12 * abs(float(t1))
    sim.close()


def test_two_step_entry_points_reject_bad_calls():
    import ctypes
    from paper_2301_01622_amd import _lib
    from paper_2301_01622_amd.lbm import LBM
    sim = LBM((8, 8, 8), 19, 0.8, storage="f64")
    a, b, c = (sim.new_checkpoint() for _ in range(3))
    lib, ctx, p = sim._lib, sim._ctx, (lambda t: ctypes.c_void_p(t.data_ptr()))
    assert lib.lbm_step_state2(ctx, p(a), p(b), p(c)) == _lib.LBM_ESTATE
    lam, lo = sim.new_costate(), sim.new_costate()
    assert lib.lbm_adjoint_step2_stored(ctx, p(a), p(b), p(lam), p(lo), None) == _lib.LBM_ESTATE
    sim.close()
    sim = LBM((8, 8, 8), 19, 0.8, storage="f32")
    a, b, c = (sim.new_checkpoint() for _ in range(3))
    lib, ctx = sim._lib, sim._ctx
    assert lib.lbm_step_state2(ctx, p(a), p(a), p(c)) == _lib.LBM_EINVAL
    assert lib.lbm_step_state2(ctx, p(a), None, p(c)) == _lib.LBM_EINVAL
    lam = sim.new_costate()
    assert lib.lbm_adjoint_step2_stored(ctx, p(a), p(b), p(lam), p(lam), None) == _lib.LBM_EINVAL
    sim.close()


def test_steps_per_sweep_is_reported():
    from paper_2301_01622_amd.lbm import LBM
    cases = [(dict(storage="f32"), True), (dict(storage="bf16"), True), (dict(storage="f64"), False),
             (dict(storage="f32", steps_per_sweep=1), False), (dict(storage="f32", split=True), False)]
    for kw, expect in cases:
        sim = LBM((8, 8, 8), 19, 0.8, **kw)
        assert sim.sweeps == expect, kw
        sim.close()
    sim = LBM((8, 8, 8), 19, 0.8, species=2)
    assert not sim.sweeps
    sim.close()
