"""The paper's split approach (Sec. III.A): a collision pass stores the
post-collision moments, a streaming pass reconstructs, pulls and sums.  The
split is a different schedule of the same arithmetic, so with FP32/FP64
storage (S' stored exactly in the precision it is computed in) it must equal
the fused step bit for bit; with 16-bit storage S' is rounded once more per
step, and the error against the FP64 oracle is bounded like the fused
step's with that extra rounding."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402

MANTISSA = {"f16": 10, "bf16": 7}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _run(H, q, tau, steps, storage, split):
    from paper_2301_01622_amd.lbm import LBM
    nf, nz, ny, nx = H.shape
    sim = LBM((nx, ny, nz), q, tau, storage=storage, split=split)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(steps)
    out = sim.get_moments(torch.float64).cpu().numpy()
    mem = sim.memory_info()
    sim.close()
    return out, mem


@pytest.mark.parametrize("shape", [(11, 13, 17), (5, 6, 256)])
@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_split_equals_fused_and_oracle(oracle, shape, q, storage, tol):
    _say(f"split approach {shape} D3Q{q} {storage} 9 steps")
    H = I.random_moments(shape, seed=70 + q)
    split, mem_s = _run(H, q, 0.7, 9, storage, True)
    fused, mem_f = _run(H, q, 0.7, 9, storage, False)
    np.testing.assert_array_equal(split, fused)
    assert np.abs(split - oracle.moment_run(H, q, 0.7, 9)).max() <= tol
    N = int(np.prod(shape))
    elem = 8 if storage == "f64" else 4
    assert mem_f[1] == 20 * elem * N and mem_s[1] == 36 * elem * N
    assert mem_s[0] == mem_f[0]


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_split_reduced_precision(oracle, storage):
    n, T, tau = 24, 100, 0.55
    _say(f"split approach {n}^3 D3Q27 {storage} {T} steps")
    rho, u = I.shear_wave_with_noise(n, seed=I.SEED_C4, u0=0.01, noise=1e-4)
    H = oracle.equilibrium_moments(rho, u)
    ref = oracle.moment_run(H, 27, tau, T)
    ur = ref[1:4] / ref[0]
    eps = 2.0 ** -(MANTISSA[storage] + 1)
    bound = 16 * np.sqrt(2.0) * eps * np.abs(ur).max() * np.sqrt(T)
    for split in (False, True):
        got, _ = _run(H, 27, tau, T, storage, split)
        err = np.abs(got[1:4] / got[0] - ur).max()
        _say(f"  split={split} max|du| = {err:.3e} (bound {bound:.3e})")
        assert np.isfinite(got).all() and err <= bound


def test_split_context_rejects_step_state():
    from paper_2301_01622_amd import _lib
    from paper_2301_01622_amd.lbm import LBM
    sim = LBM((8, 8, 8), 19, 0.8, split=True)
    a = sim.new_checkpoint()
    b = sim.new_checkpoint()
    with pytest.raises(_lib.LbmError) as e:
        sim.step_state(a, b)
    assert e.value.code == _lib.LBM_ESTATE
    sim.close()


def _droplet_state(oracle, shape, gap=3.0, R=5.0):
    nz, ny, nx = shape
    c1 = (nx / 2 - gap / 2 - R, ny / 2 + 0.3, nz / 2 - 0.2)
    c2 = (nx / 2 + gap / 2 + R, ny / 2 - 0.4, nz / 2 + 0.1)
    r1, r2, u = I.droplets(shape, centres=[c1, c2], radius=R, velocities=[(0.02, 0, 0), (-0.02, 0, 0)], width=1.0)
    H = oracle.equilibrium_moments2(r1, r2, u)
    # a generic non-equilibrium part, so that the relaxation matters
    H[5:] += 1e-3 * np.random.default_rng(77).standard_normal(H[5:].shape)
    return np.ascontiguousarray(H)


def _run2(H, q, steps, storage, split, nc_A=0.0):
    from paper_2301_01622_amd.lbm import LBM
    nf, nz, ny, nx = H.shape
    sim = LBM((nx, ny, nz), q, 0.8, species=2, storage=storage, sigma=0.01, beta=0.7, split=split, nc_A=nc_A,
              nc_hmax=4 if nc_A else 0)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(steps)
    out = sim.get_moments(torch.float64).cpu().numpy()
    mem = sim.memory_info()
    sim.close()
    return out, mem


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("nc_A", [0.0, 0.05])
def test_split_two_species_equals_fused_and_oracle(oracle, q, storage, tol, nc_A):
    """The colour-gradient step as a phase pass, a collision pass and a
    streaming pass, on a ragged 70 x 21 x 13 box (several tiles, partial
    ones) with two drops three nodes apart, 6 steps, with and without the
    near-contact force: equal to the fused step bit for bit, and to the
    oracle within the fused step's bound."""
    shape = (13, 21, 70)
    _say(f"two-species split {shape} D3Q{q} {storage} nc_A={nc_A} 6 steps")
    H = _droplet_state(oracle, shape)
    split, mem_s = _run2(H, q, 6, storage, True, nc_A)
    fused, mem_f = _run2(H, q, 6, storage, False, nc_A)
    np.testing.assert_array_equal(split, fused)
    A = oracle.sigma_to_A(0.01, 0.8)
    ref = oracle.cg_moment_run(H, q, 0.8, A, 0.7, 6, Ah=nc_A, hmax=4 if nc_A else 0)
    err = np.abs(split - ref).max()
    _say(f"  max err vs oracle {err:.3e}")
    assert err <= tol
    N = int(np.prod(shape))
    elem = 8 if storage == "f64" else 4
    assert mem_f[1] == 22 * elem * N and mem_s[1] == (52 if nc_A else 49) * elem * N
    assert mem_s[0] == mem_f[0] + 4 * elem * N


@pytest.mark.parametrize("nc_A", [0.0, 0.01])
def test_split_two_species_full_size_equals_fused(nc_A):
    """The 512 x 256 x 256 two-component box in the launch configuration the
    benchmark times, two drops of radius 40 three nodes apart (so that the
    near-contact force acts), 4 steps: the split schedule equals the fused
    step bit for bit."""
    from paper_2301_01622_amd.lbm import LBM
    nz, ny, nx = 256, 256, 512
    _say(f"two-species split full size {(nz, ny, nx)} FP32 nc_A={nc_A} 4 steps")
    r1, r2, u = I.droplets((nz, ny, nx), centres=[(214.5, 127.6, 128.3), (297.5, 128.4, 127.8)], radius=40.0,
                           velocities=[(0.02, 0.0, 0.0), (-0.02, 0.0, 0.0)])
    prim, uu = torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda()
    del r1, r2, u
    out = []
    for split in (True, False):
        sim = LBM((nx, ny, nz), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, split=split, nc_A=nc_A,
                  nc_hmax=4 if nc_A else 0)
        sim.set_equilibrium(prim, uu)
        sim.step(4)
        out.append(sim.get_moments(torch.float32))
        sim.close()
    same = torch.equal(out[0], out[1])
    _say(f"  bitwise equal: {same}; max |split - fused| {float((out[0] - out[1]).abs().max()):.3e}")
    assert same


def test_split_two_species_equals_fused_over_a_moving_film():
    """Two drops three nodes apart carried by a uniform flow of 0.08 along y
    across a ragged 70 x 44 x 24 box, 80 steps with the near-contact force.
    The film and the interfaces move by more than one 4-row block of the
    force pass, so blocks that held a force become force-free and the fused
    step (which skips the force loads of such blocks) must still equal the
    split schedule (which reads the force arrays everywhere) bit for bit."""
    from paper_2301_01622_amd.lbm import LBM
    nz, ny, nx = 24, 44, 70
    _say(f"two-species split vs fused, moving film {(nz, ny, nx)} FP32 nc_A=0.05 80 steps")
    r1, r2, u = I.droplets((nz, ny, nx), centres=[(27.5, 14.3, 11.6), (42.5, 13.7, 12.2)], radius=6.0,
                           velocities=[(0.01, 0.0, 0.0), (-0.01, 0.0, 0.0)], width=1.0)
    u[1] += 0.08
    prim, uu = torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda()
    out = []
    for split in (True, False):
        sim = LBM((nx, ny, nz), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, split=split, nc_A=0.05,
                  nc_hmax=4)
        sim.set_equilibrium(prim, uu)
        sim.step(80)
        out.append(sim.get_moments(torch.float64).cpu().numpy())
        sim.close()
    same = np.array_equal(out[0], out[1])
    _say(f"  bitwise equal: {same}; max |split - fused| {np.abs(out[0] - out[1]).max():.3e}")
    assert same
    rho1 = out[1][0]
    y = np.arange(ny)[None, :, None]
    inside = rho1 > 0.5
    y0 = float((r1 > 0.5).nonzero()[1].mean())
    y1 = float(np.broadcast_to(y, rho1.shape)[inside].mean())
    _say(f"  species-1 centroid y {y0:.2f} -> {y1:.2f}")
    assert y1 - y0 > 4.0
