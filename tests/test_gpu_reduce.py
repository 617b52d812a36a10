"""GPU parity of the FP64 global reductions (lbm_reduce): the per-species
masses and the momentum totals of the state, summed on the device in FP64.

Two independent checks per scheme and storage format, after T steps from a
seeded state whose totals are all distinct and non-zero (so a reduction that
read the wrong field, or mapped rho1 and rho2 the wrong way round, fails):

  * the kernel: lbm_reduce against FP64 sums of the same state read back with
    lbm_get_moments, to 1e-12 of the summed magnitudes (both sides sum the
    same stored values, in different orders);
  * the method: lbm_reduce against the totals of the FP64 oracle's state
    after the same steps, to the per-node tolerance of the storage format
    times sqrt(N) (independent rounding errors of N nodes).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402

SHAPE = (23, 29, 37)  # (nz, ny, nx): several tiles, ragged on every axis
NODE_TOL = {"f64": 1e-12, "f32": 1e-6}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _totals(H, species):
    """(sum rho1 | sum rho, sum rho2 | 0, sum j) of a public moment array."""
    if species == 1:
        return np.array([H[0].sum(), 0.0, H[1].sum(), H[2].sum(), H[3].sum()])
    return np.array([H[0].sum(), H[1].sum(), H[2].sum(), H[3].sum(), H[4].sum()])


def _magnitudes(H, species):
    if species == 1:
        return np.array([np.abs(H[0]).sum(), 1.0, *(np.abs(H[1 + a]).sum() for a in range(3))])
    return np.array([np.abs(H[k]).sum() for k in range(5)])


def _two_drops():
    nz, ny, nx = SHAPE
    r1, r2, u = I.droplets(SHAPE, centres=[(nx * 0.3, ny * 0.45, nz * 0.5), (nx * 0.72, ny * 0.55, nz * 0.5)],
                           radius=6.0, velocities=[(0.05, 0.02, -0.01), (-0.03, 0.01, 0.02)])
    return r1, r2, u


def _check(sim, ref, species, storage, what):
    N = sim.n_nodes
    red = sim.reduce()
    got = sim.get_moments(torch.float64).cpu().numpy()
    own = _totals(got, species)
    mag = _magnitudes(got, species)
    k_err = np.abs(red - own)
    _say(f"  {what}: reduce {red}")
    _say(f"  {what}: |reduce - sum(get_moments)| {k_err}")
    assert (k_err <= 1e-12 * mag).all(), (red, own)
    o_err = np.abs(red - _totals(ref, species))
    _say(f"  {what}: |reduce - oracle totals| {o_err}")
    assert (o_err <= NODE_TOL[storage] * np.sqrt(N)).all(), (red, _totals(ref, species))
    # the totals are distinct, so a swapped or shifted field cannot pass
    assert len({round(v, 6) for v in red}) == 5


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("steps", [0, 7])
def test_reduce_one_species_moment(oracle, storage, steps):
    from paper_2301_01622_amd.lbm import LBM
    q, tau = 19, 0.7
    _say(f"reduce one species moment {storage} {SHAPE} D3Q{q} {steps} steps")
    H = I.random_moments(SHAPE, seed=7)
    H[1] += 0.003  # non-zero, distinct momentum totals
    H[2] -= 0.002
    H[3] += 0.001
    ref = oracle.moment_run(H, q, tau, steps)
    nz, ny, nx = SHAPE
    sim = LBM((nx, ny, nz), q, tau, storage=storage)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(steps)
    _check(sim, ref, 1, storage, "moment")
    sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("steps", [0, 5])
def test_reduce_two_species_moment(oracle, storage, steps):
    from paper_2301_01622_amd.lbm import LBM
    q, tau, sigma, beta = 19, 0.8, 0.01, 0.7
    _say(f"reduce two species moment {storage} {SHAPE} D3Q{q} {steps} steps")
    r1, r2, u = _two_drops()
    H = oracle.equilibrium_moments2(r1, r2, u)
    ref = oracle.cg_moment_run(H, q, tau, oracle.sigma_to_A(sigma, tau), beta, steps)
    nz, ny, nx = SHAPE
    sim = LBM((nx, ny, nz), q, tau, species=2, storage=storage, sigma=sigma, beta=beta)
    sim.set_equilibrium(torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda())
    sim.step(steps)
    _check(sim, ref, 2, storage, "moment, two species")
    sim.close()


@pytest.mark.parametrize("scheme,storage,steps", [
    ("population", "f64", 4), ("population", "f32", 4),
    ("population_aa", "f64", 3), ("population_aa", "f64", 4), ("population_aa", "f32", 3),
])
def test_reduce_population_baselines(oracle, scheme, storage, steps):
    """The baselines' totals, including the in-place scheme after an odd
    number of steps (populations in the reversed slots)."""
    from paper_2301_01622_amd.lbm import LBM
    q, tau = 19, 0.7
    _say(f"reduce {scheme} {storage} {SHAPE} D3Q{q} {steps} steps")
    H = I.random_moments(SHAPE, seed=8)
    H[1] += 0.003
    H[2] -= 0.002
    H[3] += 0.001
    f = oracle.populations_from_moments(H, q)
    ref = oracle.moments_from_populations(oracle.population_run(f, q, tau, steps), q)
    nz, ny, nx = SHAPE
    sim = LBM((nx, ny, nz), q, tau, storage=storage, scheme=scheme)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(steps)
    _check(sim, ref, 1, storage, scheme)
    sim.close()


@pytest.mark.parametrize("steps", [0, 4])
def test_reduce_two_species_population(oracle, steps):
    from paper_2301_01622_amd.lbm import LBM
    q, tau, sigma, beta = 19, 0.8, 0.01, 0.7
    _say(f"reduce two species population f32 {SHAPE} D3Q{q} {steps} steps")
    r1, r2, u = _two_drops()
    H = oracle.equilibrium_moments2(r1, r2, u)
    f1, f2 = oracle.cg_populations_from_moments(H, q)
    g1, g2 = oracle.cg_population_run(f1, f2, q, tau, oracle.sigma_to_A(sigma, tau), beta, steps)
    ref = oracle.cg_moments_from_populations(g1, g2, q)
    nz, ny, nx = SHAPE
    sim = LBM((nx, ny, nz), q, tau, species=2, storage="f32", sigma=sigma, beta=beta, scheme="population")
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(steps)
    _check(sim, ref, 2, "f32", "population, two species")
    sim.close()
