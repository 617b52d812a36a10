"""GPU parity of the near-contact force (the LBNCI term of Sec. III.B, under
the readings stated in csrc/nc_force.hip and the oracle) for both
two-component schemes, against the FP64 oracle: two drops whose interfaces
are a few nodes apart, so that films are found by the probes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402

TAU, SIGMA, BETA = 0.8, 0.01, 0.7
AH, HMAX = 0.05, 4


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def LBM():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_01622_amd.lbm import LBM as _LBM
    return _LBM


def _contact_state(oracle, shape, gap=3.0, R=5.0):
    nz, ny, nx = shape
    c1 = (nx / 2 - gap / 2 - R, ny / 2 + 0.3, nz / 2 - 0.2)
    c2 = (nx / 2 + gap / 2 + R, ny / 2 - 0.4, nz / 2 + 0.1)
    r1, r2, u = I.droplets(shape, centres=[c1, c2], radius=R, velocities=[(0.02, 0, 0), (-0.02, 0, 0)], width=1.0)
    return np.ascontiguousarray(oracle.equilibrium_moments2(r1, r2, u)), r1


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("shape", [(14, 17, 31), (14, 17, 132)])
def test_near_contact_moment_scheme_matches_oracle(LBM, oracle, q, storage, tol, shape):
    # nx = 132: three 64-wide block columns of the force pass, the last one
    # 4 nodes wide, and the film across the first column boundary.
    _say(f"near-contact moment scheme {shape} D3Q{q} {storage} 6 steps")
    H, r1 = _contact_state(oracle, shape)
    F, h = oracle.nc_force(2 * r1 - 1, q, AH, HMAX)
    assert (h > 0).sum() > 20  # films are found between the drops
    A = oracle.sigma_to_A(SIGMA, TAU)
    ref = oracle.cg_moment_run(H, q, TAU, A, BETA, 6, Ah=AH, hmax=HMAX)
    free = oracle.cg_moment_run(H, q, TAU, A, BETA, 6)
    assert np.abs(ref - free).max() > 1e-4  # the force matters
    nf, nz, ny, nx = H.shape
    sim = LBM((nx, ny, nz), q, TAU, species=2, storage=storage, sigma=SIGMA, beta=BETA, nc_A=AH, nc_hmax=HMAX)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(6)
    got = sim.get_moments(torch.float64).cpu().numpy()
    sim.close()
    err = np.abs(got - ref).max(axis=(1, 2, 3))
    _say(f"  max err per field {err}")
    assert err.max() <= tol


@pytest.mark.parametrize("q", [19, 27])
def test_near_contact_population_scheme_matches_oracle(LBM, oracle, q):
    shape = (14, 17, 31)
    _say(f"near-contact population scheme {shape} D3Q{q} f32 6 steps")
    H, _ = _contact_state(oracle, shape)
    A = oracle.sigma_to_A(SIGMA, TAU)
    f1, f2 = oracle.cg_populations_from_moments(H, q)
    g1, g2 = oracle.cg_population_run(f1, f2, q, TAU, A, BETA, 6, Ah=AH, hmax=HMAX)
    ref = oracle.cg_moments_from_populations(g1, g2, q)
    nf, nz, ny, nx = H.shape
    sim = LBM((nx, ny, nz), q, TAU, species=2, storage="f32", sigma=SIGMA, beta=BETA, scheme="population",
              nc_A=AH, nc_hmax=HMAX)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(6)
    got = sim.get_moments(torch.float64).cpu().numpy()
    sim.close()
    err = np.abs(got - ref).max(axis=(1, 2, 3))
    _say(f"  max err per field {err}")
    assert err.max() <= 5e-6


def test_near_contact_rejects_adjoint(LBM):
    import ctypes
    from paper_2301_01622_amd import _lib
    sim = LBM((8, 8, 8), 19, TAU, species=2, storage="f32", sigma=SIGMA, beta=BETA, nc_A=AH, nc_hmax=HMAX)
    st = sim.new_checkpoint()
    lam, lo = sim.new_costate(), sim.new_costate()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert sim._lib.lbm_adjoint_step_stored(sim._ctx, p(st), p(lam), p(lo), None) == _lib.LBM_ESTATE
    sim.close()


@pytest.mark.parametrize("hmax", [1, 2, 3, 7])
@pytest.mark.parametrize("shape", [(20, 21, 70), (3, 4, 5)])
def test_near_contact_probe_ranges_and_ragged_tiles(LBM, oracle, hmax, shape):
    """Probe ranges within one batch of four probe loads and beyond it, on a
    box with ragged 64 x 4 launch tiles and on one shorter than the probe
    range (probes wrap, some several times); random phase field, so films
    are found all over the box."""
    nz, ny, nx = shape
    q = 27
    _say(f"near-contact probes h_max={hmax} {shape} D3Q{q} f64 2 steps")
    rng = np.random.default_rng(1000 + hmax)
    r1 = rng.uniform(0.35, 0.65, shape)
    r2 = 1.0 - r1 + rng.uniform(-0.05, 0.05, shape)
    u = rng.uniform(-0.02, 0.02, (3,) + shape)
    H = np.ascontiguousarray(oracle.equilibrium_moments2(r1, r2, u))
    F, h = oracle.nc_force(2 * r1 / (r1 + r2) - 1, q, AH, hmax)
    assert (h > 0).sum() > 0
    A = oracle.sigma_to_A(SIGMA, TAU)
    ref = oracle.cg_moment_run(H, q, TAU, A, BETA, 2, Ah=AH, hmax=hmax)
    sim = LBM((nx, ny, nz), q, TAU, species=2, storage="f64", sigma=SIGMA, beta=BETA, nc_A=AH, nc_hmax=hmax)
    sim.set_moments(torch.from_numpy(H).cuda())
    sim.step(2)
    got = sim.get_moments(torch.float64).cpu().numpy()
    sim.close()
    err = np.abs(got - ref).max()
    _say(f"  max err {err:.3e}")
    assert err <= 1e-12


def _sampled_nc(oracle, r1, r2, u, q, scheme, nodes, Ah, hmax):
    """One step of the oracle on the periodic block of radius hmax + 2 around
    each node: the node's new moments depend on the forces one node away,
    and those on the phase field up to h_max nodes further."""
    r = hmax + 2
    A = oracle.sigma_to_A(SIGMA, TAU)
    out = []
    for (z, y, x) in nodes:
        idx = [np.arange(c - r, c + r + 1) for c in (z, y, x)]

        def cut(a):
            return np.ascontiguousarray(a.take(idx[0], axis=-3, mode="wrap").take(idx[1], axis=-2, mode="wrap")
                                        .take(idx[2], axis=-1, mode="wrap"))
        H = np.ascontiguousarray(oracle.equilibrium_moments2(cut(r1), cut(r2), cut(u)))
        if scheme == "moment":
            res = oracle.cg_moment_run(H, q, TAU, A, BETA, 1, Ah=Ah, hmax=hmax)
        else:
            f1, f2 = oracle.cg_populations_from_moments(H, q)
            g1, g2 = oracle.cg_population_run(f1, f2, q, TAU, A, BETA, 1, Ah=Ah, hmax=hmax)
            res = oracle.cg_moments_from_populations(g1, g2, q)
        out.append(res[:, r, r, r])
    return np.array(out)


@pytest.mark.parametrize("scheme", ["moment", "population"])
def test_full_size_near_contact_sampled(LBM, oracle, scheme):
    """512 x 256 x 256 D3Q19 FP32 with the near-contact force (A_h = 0.01,
    h_max = 4), in the launch configuration of the benchmark: two drops of
    radius 40 three nodes apart, one step, nodes in the film between them,
    on the interfaces, in the drops, in the carrier and at the box corners,
    node by node against the oracle."""
    shape = (256, 256, 512)
    Ah, hmax = 0.01, 4
    _say(f"512x256x256 near-contact {scheme} scheme sampled, 1 step")
    c1, c2 = (256 - 1.5 - 40, 128.3, 127.8), (256 + 1.5 + 40, 127.6, 128.1)
    r1, r2, u = I.droplets(shape, centres=[c1, c2], radius=40.0, velocities=[(0.02, 0, 0), (-0.02, 0, 0)],
                           width=1.0)
    sim = LBM((512, 256, 256), 19, TAU, species=2, storage="f32", sigma=SIGMA, beta=BETA, scheme=scheme,
              nc_A=Ah, nc_hmax=hmax)
    sim.set_equilibrium(torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda())
    sim.step(1)
    got = sim.get_moments(torch.float64).cpu().numpy()
    sim.close()
    rng = np.random.default_rng(11)
    film = [(128, 128, 256), (128, 128, 255), (128, 128, 257), (130, 126, 256), (125, 131, 254), (128, 136, 256)]
    film += [(128 + int(rng.integers(-6, 7)), 128 + int(rng.integers(-6, 7)), 256 + int(rng.integers(-3, 4)))
             for _ in range(8)]
    nodes = list(film) + [(0, 0, 0), (255, 255, 511), (128, 128, 176), (128, 128, 336)]
    for _ in range(8):
        c = [(127.8, 128.3, c1[0]), (128.1, 127.6, c2[0])][rng.integers(2)]
        d = rng.standard_normal(3)
        d *= 40.0 / np.linalg.norm(d)
        nodes.append(tuple(int(round(c[k] + d[k])) % shape[k] for k in range(3)))
    nodes += [(int(rng.integers(0, 256)), int(rng.integers(0, 256)), int(rng.integers(0, 512))) for _ in range(6)]
    ref = _sampled_nc(oracle, r1, r2, u, 19, scheme, nodes, Ah, hmax)
    free = _sampled_nc(oracle, r1, r2, u, 19, scheme, film, 0.0, 0)
    assert np.abs(ref[:len(film)] - free).max() > 1e-5  # the force acts in the film
    g = np.array([got[:, z, y, x] for (z, y, x) in nodes])
    err = np.abs(g - ref).max(axis=0)
    _say(f"  max err per field {err}")
    assert err.max() <= 2e-6


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_phase_field_reuse_across_steps_is_exact(LBM, oracle, storage):
    """The step writes the phase field of its output for the next step's
    force; the state after six steps is bitwise the same when that reuse is
    interrupted by a reload of the state, and when a step of other buffers
    (which overwrites the scratch) comes between two steps."""
    shape = (14, 17, 70)
    _say(f"near-contact phase-field reuse {shape} D3Q19 {storage}")
    H, _ = _contact_state(oracle, shape)
    nf, nz, ny, nx = H.shape

    def fresh():
        s = LBM((nx, ny, nz), 19, TAU, species=2, storage=storage, sigma=SIGMA, beta=BETA, nc_A=AH, nc_hmax=HMAX)
        s.set_moments(torch.from_numpy(H).cuda())
        return s

    a = fresh()
    a.step(6)
    ref = a.get_moments(torch.float64)
    b = fresh()
    b.step(3)
    st = b.new_checkpoint()
    b.save_state(st)
    b.load_state(st)
    b.step(3)
    c = fresh()
    c.step(2)
    x, y = c.new_checkpoint(), c.new_checkpoint()
    a.save_state(x)  # another state, six steps on
    c.step_state(x, y)
    c.step(4)
    for s in (b, c):
        assert torch.equal(s.get_moments(torch.float64), ref)
    for s in (a, b, c):
        s.close()
