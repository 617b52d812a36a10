"""The boundary's equilibrium map and its transpose (the chain from initial
densities and velocity to the initial moments, and back) against the oracle,
with host and device buffers of either precision, and contexts whose state
copies are caller-owned torch buffers."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import inputs as I  # noqa: E402


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def LBM():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_01622_amd.lbm import LBM as cls
    return cls


def _primitive(species, shape, seed):
    rng = np.random.default_rng(seed)
    rho_k = 0.2 + rng.random((species,) + shape)
    u = 0.05 * rng.standard_normal((3,) + shape)
    return rho_k, u


@pytest.mark.parametrize("species", [1, 2])
@pytest.mark.parametrize("where,dtype", [("device", "f64"), ("device", "f32"), ("host", "f64")])
def test_equilibrium_map_matches_oracle(LBM, oracle, species, where, dtype):
    """lbm_equilibrium_moments on a ragged box: FP64 arithmetic, so with FP64
    buffers the moments equal the oracle's to a few units of rounding, with
    FP32 buffers to one FP32 rounding of the inputs and the result."""
    shape = (5, 11, 13)
    nz, ny, nx = shape
    _say(f"equilibrium map species={species} {where} {dtype}")
    rho_k, u = _primitive(species, shape, 40 + species)
    ref = oracle.equilibrium_moments(rho_k[0], u) if species == 1 else \
        oracle.equilibrium_moments2(rho_k[0], rho_k[1], u)
    sim = LBM((nx, ny, nz), 19, 0.8, species=species, storage="f64")
    prim = np.ascontiguousarray(np.concatenate([rho_k, u]))
    if dtype == "f32":
        prim = prim.astype(np.float32)
        ref32 = oracle.equilibrium_moments(prim[0].astype(np.float64), prim[1:].astype(np.float64)) \
            if species == 1 else oracle.equilibrium_moments2(prim[0].astype(np.float64),
                                                             prim[1].astype(np.float64),
                                                             prim[2:].astype(np.float64))
        ref = ref32
    if where == "device":
        got = sim.equilibrium(torch.from_numpy(prim).cuda()).cpu().numpy()
    else:
        out = np.empty((9 + species,) + shape, dtype=prim.dtype)
        got = sim.equilibrium(prim, out=out)
    sim.close()
    tol = 4e-16 if dtype == "f64" else 2 ** -24
    err = np.abs(got.astype(np.float64) - ref).max() / np.abs(ref).max()
    _say(f"  rel err {err:.3e}")
    assert got.dtype == prim.dtype
    assert err <= tol


@pytest.mark.parametrize("species", [1, 2])
@pytest.mark.parametrize("where", ["device", "host"])
def test_equilibrium_adjoint_matches_oracle(LBM, oracle, species, where):
    """lbm_equilibrium_moments_adjoint (FP64) against the oracle's chain
    through the equilibrium map, which is pinned by a dot-product test."""
    shape = (5, 11, 13)
    nz, ny, nx = shape
    _say(f"equilibrium adjoint species={species} {where}")
    rho_k, u = _primitive(species, shape, 50 + species)
    g = np.random.default_rng(60 + species).standard_normal((9 + species,) + shape)
    ref = oracle.equilibrium_adjoint(rho_k[0] if species == 1 else rho_k, u, g)
    sim = LBM((nx, ny, nz), 27, 0.8, species=species, storage="f32")
    prim = np.ascontiguousarray(np.concatenate([rho_k, u]))
    if where == "device":
        got = sim.equilibrium_adjoint(torch.from_numpy(prim).cuda(), torch.from_numpy(g).cuda()).cpu().numpy()
    else:
        got = sim.equilibrium_adjoint(prim, g, out=np.empty_like(prim))
    sim.close()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(f"  rel err {err:.3e}")
    assert err <= 1e-15


@pytest.mark.parametrize("species,storage", [(1, "f32"), (1, "bf16"), (2, "f32")])
def test_caller_owned_state_buffers(LBM, species, storage):
    """A context running on two torch-allocated state buffers gives the same
    moments bit for bit as one whose buffers the library allocates, keeps its
    state in those buffers, and leaves them to the caller after closing."""
    shape = (21, 18, 33)
    nz, ny, nx = shape
    _say(f"caller-owned state buffers species={species} {storage}")
    if species == 1:
        rho, u = I.random_solenoidal_box(24, seed=I.SEED_C2, umax=1e-2)
        rho, u = np.ascontiguousarray(rho[:nz, :ny, :24]), np.ascontiguousarray(u[:, :nz, :ny, :24])
        shape = rho.shape
        prim = (torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    else:
        r1, r2, u = I.droplets(shape, centres=[(10.0, 9.0, 10.0), (23.0, 9.0, 10.0)], radius=5.0,
                               velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
        prim = (torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda())
    nz, ny, nx = shape
    kw = dict(species=species, storage=storage, sigma=0.01, beta=0.7)
    need = LBM.state_bytes_for((nx, ny, nz), 19, species, storage=storage)
    bufs = [torch.full((need,), 7, dtype=torch.uint8, device="cuda") for _ in range(2)]
    own = LBM((nx, ny, nz), 19, 0.8, **kw)
    ext = LBM((nx, ny, nz), 19, 0.8, state_buffers=bufs, **kw)
    assert ext.state_bytes == need == own.state_bytes
    results = []
    for sim in (own, ext):
        sim.set_equilibrium(*prim)
        sim.step(7)
        results.append(sim.get_moments(torch.float64))
    saved = ext.new_checkpoint()
    ext.save_state(saved)
    # Every launch flips the pair: 7 steps are 3 two-step sweeps and one
    # single step where the context runs sweeps, else 7 single steps.
    launches = 4 if ext.sweeps else 7
    cur = bufs[launches % 2]
    torch.cuda.synchronize()
    own.close()
    ext.close()
    assert torch.equal(results[0], results[1])
    # the context's state lives in the caller's buffer, which outlives it
    assert torch.equal(saved, cur)
    assert not torch.equal(bufs[0], bufs[1])
