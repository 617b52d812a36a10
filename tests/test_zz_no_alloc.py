"""The allocation-free reverse step (lbm_adjoint_step_stored_noalloc) through
the C ABI against lbm_adjoint_step_stored: identical co-states and dL/dtau,
bit for bit, on two calls in a row, the second on a smaller box (the static
scratch still holds the first call's larger co-state), for two species in
FP32 and FP64 and for one species; and the refusal of a box whose
colour-gradient co-state exceeds the static maximum."""
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
    from paper_2301_01622_amd import _lib
    from paper_2301_01622_amd.lbm import LBM
    return LBM, _lib


def _case(LBM, _lib, oracle, dims, species, storage, seed):
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    if species == 1:
        M = I.random_moments(shape, seed=seed)
    else:
        r1, r2, u = I.droplets(shape, centres=[(nx * 0.3, ny * 0.45, nz * 0.5), (nx * 0.7, ny * 0.55, nz * 0.5)],
                               radius=min(shape) * 0.25, velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
        M = oracle.equilibrium_moments2(r1, r2, u)
    lam = np.random.default_rng(seed + 1).standard_normal(M.shape)
    sim = LBM(dims, 19, 0.8, species=species, storage=storage, sigma=0.01, beta=0.7)
    sim.set_moments(torch.from_numpy(M).cuda())
    st = sim.new_checkpoint()
    sim.save_state(st)
    lam_in = sim.new_costate()
    sim.costate_to_stored(torch.from_numpy(lam).to(sim.real_dtype).cuda().contiguous(), lam_in)
    out_ref, out_na = sim.new_costate(), sim.new_costate()
    out_na.fill_(float("nan"))
    d_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    d_na = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = _lib.load()
    p = ctypes.c_void_p
    _say(f"no-alloc reverse step {dims} species={species} {storage}")
    sim.adjoint_step_stored(st, lam_in, out_ref, d_ref)
    rc = lib.lbm_adjoint_step_stored_noalloc(sim._ctx, p(st.data_ptr()), p(lam_in.data_ptr()),
                                             p(out_na.data_ptr()), p(d_na.data_ptr()))
    assert rc == _lib.LBM_OK, lib.lbm_last_error(sim._ctx)
    torch.cuda.synchronize()
    # slots of the blocked layout that belong to no node are left untouched
    pub_ref = torch.empty((sim.nfields,) + sim.shape, dtype=sim.real_dtype, device="cuda")
    pub_na = torch.empty_like(pub_ref)
    sim.costate_from_stored(out_ref, pub_ref)
    sim.costate_from_stored(out_na, pub_na)
    torch.cuda.synchronize()
    sim.close()
    assert torch.equal(pub_na, pub_ref)
    assert float(d_na) == float(d_ref) and float(d_ref) != 0.0


@pytest.mark.parametrize("species,storage", [(2, "f32"), (2, "f64"), (1, "f32")])
def test_noalloc_reverse_step_matches_the_allocating_one(mods, oracle, species, storage):
    LBM, _lib = mods
    _case(LBM, _lib, oracle, (70, 37, 23), species, storage, seed=11)
    _case(LBM, _lib, oracle, (21, 13, 9), species, storage, seed=13)


def test_noalloc_refuses_beyond_the_static_scratch(mods):
    """512 x 512 x 32 two-species FP32: the colour-gradient co-state takes
    3 x 4 B x 8.4 M = 100 MB > 64 MiB, refused before any launch."""
    LBM, _lib = mods
    sim = LBM((512, 512, 32), 19, 0.8, species=2, storage="f32")
    st = sim.new_checkpoint()
    a, b = sim.new_costate(), sim.new_costate()
    lib = _lib.load()
    p = ctypes.c_void_p
    rc = lib.lbm_adjoint_step_stored_noalloc(sim._ctx, p(st.data_ptr()), p(a.data_ptr()), p(b.data_ptr()), None)
    msg = lib.lbm_last_error(sim._ctx).decode()
    sim.close()
    assert rc == _lib.LBM_EINVAL
    assert "static scratch" in msg
