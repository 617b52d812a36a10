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
