"""Host logic of the checkpointed rollout (paper_2301_01622_amd/autograd.py),
on the CPU with a stand-in context whose "states" are step counts and whose
adjoint steps record the state they linearise about: every recomputed
state must be the right one, the reverse steps must visit t = T-1 ... 0 in
order, pairs of reverse steps must use (t, t-1), and none may be missing or
repeated, for one- and two-step passes and any checkpoint interval."""
import pytest

torch = pytest.importorskip("torch")

from paper_2301_01622_amd import autograd as AG  # noqa: E402


class FakeSim:
    """States are 1-element tensors holding the step count they represent;
    a co-state is a tensor whose first entry counts reverse steps."""

    def __init__(self, sweeps: bool):
        self.scheme, self.species, self.tau, self.sweeps = "moment", 1, 0.8, sweeps
        self.nfields, self.shape = 10, (1, 1, 1)
        self.real_dtype = torch.float64
        self.t = 0
        self.reverse = []  # state times the reverse steps linearised about, in order

    # forward
    def set_moments(self, M):
        self.t = 0

    def new_checkpoint(self):
        return torch.zeros(1, dtype=torch.float64)

    def save_state(self, buf):
        buf[0] = self.t

    def step(self, n):
        self.t += n

    def get_moments(self, dtype):
        return torch.full((10, 1, 1, 1), float(self.t), dtype=dtype)

    # the equilibrium map: a primitive (rho, u) of all zeros maps to the state
    # at step 0; its transpose passes the co-state's first entry to every
    # primitive field
    def equilibrium(self, prim):
        assert prim.shape == (4, 1, 1, 1)
        return torch.zeros((10, 1, 1, 1), dtype=prim.dtype)

    def equilibrium_adjoint(self, prim, g):
        assert prim.shape == (4, 1, 1, 1) and g.shape == (10, 1, 1, 1)
        return torch.full((4, 1, 1, 1), float(g[0, 0, 0, 0]), dtype=prim.dtype)

    # reverse
    def new_costate(self):
        return torch.zeros(1, dtype=torch.float64)

    def costate_to_stored(self, pub, lam):
        lam[0] = 0

    def costate_from_stored(self, lam, pub):
        pub.fill_(float(lam[0]))

    def step_state(self, src, dst):
        dst[0] = src[0] + 1

    def step_state2(self, src, mid, dst):
        assert self.sweeps
        mid[0] = src[0] + 1
        dst[0] = src[0] + 2

    def adjoint_step_stored(self, state, lam, lam_out, dtau):
        self.reverse.append(int(state[0]))
        lam_out[0] = lam[0] + 1
        dtau += 1.0

    def adjoint_step2_stored(self, state_t1, state_t0, lam, lam_out, dtau):
        assert self.sweeps and int(state_t1[0]) == int(state_t0[0]) + 1
        self.reverse += [int(state_t1[0]), int(state_t0[0])]
        lam_out[0] = lam[0] + 2
        dtau += 2.0


@pytest.mark.parametrize("sweeps", [False, True])
@pytest.mark.parametrize("T,K", [(1, 1), (7, 1), (7, 3), (8, 4), (13, 5), (12, 12), (5, 20)])
def test_reverse_steps_visit_every_state_once(sweeps, T, K):
    sim = FakeSim(sweeps)
    M0 = torch.zeros((10, 1, 1, 1), dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    MT = AG.rollout(sim, M0, tau, T, K=K)
    assert float(MT[0, 0, 0, 0]) == T
    MT.sum().backward()
    assert sim.reverse == list(range(T - 1, -1, -1))
    assert float(M0.grad[0, 0, 0, 0]) == T          # one co-state update per step
    assert float(tau.grad) == T                     # one sensitivity term per step


@pytest.mark.parametrize("sweeps", [False, True])
@pytest.mark.parametrize("T,K", [(1, 1), (7, 3), (8, 4)])
def test_rollout_from_primitive_fields(sweeps, T, K):
    """MomentLBRollout.apply(rho, u0, tau, sim, n, K): the same schedule,
    with the co-state of M0 handed to the transpose of the equilibrium map
    and split into the gradients of rho and u0."""
    sim = FakeSim(sweeps)
    rho = torch.zeros((1, 1, 1), dtype=torch.float64, requires_grad=True)
    u0 = torch.zeros((3, 1, 1, 1), dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    MT = AG.MomentLBRollout.apply(rho, u0, tau, sim, T, K)
    assert float(MT[0, 0, 0, 0]) == T
    MT.sum().backward()
    assert sim.reverse == list(range(T - 1, -1, -1))
    assert rho.grad.shape == rho.shape and u0.grad.shape == u0.shape
    assert float(rho.grad.flatten()[0]) == T and torch.all(u0.grad == T)
    assert float(tau.grad) == T
