"""Differentiable rollouts of the moment-only step (one or two species).

``rollout(sim, M0, tau, nsteps, K)`` returns M(T) after ``nsteps`` steps from
the public moments ``M0`` (shape (10, nz, ny, nx) for one species, (11, nz,
ny, nx) for two: rho1, rho2, j, P); the result carries an autograd graph
whose backward is the library's discrete adjoint step:

  forward : the state is saved every K steps (device copies of the stored
            state) while the library advances the fluid;
  backward: for each segment, last first, the K states are recomputed from
            its checkpoint straight into K buffers (``lbm_step_state``), then
            K adjoint steps (``lbm_adjoint_step``) carry the co-state back and
            add each step's dL/dtau on the device (FP64).

Per step of the backward pass the device moves one forward step (recompute)
plus one adjoint step; no state is copied besides the checkpoints, and the
co-state stays in the library's stored layout until the end.  Where the
context runs two-step sweeps, pairs of states are recomputed in one pass
(``lbm_step_state2``) and pairs of adjoint steps run in one pass
(``lbm_adjoint_step2_stored``), with the same results.
``tau`` is a 0-d tensor whose value must equal the context's relaxation
time; its gradient is dL/dtau (two species: at fixed surface tension sigma,
so the perturbation amplitude A = 9 sigma/(2 tau) moves with tau).  The
gradient to M0 does not depend on K (bit for bit), dL/dtau up to FP64
rounding of how the per-step sums are grouped.
"""
from __future__ import annotations

import torch


class MomentLBRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M0: torch.Tensor, tau: torch.Tensor, sim, nsteps: int, K: int):
        if sim.scheme != "moment":
            raise ValueError("rollout: moment scheme only")
        if M0.shape[0] != (11 if sim.species == 2 else 10):
            raise ValueError("rollout: M0 must hold the public moment fields of the context")
        if abs(float(tau) - sim.tau) > 1e-12 * sim.tau:
            raise ValueError("rollout: tau must equal the context's relaxation time")
        if nsteps < 1 or K < 1:
            raise ValueError("rollout: nsteps and K must be positive")
        sim.set_moments(M0.detach().contiguous())
        ckpts = []
        done = 0
        while done < nsteps:
            buf = sim.new_checkpoint()
            sim.save_state(buf)
            ckpts.append(buf)
            n = min(K, nsteps - done)
            sim.step(n)
            done += n
        MT = sim.get_moments(dtype=M0.dtype)
        ctx.sim, ctx.nsteps, ctx.K, ctx.ckpts = sim, nsteps, K, ckpts
        ctx.M0_dtype = M0.dtype
        return MT

    @staticmethod
    def backward(ctx, grad_MT: torch.Tensor):
        sim, nsteps, K, ckpts = ctx.sim, ctx.nsteps, ctx.K, ctx.ckpts
        rdt = sim.real_dtype
        # The co-state stays in the library's stored layout between steps.
        pub = grad_MT.to(rdt).contiguous()
        lam, lam_b = sim.new_costate(), sim.new_costate()
        sim.costate_to_stored(pub, lam)
        dtau = torch.zeros(1, dtype=torch.float64, device=pub.device)
        slots = [None] + [sim.new_checkpoint() for _ in range(min(K, nsteps) - 1)]
        pairs = getattr(sim, "sweeps", False)
        for s in reversed(range(len(ckpts))):
            n = min(K, nsteps - s * K)
            slots[0] = ckpts[s]
            t = 1
            while t < n:
                if pairs and t + 1 < n:
                    sim.step_state2(slots[t - 1], slots[t], slots[t + 1])
                    t += 2
                else:
                    sim.step_state(slots[t - 1], slots[t])
                    t += 1
            t = n - 1
            while t >= 0:
                if pairs and t >= 1:
                    sim.adjoint_step2_stored(slots[t], slots[t - 1], lam, lam_b, dtau)
                    t -= 2
                else:
                    sim.adjoint_step_stored(slots[t], lam, lam_b, dtau)
                    t -= 1
                lam, lam_b = lam_b, lam
        sim.costate_from_stored(lam, pub)
        grad_M0 = pub.to(ctx.M0_dtype)
        grad_tau = dtau.reshape(()).to(grad_MT.dtype)
        return grad_M0, grad_tau, None, None, None


def rollout(sim, M0: torch.Tensor, tau: torch.Tensor, nsteps: int, K: int = 20) -> torch.Tensor:
    """M(T) with gradients to M0 and tau (see the module docstring)."""
    return MomentLBRollout.apply(M0, tau, sim, nsteps, K)


def equilibrium_moments(rho: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Public moments with zero non-equilibrium part from (rho, u), as
    differentiable torch operations (the chain from an initial velocity field
    to M0): j = rho u, P = rho c_s^2 I + rho u u."""
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    rows = [rho] + [rho * u[a] for a in range(3)]
    rows += [rho * u[a] * u[b] + (rho / 3.0 if a == b else 0.0) for a, b in pairs]
    return torch.stack(rows, dim=0)


def equilibrium_moments2(rho1: torch.Tensor, rho2: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Two-species public moments (rho1, rho2, j, P) with zero non-equilibrium
    part from the species densities and a shared velocity, as differentiable
    torch operations: rho = rho1 + rho2, j = rho u, P = rho c_s^2 I + rho u u."""
    rho = rho1 + rho2
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    rows = [rho1, rho2] + [rho * u[a] for a in range(3)]
    rows += [rho * u[a] * u[b] + (rho / 3.0 if a == b else 0.0) for a, b in pairs]
    return torch.stack(rows, dim=0)
