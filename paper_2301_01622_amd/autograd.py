"""Differentiable rollouts of the moment-only step (one or two species).

``MomentLBRollout.apply(rho_k, u0, tau, sim, nsteps, K)`` returns the public
moments M(T) after ``nsteps`` steps from the equilibrium state of the initial
densities ``rho_k`` (shape (nz, ny, nx) for one species, (2, nz, ny, nx) for
two) and velocity ``u0`` (3, nz, ny, nx); ``rollout(sim, M0, tau, nsteps, K)``
does the same from a given moment state M0 (shape (10, nz, ny, nx) for one
species, (11, nz, ny, nx) for two: rho1, rho2, j, P).  The results carry an
autograd graph whose backward runs the library's discrete adjoint:

  forward : M0 from (rho_k, u0) by the library's equilibrium map
            (``lbm_equilibrium_moments``); the state is saved every K steps
            (device copies of the stored state) while the library advances
            the fluid;
  backward: for each segment, last first, the K states are recomputed from
            its checkpoint straight into K buffers (``lbm_step_state``), then
            K adjoint steps (``lbm_adjoint_step_stored``) carry the co-state
            back and add each step's dL/dtau on the device (FP64); the
            gradient of M0 goes through the transpose of the equilibrium map
            (``lbm_equilibrium_moments_adjoint``) to rho_k and u0.

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
rounding of how the per-step sums are grouped.  This module only marshals
tensors and calls the library; every step of the method, forward and
reverse, runs in its kernels.
"""
from __future__ import annotations

import torch


def _check_common(sim, tau, nsteps: int, K: int) -> None:
    if sim.scheme != "moment":
        raise ValueError("rollout: moment scheme only")
    if abs(float(tau) - sim.tau) > 1e-12 * sim.tau:
        raise ValueError("rollout: tau must equal the context's relaxation time")
    if nsteps < 1 or K < 1:
        raise ValueError("rollout: nsteps and K must be positive")


def _run_forward(sim, M0: torch.Tensor, nsteps: int, K: int):
    """Advances the context from M0, saving the state every K steps; returns
    (M(T) in M0's dtype, the checkpoints)."""
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
    return sim.get_moments(dtype=M0.dtype), ckpts


def _run_backward(sim, ckpts, nsteps: int, K: int, grad_MT: torch.Tensor):
    """Reverse pass over the checkpointed segments; returns (dL/dM0 in the
    kernels' real type, public layout; dL/dtau as a 1-element FP64 tensor)."""
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
    return pub, dtau


def _primitive(sim, rho_k: torch.Tensor, u0: torch.Tensor) -> torch.Tensor:
    """(rho | rho1, rho2, ux, uy, uz) as one contiguous buffer."""
    return torch.cat([rho_k.reshape((sim.species,) + sim.shape), u0.to(rho_k.dtype)], dim=0).contiguous()


class StateRollout(torch.autograd.Function):
    """M(T) from a moment state M0, differentiable in M0 and tau."""

    @staticmethod
    def forward(ctx, M0: torch.Tensor, tau: torch.Tensor, sim, nsteps: int, K: int):
        _check_common(sim, tau, nsteps, K)
        if M0.shape[0] != sim.nfields:
            raise ValueError("rollout: M0 must hold the public moment fields of the context")
        MT, ckpts = _run_forward(sim, M0, nsteps, K)
        ctx.sim, ctx.nsteps, ctx.K, ctx.ckpts = sim, nsteps, K, ckpts
        ctx.M0_dtype = M0.dtype
        return MT

    @staticmethod
    def backward(ctx, grad_MT: torch.Tensor):
        pub, dtau = _run_backward(ctx.sim, ctx.ckpts, ctx.nsteps, ctx.K, grad_MT)
        return pub.to(ctx.M0_dtype), dtau.reshape(()).to(grad_MT.dtype), None, None, None


class MomentLBRollout(torch.autograd.Function):
    """M(T) from initial densities rho_k and velocity u0 (the state starts at
    the equilibrium of those fields), differentiable in rho_k, u0 and tau."""

    @staticmethod
    def forward(ctx, rho_k: torch.Tensor, u0: torch.Tensor, tau: torch.Tensor, sim, nsteps: int, K: int = 20):
        _check_common(sim, tau, nsteps, K)
        prim = _primitive(sim, rho_k.detach(), u0.detach())
        M0 = sim.equilibrium(prim)
        MT, ckpts = _run_forward(sim, M0, nsteps, K)
        ctx.sim, ctx.nsteps, ctx.K, ctx.ckpts = sim, nsteps, K, ckpts
        ctx.prim, ctx.rho_shape, ctx.rho_dtype, ctx.u_dtype = prim, rho_k.shape, rho_k.dtype, u0.dtype
        return MT

    @staticmethod
    def backward(ctx, grad_MT: torch.Tensor):
        sim = ctx.sim
        pub, dtau = _run_backward(sim, ctx.ckpts, ctx.nsteps, ctx.K, grad_MT)
        g = sim.equilibrium_adjoint(ctx.prim, pub.to(ctx.prim.dtype))
        s = sim.species
        grad_rho = g[:s].reshape(ctx.rho_shape).to(ctx.rho_dtype)
        grad_u = g[s:].to(ctx.u_dtype)
        return grad_rho, grad_u, dtau.reshape(()).to(grad_MT.dtype), None, None, None


class Equilibrium(torch.autograd.Function):
    """The library's equilibrium map (rho^k, u) -> public moments, with its
    transposed Jacobian as backward."""

    @staticmethod
    def forward(ctx, prim: torch.Tensor, sim):
        prim = prim.detach().contiguous()
        ctx.sim, ctx.prim = sim, prim
        return sim.equilibrium(prim)

    @staticmethod
    def backward(ctx, grad_M: torch.Tensor):
        g = ctx.sim.equilibrium_adjoint(ctx.prim, grad_M.to(ctx.prim.dtype).contiguous())
        return g, None


def rollout(sim, M0: torch.Tensor, tau: torch.Tensor, nsteps: int, K: int = 20) -> torch.Tensor:
    """M(T) with gradients to M0 and tau (see the module docstring)."""
    return StateRollout.apply(M0, tau, sim, nsteps, K)


def equilibrium_moments(sim, rho: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Public moments with zero non-equilibrium part from (rho, u) (one
    species), computed by the library and differentiable through it."""
    return Equilibrium.apply(_primitive(sim, rho, u), sim)


def equilibrium_moments2(sim, rho1: torch.Tensor, rho2: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Two-species public moments (rho1, rho2, j, P) with zero
    non-equilibrium part from the species densities and a shared velocity,
    computed by the library and differentiable through it."""
    return Equilibrium.apply(_primitive(sim, torch.stack([rho1, rho2]), u), sim)
