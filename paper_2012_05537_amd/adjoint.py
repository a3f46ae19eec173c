"""Gradients of a rollout of the SLLBM through its hand-written adjoint.

The rollout maps perturbation amplitudes a (of velocity modes added to a base
flow) and the viscosity mu_inf to a flow functional of the final state:

    u0 = u_base + sum_m a_m B_m,    X_0 = equilibrium(rho0, u0, T0),
    X_{k+1} = S(C(X_k)),  k < n,    L = loss(X_n)

(C: collision, Eq. (5) with App. D; S: semi-Lagrangian streaming, Eq. (9);
loss: sllbm_loss).  The backward pass runs the reverse steps of the library
(sllbm_adjoint_step) from lambda_n = dL/dX_n down to lambda_0, then the VJP of
the equilibrium initialisation, and projects dL/du0 on the mode fields.

Memory: the forward pass keeps one pre-collision state every ``checkpoint``
steps; the backward pass replays each segment from its checkpoint (one
sllbm_step_record call) and walks it backwards.  ``checkpoint="sqrt"`` uses
ceil(sqrt(n)) steps per segment, so about 2 sqrt(n) states are resident.

Every step of the path runs in the library's kernels, the mode
superposition and the final projection on the modes included
(sllbm_superpose, sllbm_project); this module only allocates buffers, orders
the calls and scales the 17 host results by the upstream gradient.
"""
import math

import torch

from .sllbm import SLLBM


def segment_bounds(n_steps, checkpoint):
    """Segment starts and ends [(s0, s1), ...] covering 0..n_steps."""
    if n_steps < 0:
        raise ValueError("n_steps must be >= 0")
    if checkpoint == "sqrt":
        k = max(1, math.ceil(math.sqrt(n_steps)))
    else:
        k = int(checkpoint)
        if k < 1:
            raise ValueError("checkpoint interval must be >= 1")
    return [(s, min(s + k, n_steps)) for s in range(0, n_steps, k)]


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, amps, mu_inf, roll):
        sim = roll.sim
        sim.set_viscosity(float(mu_inf))
        u0 = roll.u0(amps)
        sim.init_equilibrium(roll.rho0, u0, roll.T0)
        checkpoints = []
        for s0, s1 in roll.segments:
            checkpoints.append(sim.get_state())
            sim.step(s1 - s0)
        final = sim.get_state()
        loss = sim.loss(final)
        fctx.roll = roll
        fctx.checkpoints = checkpoints
        fctx.final = final
        fctx.u0 = u0
        fctx.mu_inf = float(mu_inf)
        fctx.amps_device = amps.device
        fctx.mu_device = mu_inf.device
        return torch.tensor(loss, dtype=torch.float64, device=amps.device)

    @staticmethod
    def backward(fctx, grad):
        roll = fctx.roll
        sim = roll.sim
        sim.set_viscosity(fctx.mu_inf)
        lam = sim.loss_grad(fctx.final)        # the gradient is linear in lam: scaled by grad at the end
        other = torch.empty_like(lam)
        dmu = torch.zeros(1, dtype=torch.float64, device=lam.device)
        seg_max = max((s1 - s0 for s0, s1 in roll.segments), default=1)
        record = torch.empty((max(seg_max - 1, 1),) + tuple(lam.shape), dtype=lam.dtype, device=lam.device)
        for (s0, s1), ck in zip(reversed(roll.segments), reversed(fctx.checkpoints)):
            # states X_{s0} .. X_{s1-1}: the checkpoint, then s1-s0-1 recorded steps
            sim.set_state(ck)
            if s1 - s0 > 1:
                sim.step_record(s1 - s0 - 1, record)
            for n in range(s1 - 1, s0 - 1, -1):
                x_n = ck if n == s0 else record[n - s0 - 1]
                sim.adjoint_step(x_n, lam, other, dmu)
                lam, other = other, lam
        _, du, _ = sim.init_equilibrium_vjp(roll.rho0, fctx.u0, roll.T0, lam)
        g = float(grad)
        damps = torch.tensor([g * x for x in sim.project(roll.basis, du)], dtype=torch.float64,
                             device=fctx.amps_device)
        dmu_v = torch.tensor(g * float(dmu[0]), dtype=torch.float64, device=fctx.mu_device)
        return damps, dmu_v, None


class Rollout:
    """n-step rollout of a context from a perturbed base flow, differentiable
    in the mode amplitudes and mu_inf.

    sim      : an SLLBM context (its viscosity is set from mu_inf at each call)
    rho0, T0 : base density and temperature (N,), float64
    u_base   : base velocity (3, N), float64
    basis    : mode velocity fields (M, 3, N), float64
    """

    def __init__(self, sim: SLLBM, rho0, u_base, T0, basis, n_steps, checkpoint=10):
        dev = sim.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.sim = sim
        self.rho0 = torch.as_tensor(rho0).to(**f64).contiguous()
        self.u_base = torch.as_tensor(u_base).to(**f64).contiguous()
        self.T0 = torch.as_tensor(T0).to(**f64).contiguous()
        self.basis = torch.as_tensor(basis).to(**f64).contiguous()
        self.n_steps = int(n_steps)
        self.segments = segment_bounds(self.n_steps, checkpoint)

    def u0(self, amps):
        """u_base + sum_m amps[m] basis[m] (sllbm_superpose)."""
        return self.sim.superpose(self.u_base, self.basis, amps.detach().cpu().tolist())

    def __call__(self, amps, mu_inf):
        mu = mu_inf if torch.is_tensor(mu_inf) else torch.tensor(float(mu_inf), dtype=torch.float64)
        return _RolloutFn.apply(amps, mu, self)


SLLBMRollout = _RolloutFn
