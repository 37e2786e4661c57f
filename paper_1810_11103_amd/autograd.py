"""Differentiable time integration: a torch.autograd.Function over N TVD-RK3
steps of the WENOIU residual at a fixed time step, with the hand-written
adjoint of libwenoiu (wiu_rk3_step_vjp) and checkpointing.

Forward keeps the state every `every` steps (checkpoints).  Backward walks
the segments in reverse: it restores the segment's checkpoint, recomputes
the segment forward while storing the two RK stage states of every step
(wiu_rk3_step_stages), then applies the step adjoints in reverse order.
Memory: N/every checkpoints plus 3 x every states for one segment.
Metrics and the time step are held fixed (no gradient flows to them).
"""
import torch

from . import wenoiu


class RK3Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, every):
        U = U0.detach().clone().contiguous()
        solver.dt.fill_(float(dt))
        ckpts = []
        for s in range(nsteps):
            if s % every == 0:
                ckpts.append(U.clone())
            solver.rk3_step(U)
        ctx.solver, ctx.nsteps, ctx.dt, ctx.every = solver, nsteps, float(dt), every
        ctx.ckpts = ckpts
        return U

    @staticmethod
    def backward(ctx, gU):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.every
        solver.dt.fill_(ctx.dt)
        Ub = gU.detach().clone().contiguous()
        nseg = len(ctx.ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * every
            s1 = min(nsteps, s0 + every)
            U = ctx.ckpts[seg].clone()
            stages = []
            for _ in range(s0, s1):
                Un = U.clone()
                U1, U2 = torch.empty_like(U), torch.empty_like(U)
                solver.rk3_step_stages(U, U1, U2)
                stages.append((Un, U1, U2))
            for Un, U1, U2 in reversed(stages):
                solver.rk3_step_vjp(Un, Ub, U1, U2, out=Ub)
            del stages
        ctx.ckpts = None
        return Ub, None, None, None, None


def rollout(U0, solver, nsteps, dt, every=20):
    """U(T) after `nsteps` RK3 steps of size dt from U0, differentiable in U0."""
    return RK3Rollout.apply(U0, solver, int(nsteps), float(dt), int(every))


# ---------------------------------------------------------------------------
# Differentiable initial state of the isentropic vortex (Sec. 6.3(1)) in torch,
# so that gradients reach the vortex strength.  Same formulas as
# workloads.vortex_state.
# ---------------------------------------------------------------------------
def vortex_state_torch(x, y, strength, center=(5.0, 5.0), alpha=0.5, rc=1.0, mach=0.5, angle=None,
                       gamma=1.4, period=(10.0, 10.0)):
    import math
    angle = math.pi / 4 if angle is None else angle
    c = math.sqrt(gamma)
    u0 = mach * c * math.cos(angle)
    v0 = mach * c * math.sin(angle)
    dx = x - center[0]
    dy = y - center[1]
    if period[0]:
        dx = dx - period[0] * torch.round(dx / period[0])
    if period[1]:
        dy = dy - period[1] * torch.round(dy / period[1])
    dx, dy = dx / rc, dy / rc
    r2 = dx * dx + dy * dy
    f = strength * torch.exp(alpha * (1.0 - r2))
    u = u0 + f * dy
    v = v0 - f * dx
    T = 1.0 - (gamma - 1.0) * strength ** 2 / (4.0 * alpha * gamma) * torch.exp(2.0 * alpha * (1.0 - r2))
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return torch.stack([rho, rho * u, rho * v, e]).contiguous()


def density_objective(U, rho_inf=1.0):
    """J = sqrt(sum_ij (rho_ij - rho_inf)^2): plain node sum, no area weights."""
    return torch.sqrt(((U[0] - rho_inf) ** 2).sum())
