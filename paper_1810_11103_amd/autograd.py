"""Differentiable time integration: a torch.autograd.Function over N TVD-RK3
steps of the WENOIU residual at a fixed time step, with the hand-written
adjoint of libwenoiu (wiu_rk3_step_vjp).

Two ways to have the stage states at hand in the backward pass:
  every = 0   forward stores (U_n, U1, U2) of every step (3 N states, no
              recomputation) -- the choice whenever it fits in device memory;
  every = k   forward keeps U_n every k steps (checkpoints); backward walks
              the segments in reverse, recomputes each segment forward with
              its stage states (wiu_rk3_step_stages), then applies the step
              adjoints in reverse order (N/k checkpoints + 3 k states).  The
              last segment's stage states are the forward pass's own (kept
              as it runs them), so the backward pass starts with adjoints
              while the next segment is recomputed beside it.
The stage-storing steps of a segment (or of the whole rollout) run as one
library call (wiu_rk3_steps_stages), whose steps after the first take their
line maxima from the step before.
rollout(every="auto") stores everything when 3 N states fit in the given
fraction of free device memory, else checkpoints every ~sqrt(N/3) steps,
which minimises N/k + 3k.  Metrics and the time step are held fixed (no
gradient flows to them).
"""
import math

import torch

from . import wenoiu


class RK3Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps, dt, every):
        U = U0.detach().clone().contiguous()
        solver.dt.fill_(float(dt))
        ckpts, stages, recs = [], None, None
        if nsteps <= 0:
            every = 0
        if every == 0:  # one allocation for all (U_n, U1, U2), and their step records
            stages = torch.empty((max(nsteps, 0), 3) + tuple(U.shape), dtype=U.dtype, device=U.device)
            recs = solver.step_record(max(nsteps, 0))
        else:  # the last segment's stages and step records
            first_last = (nsteps - 1) // every * every
            stages = torch.empty((nsteps - first_last, 3) + tuple(U.shape), dtype=U.dtype, device=U.device)
            recs = solver.step_record(nsteps - first_last)
        if every == 0:
            if nsteps > 0:
                solver.rk3_steps_stages(U, stages, recs)  # all steps in one call
        else:
            for s in range(first_last):
                if s % every == 0:
                    ckpts.append(U.clone())
                solver.rk3_step(U)
            ckpts.append(U.clone())  # the last segment's start, kept with its stages
            solver.rk3_steps_stages(U, stages, recs)
        ctx.solver, ctx.nsteps, ctx.dt, ctx.every = solver, nsteps, float(dt), every
        ctx.ckpts, ctx.stages, ctx.recs = ckpts, stages, recs
        return U

    @staticmethod
    def backward(ctx, gU):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.every
        solver.dt.fill_(ctx.dt)
        Ub = gU.detach().clone().contiguous()
        if every == 0:
            for s in reversed(range(nsteps)):
                st = ctx.stages[s]
                solver.rk3_step_vjp(st[0], Ub, st[1], st[2], out=Ub, rec=ctx.recs[s])
        else:
            _checkpointed_backward(ctx, Ub)
        ctx.ckpts = ctx.stages = ctx.recs = None
        return Ub, None, None, None, None


def _checkpointed_backward(ctx, Ub):
    """Segments in reverse order: the last one from the stages the forward
    pass kept; for the others, the forward recomputation of segment k-1 runs
    on a second stream (its own workspace, one of two stage buffers) while
    the step adjoints of segment k run on the caller's stream."""
    solver, nsteps, every, ckpts = ctx.solver, ctx.nsteps, ctx.every, ctx.ckpts
    nseg = len(ckpts)
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream(device=Ub.device)  # default priority
    ws2 = solver.side_workspace()
    bufs = torch.empty((2, every, 3) + tuple(Ub.shape), dtype=Ub.dtype, device=Ub.device)
    recs = solver.step_record(2 * every).view(2, every, -1)
    work = torch.empty((2,) + tuple(Ub.shape), dtype=Ub.dtype, device=Ub.device)
    ready = [torch.cuda.Event() for _ in range(nseg)]
    freed = [torch.cuda.Event() for _ in range(nseg)]
    side.wait_stream(main)  # dt, checkpoints and buffers are ready

    def recompute(seg):
        with torch.cuda.stream(side):
            if seg + 2 < nseg:
                side.wait_event(freed[seg + 2])  # its buffer set was last used by segment seg+2
            B, U = bufs[seg % 2], work[seg % 2]
            U.copy_(ckpts[seg])
            n = min(nsteps, (seg + 1) * every) - seg * every
            solver.rk3_steps_stages(U, B[:n], recs[seg % 2, :n], ws=ws2)
            ready[seg].record(side)

    for seg in reversed(range(nseg)):
        if seg > 0:
            recompute(seg - 1)
        if seg == nseg - 1:
            B, R = ctx.stages, ctx.recs
        else:
            main.wait_event(ready[seg])
            B, R = bufs[seg % 2], recs[seg % 2]
        for i in reversed(range(min(nsteps, (seg + 1) * every) - seg * every)):
            solver.rk3_step_vjp(B[i, 0], Ub, B[i, 1], B[i, 2], out=Ub, rec=R[i])
        freed[seg].record(main)
    main.wait_stream(side)
    bufs.record_stream(side)
    work.record_stream(side)
    recs.record_stream(side)


def choose_every(nsteps, state_bytes, memory_fraction=0.5, free_bytes=None):
    """0 (store every stage) if 3 nsteps states fit in memory_fraction of the
    free device memory, else the checkpoint spacing round(sqrt(nsteps/3))."""
    if free_bytes is None:
        free_bytes = torch.cuda.mem_get_info()[0]
    if 3 * nsteps * state_bytes <= memory_fraction * free_bytes:
        return 0
    return max(1, int(round(math.sqrt(nsteps / 3.0))))


def rollout(U0, solver, nsteps, dt, every="auto", memory_fraction=0.5):
    """U(T) after `nsteps` RK3 steps of size dt from U0, differentiable in U0."""
    if every == "auto":
        every = choose_every(int(nsteps), U0.numel() * U0.element_size(), memory_fraction)
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
