"""Differentiable SSP-RK3 trajectories on top of the library's step adjoint.

`rk3_trajectory(U0, grid, scheme, nsteps, checkpoint_every)` advances U0 by
`nsteps` SSP-RK3 steps with `tenoaa_step` and returns the final state as a
tensor that autograd can differentiate with respect to U0.  Each step's dt is
computed on the device in the forward pass and then frozen; the threshold
decisions are frozen at the states the forward pass visited.  Only every
`checkpoint_every`-th state is kept: the backward pass recomputes each
segment from its checkpoint (bitwise the same states, since the kernels are
deterministic and dt is replayed) and chains `tenoaa_step_vjp` backwards
through it.  With `tape=True` the recomputation keeps each step's tape
(`tenoaa_step_tape`: the stage states and every stage's decisions and
fluxes, one workspace per step of the segment) and the reverse pass runs
`tenoaa_step_vjp_tape`, which skips the stage recomputation inside each
step's adjoint; the gradient is the same bit for bit.
"""
import torch

from . import tenoaa


class _RK3Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, grid, scheme, gamma, cfl, nsteps, every, tape):
        if nsteps < 1 or every < 1:
            raise ValueError("nsteps and checkpoint_every must be positive")
        U = U0.detach().clone()
        ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, U.device)
        dts = torch.zeros(nsteps, dtype=torch.float64, device=U.device)
        ckpts = [U.clone()]
        for n in range(nsteps):
            tenoaa.step(grid, scheme, U, dts[n:n + 1], gamma=gamma, cfl=cfl, ws=ws)
            if (n + 1) % every == 0 and n + 1 < nsteps:
                ckpts.append(U.clone())
        ctx.grid, ctx.scheme, ctx.gamma, ctx.cfl = grid, scheme, gamma, cfl
        ctx.nsteps, ctx.every, ctx.tape = nsteps, every, tape
        ctx.save_for_backward(dts, *ckpts)
        return U

    @staticmethod
    def backward(ctx, gU):
        dts, *ckpts = ctx.saved_tensors
        grid, scheme, gamma = ctx.grid, ctx.scheme, ctx.gamma
        ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, gU.device)
        ws_vjp = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP_VJP, gU.device)
        bar = gU.detach().contiguous().clone()
        nxt = torch.empty_like(bar)
        nseg = len(ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * ctx.every
            s1 = min(s0 + ctx.every, ctx.nsteps)
            states = [ckpts[seg]]
            if ctx.tape:
                tapes = []
                for n in range(s0, s1):
                    U, wt = tenoaa.step_tape(grid, scheme, states[-1], dts[n:n + 1], gamma=gamma, cfl=ctx.cfl)
                    tapes.append(wt)
                    if n + 1 < s1:
                        states.append(U)
                for n in reversed(range(s0, s1)):
                    tenoaa.step_vjp_tape(grid, scheme, states[n - s0], dts[n:n + 1], bar, tapes[n - s0],
                                         gamma=gamma, out=nxt)
                    bar, nxt = nxt, bar
                    tapes[n - s0] = None
                continue
            U = ckpts[seg].clone()
            for n in range(s0, s1 - 1):
                tenoaa.step(grid, scheme, U, dts[n:n + 1], gamma=gamma, cfl=ctx.cfl, ws=ws)
                states.append(U.clone())
            for n in reversed(range(s0, s1)):
                tenoaa.step_vjp(grid, scheme, states[n - s0], dts[n:n + 1], bar, gamma=gamma, out=nxt, ws=ws_vjp)
                bar, nxt = nxt, bar
        return bar, None, None, None, None, None, None, None


def rk3_trajectory(U0, grid, scheme, nsteps, checkpoint_every=10, gamma=1.4, cfl=0.4, tape=False):
    """Final state after nsteps SSP-RK3 steps; differentiable w.r.t. U0.
    tape: keep each recomputed step's tape in the backward pass (one
    WS_STEP_TAPE workspace per step of a segment) instead of recomputing the
    stages inside every step's adjoint."""
    return _RK3Trajectory.apply(U0, grid, scheme, gamma, cfl, nsteps, checkpoint_every, tape)


def record_trajectory(U0, grid, scheme, nsteps, gamma=1.4, cfl=0.4):
    """Forward run that records each step's dt and the decisions of every stage:
    returns (U_final, dts, flags) with flags of shape (nsteps, 3 * flags_size)."""
    U = U0.detach().clone()
    ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, U.device)
    nfl = tenoaa.flags_size(grid)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=U.device)
    flags = torch.zeros((nsteps, 3 * nfl), dtype=torch.uint8, device=U.device)
    for n in range(nsteps):
        tenoaa.step_flags(grid, scheme, U, dts[n:n + 1], flags[n], tenoaa.FLAGS_RECORD, gamma=gamma, cfl=cfl, ws=ws)
    return U, dts, flags


def replay_trajectory(U0, grid, scheme, dts, flags, gamma=1.4):
    """Forward run with every dt and decision replayed from record_trajectory."""
    U = U0.detach().clone()
    ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, U.device)
    for n in range(dts.numel()):
        tenoaa.step_flags(grid, scheme, U, dts[n:n + 1], flags[n], tenoaa.FLAGS_REPLAY, gamma=gamma, ws=ws)
    return U


def record_trajectory_near(U0, grid, scheme, nsteps, tol=1e-3, gamma=1.4, cfl=0.4):
    """Forward run recording each step's dt, the decisions of every stage and
    which of them lie within `tol` (relative) of a threshold: returns
    (U_final, dts, flags, near), flags and near of shape (nsteps, 3 * flags_size)."""
    U = U0.detach().clone()
    ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, U.device)
    nfl = tenoaa.flags_size(grid)
    dts = torch.zeros(nsteps, dtype=torch.float64, device=U.device)
    flags = torch.zeros((nsteps, 3 * nfl), dtype=torch.uint8, device=U.device)
    near = torch.zeros((nsteps, 3 * nfl), dtype=torch.uint8, device=U.device)
    for n in range(nsteps):
        tenoaa.step_near(grid, scheme, U, dts[n:n + 1], flags_out3=flags[n], near_out3=near[n], tol=tol,
                         gamma=gamma, cfl=cfl, ws=ws)
    return U, dts, flags, near


def near_replay_trajectory(U0, grid, scheme, dts, flags, near, tol=1e-3, gamma=1.4):
    """Forward run with the recorded dt of every step, the decisions that
    `near` marks replayed from `flags` and every other decision taken live:
    returns (U_final, flags_used)."""
    U = U0.detach().clone()
    ws = tenoaa.workspace(grid, scheme, tenoaa.WS_STEP, U.device)
    used = torch.empty_like(flags)
    for n in range(dts.numel()):
        tenoaa.step_near(grid, scheme, U, dts[n:n + 1], base3=flags[n], near_in3=near[n], flags_out3=used[n],
                         tol=tol, gamma=gamma, ws=ws)
    return U, used
