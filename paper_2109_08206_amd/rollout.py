"""Differentiable multi-step rollout of the steric step.

``Rollout`` is a ``torch.autograd.Function`` over the C-ABI.
  * Forward: T calls of ``rl_step`` (the linearised Euler step of
    eq. constrainedeom_euler, one complementarity solve per step).  It keeps
    (x, theta) every ``checkpoint_every`` steps.  With ``tape=True`` it also
    keeps every step's constraint forces gamma (8 bytes per constraint;
    about 3 MB per step at 50,000 rods).
  * Backward: walks the segments in reverse.  For each one it recomputes the
    segment's states from its checkpoint with ``rl_step``, then calls
    ``rl_step_adjoint`` step by step in reverse.  A replayed tape starts each
    of those solves at its own solution, so they stop at once.  The results
    are bitwise those of cold solves: every sum runs in a fixed order, and
    the recomputed states equal the forward ones.
The output is the unwrapped centres x0 + h sum_t U_t (plus theta_T), which
``rl_step`` advances beside the wrapped ones.
Wrapping into the periodic box shifts by whole box lengths and does not
change the derivative.  Marshalling only: every step runs in the HIP
kernels.
"""
from __future__ import annotations

import torch

from . import NOT_CONVERGED, STAGNATED, TAPE_REPLAY, RodLCPError


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, quat0, F, solver, length, checkpoint_every, cg_tol, tape):
        T, n = F.shape[0], x0.shape[0]
        k = max(1, int(checkpoint_every))
        x = x0.detach().clone()
        quat = quat0.detach().clone()
        xu = x0.detach().clone()
        U = torch.empty((n, 6), dtype=torch.float64, device=x0.device)
        ckpt, tapes, infos = [], [], []
        cap = 16 * n + 64
        for t in range(T):
            if t % k == 0:
                ckpt.append((x.clone(), quat.clone()))
            if tape:
                _, info, g = solver.step_recording(x, quat, length, F[t], U=U, capacity=cap, x_unwrapped=xu)
                tapes.append(g)
                npairs = g.shape[0]
                cap = npairs + npairs // 4 + 1024
            else:
                _, info, npairs = solver.step(x, quat, length, F[t], U=U, x_unwrapped=xu)
            if info.status in (NOT_CONVERGED, STAGNATED):
                raise RodLCPError(info.status, "Rollout.forward", f"step {t} did not converge")
            infos.append((info.iterations, npairs))
        ctx.solver, ctx.length, ctx.k, ctx.cg_tol = solver, length, k, cg_tol
        ctx.ckpt, ctx.tapes, ctx.infos = ckpt, tapes, infos
        ctx.save_for_backward(F)
        return xu, quat

    @staticmethod
    def backward(ctx, xu_bar, quat_bar):
        (F,) = ctx.saved_tensors
        solver, length, k, tapes = ctx.solver, ctx.length, ctx.k, ctx.tapes
        T, n = F.shape[0], F.shape[1]
        zx = torch.zeros((n, 3), dtype=torch.float64, device=F.device)
        zq = torch.zeros((n, 4), dtype=torch.float64, device=F.device)
        x_bar = (xu_bar if xu_bar is not None else zx).detach().clone().contiguous()
        q_bar = (quat_bar if quat_bar is not None else zq).detach().clone().contiguous()
        F_bar = torch.empty_like(F)
        adj = []
        for seg in reversed(range(len(ctx.ckpt))):
            t0 = seg * k
            t1 = min(T, t0 + k)
            x, quat = (v.clone() for v in ctx.ckpt[seg])
            states = []
            for t in range(t0, t1):
                states.append((x.clone(), quat.clone()))
                if t < t1 - 1:
                    if tapes:
                        solver.step(x, quat, length, F[t], tape=tapes[t], tape_mode=TAPE_REPLAY)
                    else:
                        solver.step(x, quat, length, F[t])
            for t in reversed(range(t0, t1)):
                xs, qs = states[t - t0]
                _, info = solver.step_adjoint(xs, qs, length, F[t], x_bar, q_bar, F_bar=F_bar[t],
                                              cg_tol=ctx.cg_tol, tape=tapes[t] if tapes else None)
                adj.append(info)
        ctx.adjoint_infos = adj
        return x_bar, q_bar, F_bar, None, None, None, None, None


def rollout(solver, x0, quat0, length, F, checkpoint_every: int = 10, cg_tol: float = 0.0, tape: bool = True):
    """Unwrapped final centres and final quaternions after F.shape[0] steps;
    differentiable with respect to x0, quat0 (on the unit sphere) and F."""
    return Rollout.apply(x0, quat0, F, solver, length, checkpoint_every, cg_tol, tape)
