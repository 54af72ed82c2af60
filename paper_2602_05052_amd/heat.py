"""Differentiable implicit-Euler heat rollout as one autograd node.

The method-of-lines system M U' + K(a) U = 0 (SM A.1) is stepped with implicit
Euler, (M + dt K(a)) u^{k+1} = M u^k, with u = 0 on the pattern's constrained
vertices.  Forward and backward each run entirely in libtg: the forward is
tg_heat_rollout (Map-Reduce assembly of M and M + dt K once, then per step an
SpMV and a Jacobi-PCG solve); the backward is tg_heat_adjoint (the discrete
adjoint recursion of Sec. 2 eq. adj, then one batched adjoint-assembly launch
for dL/dlog a and dL/dx and one SpMV for dL/du^0).  The whole rollout is a
single node of the autograd graph however many steps and PCG iterations it
takes, which keeps the graph O(1) in the way Sec. 2 asks of the assembly.

    import paper_2602_05052_amd as tg
    from paper_2602_05052_amd.heat import heat_solve
    pat = tg.Pattern(conn, n_vertices, dim=2)                 # Dirichlet on the boundary
    uN = heat_solve(pat, coords, log_a, u0, dt=1e-3, nsteps=20)
    loss = ((uN - target) ** 2).sum(); loss.backward()        # coords.grad, log_a.grad, u0.grad
"""
from __future__ import annotations

import torch

from . import Pattern, TGError, TG_E_DEGENERATE, check_status, heat_adjoint, heat_rollout, new_status


class HeatRollout(torch.autograd.Function):
    """u^N = rollout(coords, log_a, u0); backward by the hand-written adjoint."""

    @staticmethod
    def forward(ctx, coords, log_a, u0, pattern: Pattern, dt: float, nsteps: int, rtol: float, max_iter: int,
                check_every: int):
        coords = coords.detach().contiguous()
        log_a = log_a.detach().contiguous()
        u0 = u0.detach().contiguous()
        status = new_status(coords.device)
        states, iters, relres = heat_rollout(pattern, coords, log_a, u0, dt, nsteps, rtol, max_iter, check_every,
                                             status=status)
        bad = check_status(status)
        if bad is not None:
            raise TGError(TG_E_DEGENERATE, f"element {bad} is numerically singular or has a non-finite coefficient")
        ctx.save_for_backward(coords, log_a, states)
        ctx.pattern = pattern
        ctx.cfg = (dt, rtol, max_iter, check_every)
        ctx.stats = {"forward_iters": iters, "forward_relres": relres}
        return states[nsteps].clone()

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        coords, log_a, states = ctx.saved_tensors
        dt, rtol, max_iter, check_every = ctx.cfg
        need_x, need_a, need_u0 = (bool(x) for x in ctx.needs_input_grad[:3])
        if not (need_x or need_a or need_u0):
            return (None,) * 9
        g = g.detach().to(states.dtype).contiguous()
        dla, dx, du0, _, _ = heat_adjoint(ctx.pattern, coords, log_a, states, g, dt, rtol, max_iter, check_every,
                                          want=(need_a, need_x, need_u0))
        return dx, dla, du0, None, None, None, None, None, None


def heat_solve(pattern: Pattern, coords, log_a, u0, dt: float = 1e-3, nsteps: int = 20, rtol: float = 1e-10,
               max_iter: int = 10000, check_every: int = 10):
    """u^N of the implicit-Euler rollout, differentiable in coords [nv, d] (FP64), log_a [E] (FP64)
    and u0 [nv] (FP64 or FP32: the compute dtype of the matrices, vectors and PCG)."""
    return HeatRollout.apply(coords, log_a, u0, pattern, float(dt), int(nsteps), float(rtol), int(max_iter),
                             int(check_every))
