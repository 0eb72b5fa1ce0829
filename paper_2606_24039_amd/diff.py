"""Differentiable batched LTI MPC layer.

forward: the HIP ADMM solve of every instance; backward: the HIP
implicit-differentiation adjoint (Algorithm 2).  The only work done here is
the chain rule from the QP-data gradients the library returns to the layer's
parameters (D_t = diag(Q, R) for t < N, diag(Q_f, R) at t = N; bounds shared
by all stages; x_init = x0), as index sums over stages.
"""
from __future__ import annotations

import torch

from . import _abi as A


class LTIMPC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, settings, Amat, Bm, G, Qd, Rd, Qfd, lo, hi, x0):
        data = tuple(t.detach() for t in (Amat, Bm, Qd, Rd, Qfd, G, lo, hi, x0))
        solver.set_lti(*data)
        out = solver.solve(settings)
        ctx.solver = solver
        ctx.settings = settings
        ctx.generation = solver.generation  # the handle's state this backward differentiates
        ctx.save_for_backward(out["x"], *data)
        ctx.mark_non_differentiable(out["status"])
        return out["x"].clone(), out["status"]

    @staticmethod
    def backward(ctx, dx, _dstatus):
        s = ctx.solver
        x, *data = ctx.saved_tensors
        if s.generation != ctx.generation:
            # the handle was reused for another problem since this forward: restore
            # this forward's data and solve again (the solve is deterministic, so
            # the handle holds the same solution the forward returned)
            s.set_lti(*data)
            s.solve(ctx.settings)
        g = s.adjoint(dx.contiguous().to(torch.float64), ctx.settings)
        dev = x.device
        inst = torch.repeat_interleave(torch.arange(s.B, device=dev),
                                       torch.as_tensor(s.horizons + 1, device=dev, dtype=torch.long))
        last = torch.as_tensor(s.stage_off[1:] - 1, device=dev, dtype=torch.long)
        is_last = torch.zeros(s.S, dtype=torch.bool, device=dev)
        is_last[last] = True
        dD = g["d_Ddiag"]
        nx = s.nx
        dQ = torch.zeros(s.B, nx, dtype=torch.float64, device=dev).index_add_(
            0, inst[~is_last], dD[~is_last, :nx])
        dQf = dD[last, :nx].clone()
        dR = torch.zeros(s.B, s.nu, dtype=torch.float64, device=dev).index_add_(0, inst, dD[:, nx:])
        dlo = torch.zeros(s.B, s.ng, dtype=torch.float64, device=dev).index_add_(0, inst, g["d_lo"])
        dhi = torch.zeros(s.B, s.ng, dtype=torch.float64, device=dev).index_add_(0, inst, g["d_hi"])
        return None, None, None, None, None, dQ, dR, dQf, dlo, dhi, g["d_x_init"]


def lti_mpc(solver, Amat, Bm, G, Qd, Rd, Qfd, lo, hi, x0, settings=None):
    """Solve a batch of LTI MPC problems; returns (x [S, n], status [B]).
    Differentiable w.r.t. Qd, Rd, Qfd, lo, hi, x0."""
    settings = settings if settings is not None else A.default_settings()
    return LTIMPC.apply(solver, settings, Amat, Bm, G, Qd, Rd, Qfd, lo, hi, x0)
