"""Differentiable MPC layers.

LTIMPC: forward the HIP ADMM solve of every instance; backward the HIP
implicit-differentiation adjoint (Algorithm 2).  The only work done here is
the chain rule from the QP-data gradients the library returns to the layer's
parameters (D_t = diag(Q, R) for t < N, diag(Q_f, R) at t = N; bounds shared
by all stages; x_init = x0), as index sums over stages.

BicycleMPC: forward the HIP SQP solve (Algorithm 1), keeping only the final
SQP iterate (x, xi, y_f, y_g) as the checkpoint.  Backward restores it into
the handle (ocp_set_iterate; the problem data first if the handle has been
given another problem since) and differentiates the SQP solution: the KKT
conditions of the OCP at that iterate with the exact Hessian of the
Lagrangian (ocp_adjoint with OCP_ADJ_SQP_EXACT), the factorisation redone
there.  The chain rule to the parameters (x0 [B,4], the reference ref [S,4],
the weight diagonals Qd, Rd, Qfd shared by the batch) follows the explicit
dependence of the stationarity residual on them: dL/dQ_jj = -sum eta_x,j
(x_j - r_j) over t < N, dL/dQf_jj the same at t = N, dL/dR_jj = -sum eta_u,j
u_j, dL/dr_t = W_t eta_x,t plus eta_g of an active lateral-offset row times
the track normal, dL/dx0 = the initial-state rows' gradient.
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


class BicycleMPC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, settings, batch, x0, ref, Qd, Rd, Qfd):
        data = tuple(t.detach().to(torch.float64) for t in (x0, ref, Qd, Rd, Qfd))
        solver.set_bicycle(batch, x0=data[0], ref=data[1], Qd=data[2].tolist(), Rd=data[3].tolist(),
                           Qfd=data[4].tolist())
        out = solver.solve(settings)
        ctx.solver, ctx.settings, ctx.batch = solver, settings, batch
        ctx.generation = solver.generation
        ctx.save_for_backward(out["x"], out["xi"], out["y_f"], out["y_g"], *data)
        ctx.mark_non_differentiable(out["status"])
        return out["x"].clone(), out["status"]

    @staticmethod
    def backward(ctx, dx, _dstatus):
        s = ctx.solver
        x, xi, y_f, y_g, x0, ref, Qd, Rd, Qfd = ctx.saved_tensors
        if s.generation != ctx.generation:
            s.set_bicycle(ctx.batch, x0=x0, ref=ref, Qd=Qd.tolist(), Rd=Rd.tolist(), Qfd=Qfd.tolist())
        s.set_iterate(x, xi, y_f, y_g)
        st = A.ocp_settings.from_buffer_copy(ctx.settings)
        st.adj_mode = A.ADJ_SQP_EXACT
        g = s.adjoint(dx.contiguous().to(torch.float64), st)
        dev = x.device
        last = torch.zeros(s.S, dtype=torch.bool, device=dev)
        last[torch.as_tensor(s.stage_off[1:] - 1, device=dev, dtype=torch.long)] = True
        ex = g["eta_x"]
        e = x[:, :4] - ref
        dQd = -(ex[~last, :4] * e[~last]).sum(dim=0)
        dQfd = -(ex[last, :4] * e[last]).sum(dim=0)
        dRd = -(ex[:, 4:] * x[:, 4:]).sum(dim=0)
        W = torch.where(last[:, None], Qfd[None, :], Qd[None, :])
        normal = torch.as_tensor(ctx.batch.normal, dtype=torch.float64, device=dev)
        dref = W * ex[:, :4]
        dref[:, :2] += g["eta_g"][:, 2:3] * normal
        return None, None, None, g["d_x_init"], dref, dQd, dRd, dQfd


def bicycle_mpc(solver, batch, x0, ref, Qd, Rd, Qfd, settings=None):
    """SQP solve of a batch of kinematic-bicycle OCPs (the track geometry and
    bounds from `batch`); returns (x [S, 6], status [B]).  Differentiable
    w.r.t. x0 [B,4], ref [S,4] and the weight diagonals Qd [4], Rd [2], Qfd [4]:
    the derivative of the SQP solution, from its checkpointed iterate."""
    settings = settings if settings is not None else A.default_settings()
    return BicycleMPC.apply(solver, settings, batch, x0, ref, Qd, Rd, Qfd)
