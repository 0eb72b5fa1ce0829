"""OCP functions (cost l, dynamics f, inequalities g) for the kinematic
bicycle, with analytic derivatives, and its convexification into a StageQP.

Continuous dynamics (state (px, py, yaw, v), control (a, delta), wheelbase L):
    px' = v cos(yaw),  py' = v sin(yaw),  yaw' = v tan(delta) / L,  v' = a.
Implicit midpoint with zero-order hold on u (not given by the paper, which
writes the trapezoidal rule in Remark A1; the midpoint rule has the same
block structure):
    f_t = x_t + dt * fc((x_t + x_{t+1}) / 2, u_t) - x_{t+1} = 0.
Jacobians:  A_t^- = [I + dt/2 Jx, dt Ju],  A_t^+ = [-I + dt/2 Jx, 0].
The trapezoidal rule of Remark A1 (batch.integrator = 1), same hold on u:
    f_t = x_t + dt/2 (fc(x_t, u_t) + fc(x_{t+1}, u_t)) - x_{t+1} = 0,
    A_t^- = [I + dt/2 Jx(x_t), dt/2 (Ju(x_t) + Ju(x_{t+1}))],
    A_t^+ = [-I + dt/2 Jx(x_{t+1}), 0].

Cost 1/2 (x_t - r_t)'Q(x_t - r_t) + 1/2 u_t'R u_t (t < N), with Q_f at t = N,
plus the control-rate cost of the racing problem (Sec. "Hardware
Deployment: Autonomous Racing", eq. cost), 1/2 (u_t - u_{t+1})'W(u_t -
u_{t+1}) for t < N (W diagonal, zero by default; the same 1/2 as the other
terms).  It couples neighbouring stages: D_t gets W once at t = 0 and t = N
and twice in between, and E_t (block (t+1, t)) gets -W on the control rows.
Inequalities g_t = (a_t, delta_t, n_t'(p_t - p_ref_t)): hard boxes on a and
delta, the lateral offset soft (L1) within +-lat_bound.  With u_init given,
the first control is fixed, (x_0, u_0) = (x_init, u_init) as in the racing
problem: the two control rows of stage 0 get lo = hi = u_init.

The QP is written in absolute coordinates (Appendix "QP Approximation" gives
c and the shifted bounds for the absolute variable), so the linear cost term
is q_t = grad l_t(xbar_t) - D_t xbar_t.

Parity: Jacobians pinned by central differences, midpoint residual by a
Newton-solved rollout, both rules by their order of accuracy on a circle
(tests/test_oracle_sqp.py).
"""
from __future__ import annotations

import numpy as np

from .qp import HARD, SOFT_L1, StageQP


def fc(x, u, L):
    px, py, yaw, v = x
    a, d = u
    return np.array([v * np.cos(yaw), v * np.sin(yaw), v * np.tan(d) / L, a])


def fc_jac(x, u, L):
    _, _, yaw, v = x
    _, d = u
    Jx = np.zeros((4, 4))
    Jx[0, 2] = -v * np.sin(yaw)
    Jx[0, 3] = np.cos(yaw)
    Jx[1, 2] = v * np.cos(yaw)
    Jx[1, 3] = np.sin(yaw)
    Jx[2, 3] = np.tan(d) / L
    Ju = np.zeros((4, 2))
    Ju[2, 1] = v / (L * np.cos(d) ** 2)
    Ju[3, 0] = 1.0
    return Jx, Ju


def midpoint_residual(xt, ut, xn, dt, L):
    """f_t(x_t, u_t, x_{t+1}) of the implicit midpoint rule."""
    return xt + dt * fc(0.5 * (xt + xn), ut, L) - xn


def midpoint_jacobians(xt, ut, xn, dt, L):
    """(A^- [4x6], A^+ [4x6]) of f_t w.r.t. (x_t,u_t) and (x_{t+1},u_{t+1})."""
    Jx, Ju = fc_jac(0.5 * (xt + xn), ut, L)
    I = np.eye(4)
    Am = np.hstack([I + 0.5 * dt * Jx, dt * Ju])
    Ap = np.hstack([-I + 0.5 * dt * Jx, np.zeros((4, 2))])
    return Am, Ap


def trapezoid_residual(xt, ut, xn, dt, L):
    """f_t(x_t, u_t, x_{t+1}) of the trapezoidal rule (zero-order hold on u)."""
    return xt + 0.5 * dt * (fc(xt, ut, L) + fc(xn, ut, L)) - xn


def trapezoid_jacobians(xt, ut, xn, dt, L):
    """(A^- [4x6], A^+ [4x6]) of the trapezoidal f_t."""
    Jx0, Ju0 = fc_jac(xt, ut, L)
    Jx1, Ju1 = fc_jac(xn, ut, L)
    I = np.eye(4)
    Am = np.hstack([I + 0.5 * dt * Jx0, 0.5 * dt * (Ju0 + Ju1)])
    Ap = np.hstack([-I + 0.5 * dt * Jx1, np.zeros((4, 2))])
    return Am, Ap


class BicycleOCP:
    """One instance of a workloads.BicycleBatch as an OCP."""

    def __init__(self, batch, i: int):
        sl = batch.stages(i)
        self.N = int(batch.horizons[i])
        self.ref = batch.ref[sl]
        self.normal = batch.normal[sl]
        self.x_init = batch.x0[i].copy()
        self.dt = batch.dt
        self.L = batch.wheelbase
        self.Q = np.diag(batch.Qd)
        self.R = np.diag(batch.Rd)
        self.Qf = np.diag(batch.Qfd)
        # per-stage bounds [(N+1), 3]; stage 0's control rows fixed at u_init
        lo = np.array([-batch.a_bound, -batch.steer_bound, -batch.lat_bound])
        self.g_lo = np.tile(lo, (self.N + 1, 1))
        self.g_hi = np.tile(-lo, (self.N + 1, 1))
        u_init = getattr(batch, "u_init", None)
        self.u_init = None if u_init is None else np.asarray(u_init, float)[i].copy()
        if self.u_init is not None:
            self.g_lo[0, :2] = self.u_init
            self.g_hi[0, :2] = self.u_init
        self.W = np.diag(np.asarray(getattr(batch, "Wd", np.zeros(2)), float))
        self.soft = np.array([HARD, HARD, SOFT_L1])
        self.gamma1 = batch.gamma_l1
        self.nx, self.nu, self.ng = 4, 2, 3
        trap = getattr(batch, "integrator", 0) == 1
        self._res = trapezoid_residual if trap else midpoint_residual
        self._jac = trapezoid_jacobians if trap else midpoint_jacobians

    @property
    def n(self):
        return 6

    def initial_guess(self):
        """The reference trajectory with zero controls (u_0 = u_init when fixed)."""
        z = np.zeros((self.N + 1, 6))
        z[:, :4] = self.ref
        if self.u_init is not None:
            z[0, 4:] = self.u_init
        return z

    # --- cost --------------------------------------------------------------
    def stage_weights(self, t):
        W = np.zeros((6, 6))
        W[:4, :4] = self.Qf if t == self.N else self.Q
        W[4:, 4:] = self.R
        return W

    def cost(self, z):
        tot = 0.0
        for t in range(self.N + 1):
            e = np.concatenate([z[t, :4] - self.ref[t], z[t, 4:]])
            tot += 0.5 * e @ self.stage_weights(t) @ e
        for t in range(self.N):
            du = z[t, 4:] - z[t + 1, 4:]
            tot += 0.5 * du @ self.W @ du
        return tot

    def cost_grad(self, z):
        g = np.zeros_like(z)
        for t in range(self.N + 1):
            e = np.concatenate([z[t, :4] - self.ref[t], z[t, 4:]])
            g[t] = self.stage_weights(t) @ e
        for t in range(self.N):
            wdu = self.W @ (z[t, 4:] - z[t + 1, 4:])
            g[t, 4:] += wdu
            g[t + 1, 4:] -= wdu
        return g

    def cost_hessian_blocks(self):
        """(D [(N+1),6,6], E [N,6,6]) of the cost's Hessian, E_t = block (t+1, t)."""
        N = self.N
        D = np.stack([self.stage_weights(t) for t in range(N + 1)])
        E = np.zeros((N, 6, 6))
        for t in range(N):
            D[t, 4:, 4:] += self.W
            D[t + 1, 4:, 4:] += self.W
            E[t, 4:, 4:] = -self.W
        return D, E

    # --- equality constraints (init + dynamics) -----------------------------
    def eq_residual(self, z):
        """(x_0 - x_init, f_0, ..., f_{N-1}) stacked."""
        r = [z[0, :4] - self.x_init]
        for t in range(self.N):
            r.append(self._res(z[t, :4], z[t, 4:], z[t + 1, :4], self.dt, self.L))
        return np.concatenate(r)

    def eq_jac_T_times(self, z, y):
        """grad_x (y' f(x)) for y = (y_init, y_dyn...)."""
        out = np.zeros_like(z)
        out[0, :4] += y[:4]
        for t in range(self.N):
            yt = y[4 + 4 * t: 8 + 4 * t]
            Am, Ap = self._jac(z[t, :4], z[t, 4:], z[t + 1, :4], self.dt, self.L)
            out[t] += Am.T @ yt
            out[t + 1] += Ap.T @ yt
        return out

    # --- inequalities -------------------------------------------------------
    def G_block(self, t):
        Gt = np.zeros((3, 6))
        Gt[0, 4] = 1.0
        Gt[1, 5] = 1.0
        Gt[2, 0:2] = self.normal[t]
        return Gt

    def g_const(self, t):
        """g_t(x) = G_t x + g_const_t."""
        return np.array([0.0, 0.0, -self.normal[t] @ self.ref[t, :2]])

    def ineq(self, z):
        return np.stack([self.G_block(t) @ z[t] + self.g_const(t) for t in range(self.N + 1)])

    # --- convexification --------------------------------------------------
    def convexify(self, z) -> StageQP:
        """QP approximation at the trajectory z [(N+1), 6] (Appendix "QP Approximation")."""
        N = self.N
        D, E = self.cost_hessian_blocks()
        grad = self.cost_grad(z)
        # q_t = grad_t - (H z)_t with (H z)_t = D_t z_t + E_{t-1} z_{t-1} + E_t' z_{t+1}
        q = np.stack([grad[t] - D[t] @ z[t] for t in range(N + 1)])
        for t in range(N):
            q[t + 1] -= E[t] @ z[t]
            q[t] -= E[t].T @ z[t + 1]
        Am = np.zeros((N, 4, 6))
        Ap = np.zeros((N, 4, 6))
        b = np.zeros((N, 4))
        for t in range(N):
            Am[t], Ap[t] = self._jac(z[t, :4], z[t, 4:], z[t + 1, :4], self.dt, self.L)
            f = self._res(z[t, :4], z[t, 4:], z[t + 1, :4], self.dt, self.L)
            b[t] = Am[t] @ z[t] + Ap[t] @ z[t + 1] - f
        G = np.stack([self.G_block(t) for t in range(N + 1)])
        gz = self.ineq(z)
        Gz = np.einsum("tij,tj->ti", G, z)
        lo = self.g_lo - gz + Gz
        hi = self.g_hi - gz + Gz
        return StageQP(nx=4, nu=2, N=N, D=D, E=E, q=q, Am=Am, Ap=Ap, b=b,
                       x_init=self.x_init.copy(), G=G, lo=lo, hi=hi, soft=self.soft.copy(),
                       gamma2=1.0, gamma1=self.gamma1)
