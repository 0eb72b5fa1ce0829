"""Implicit derivative of the SQP solution (Algorithm 2 applied at the
converged SQP iterate; Sec. "Backward Pass"; eq. bwd:noslack_kkt_matrix with
H the Hessian of the Lagrangian).

At a KKT point (z, y_f, y_g, xi) of the OCP the conditions are
    grad l(z) + grad f(z)' y_f + G' y_g = 0,   f(z) = 0,   g_A(z) = b_A
and the VJP of a loss solves K eta = (dL/dz, 0, 0) with
    K = [[H, grad f', G_A'], [grad f, 0, 0], [G_A, 0, 0]],
    H = grad^2 l + sum_t y_f,t' grad^2 f_t     (the exact Lagrangian Hessian),
or H = grad^2 l alone (the Gauss-Newton approximation the paper offers as an
option).  This is the QP convexified at z with D_t, E_t replaced by the
blocks of H, so the dense active-set solve of oracle.adjoint applies.

Parameter gradients (theta of the kinematic-bicycle OCP; -(dF/dtheta)' eta):
    dL/dx0        = eta_f on the initial-state rows
    dL/dQ_jj      = -sum_{t<N} eta_x,t,j (z_t,j - r_t,j)     (Q_f at t = N)
    dL/dR_jj      = -sum_t eta_u,t,j u_t,j
    dL/dr_t       = W_t eta_x,t   (+ eta_g,lat n_t on the lateral row, whose
                    value n_t'(p_t - r_t) moves with r_t)
    dL/dbound     = sum_t (d_hi - d_lo) on that row (bounds -b <= g <= b)

Parity: the dynamics Hessian against central differences of the Lagrangian
gradient; the parameter gradients against central differences of tightly
converged oracle SQP solutions (tests/test_oracle_sqp_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from .adjoint import active_set, adjoint_dense, qp_vjp
from .models import BicycleOCP


def fc_hessian(x, u, L, y):
    """sum_k y_k grad^2 fc_k at (x, u), over w = (px, py, yaw, v, a, delta)."""
    _, _, yaw, v = x
    _, d = u
    A = np.zeros((6, 6))
    A[2, 2] = -y[0] * v * np.cos(yaw) - y[1] * v * np.sin(yaw)
    A[2, 3] = A[3, 2] = -y[0] * np.sin(yaw) + y[1] * np.cos(yaw)
    c2 = np.cos(d) ** 2
    A[3, 5] = A[5, 3] = y[2] / (L * c2)
    A[5, 5] = y[2] * 2.0 * v * np.tan(d) / (L * c2)
    return A


def dynamics_hessian(ocp: BicycleOCP, z, y_dyn, trapezoid=False):
    """Blocks of sum_t y_dyn,t' grad^2 f_t over the stage variables:
    Hd [N+1, 6, 6] (diagonal blocks) and He [N, 6, 6] (block (t+1, t))."""
    N, dt, L = ocp.N, ocp.dt, ocp.L
    Hd = np.zeros((N + 1, 6, 6))
    He = np.zeros((N, 6, 6))
    # variables of row t: v = (x_t [4], u_t [2], x_{t+1} [4])
    for t in range(N):
        y = y_dyn[t]
        xt, ut, xn = z[t, :4], z[t, 4:], z[t + 1, :4]
        if trapezoid:
            M1 = np.zeros((6, 10))
            M1[:4, :4] = np.eye(4)
            M1[4:, 4:6] = np.eye(2)
            M2 = np.zeros((6, 10))
            M2[:4, 6:] = np.eye(4)
            M2[4:, 4:6] = np.eye(2)
            Hv = 0.5 * dt * (M1.T @ fc_hessian(xt, ut, L, y) @ M1 + M2.T @ fc_hessian(xn, ut, L, y) @ M2)
        else:
            M = np.zeros((6, 10))
            M[:4, :4] = 0.5 * np.eye(4)
            M[:4, 6:] = 0.5 * np.eye(4)
            M[4:, 4:6] = np.eye(2)
            Hv = dt * (M.T @ fc_hessian(0.5 * (xt + xn), ut, L, y) @ M)
        Hd[t] += Hv[:6, :6]
        Hd[t + 1, :4, :4] += Hv[6:, 6:]
        He[t, :4, :] = Hv[6:, :6]
    return Hd, He


def sqp_qp_at(ocp: BicycleOCP, z, y_f, exact=True):
    """The QP convexified at z with the Hessian of the Lagrangian (exact) or
    of the cost alone (Gauss-Newton) as its P."""
    qp = ocp.convexify(z)
    if exact:
        y_dyn = np.asarray(y_f, float)[4:].reshape(ocp.N, 4)
        Hd, He = dynamics_hessian(ocp, z, y_dyn, trapezoid=ocp._res.__name__.startswith("trap"))
        qp.D = qp.D + Hd
        qp.E = qp.E + He
    return qp


def sqp_param_grads(ocp: BicycleOCP, z, xi, y_f, y_g, dL_dz, exact=True, eps_active=1e-6):
    """Gradients of a loss of the SQP solution w.r.t. the OCP parameters (see
    the module docstring).  z [(N+1), 6]; xi, y_g [(N+1) ng] or [(N+1), ng];
    y_f [(N+1) nx] (initial-state rows first).  Returns a dict with x0, Qd,
    Rd, Qfd, ref [(N+1), 4], bounds (a, delta, lateral) and the adjoint
    (eta_x, eta_f, eta_g, lower, upper)."""
    z = np.asarray(z, float).reshape(ocp.N + 1, 6)
    qp = sqp_qp_at(ocp, z, y_f, exact)
    xi = np.asarray(xi, float).reshape(-1)
    yg = np.asarray(y_g, float).reshape(-1)
    lower, upper = active_set(qp, z.reshape(-1), yg, xi=xi, eps_solve=eps_active)
    ex, ef, eg = adjoint_dense(qp, z.reshape(-1), np.asarray(dL_dz, float).reshape(-1), lower, upper)
    g = qp_vjp(qp, z.reshape(-1), ex, ef, eg, lower, upper, xi=xi)
    N = ocp.N
    exs = ex.reshape(N + 1, 6)
    egs = eg.reshape(N + 1, ocp.ng)
    e = z[:, :4] - ocp.ref
    dref = np.zeros((N + 1, 4))
    for t in range(N + 1):
        W = ocp.Qf if t == N else ocp.Q
        dref[t] = W @ exs[t, :4]
        act = lower.reshape(N + 1, -1)[t, 2] or upper.reshape(N + 1, -1)[t, 2]
        if act:
            dref[t, :2] += egs[t, 2] * ocp.normal[t]
    dbound = (g["d_hi"] - g["d_lo"]).sum(axis=0)
    return {
        "x0": g["d_x_init"],
        "Qd": -(exs[:N, :4] * e[:N]).sum(axis=0),
        "Qfd": -(exs[N, :4] * e[N]),
        "Rd": -(exs[:, 4:] * z[:, 4:]).sum(axis=0),
        "ref": dref,
        "bounds": dbound,
        "eta_x": ex, "eta_f": ef, "eta_g": eg, "lower": lower, "upper": upper,
    }
