"""Exact solve and parameter gradient of the linear-quadratic OCP, used as the
reference for the differentiation workload.

Learnable parameters per instance, theta = (diag Q [nx], diag R [nu], x0 [nx],
u_lo [nu], u_hi [nu]); the terminal weight is tied to Q (Q_f = Q) and the
control bounds are shared by all stages.  Loss  L = ||u_0||^2 + ||x_N||^2.

Parity: pinned by central finite differences of polished solves and by the
closed-form LQR gradient (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from .admm import ADMMSettings, admm_solve
from .adjoint import active_set, adjoint_dense, polish, qp_vjp
from .qp import lti_qp

TIGHT = ADMMSettings(eps_abs=1e-10, eps_rel=1e-10, max_iter=20000, k_check=25)


def theta_of(batch, i):
    nx, nu = batch.nx, batch.nu
    return np.concatenate([batch.Qd[i], batch.Rd[i], batch.x0[i], batch.lo[i][nx:], batch.hi[i][nx:]])


def qp_of_theta(batch, i, theta):
    nx, nu = batch.nx, batch.nu
    Qd, Rd, x0 = theta[:nx], theta[nx:nx + nu], theta[nx + nu:2 * nx + nu]
    ulo, uhi = theta[2 * nx + nu:2 * nx + 2 * nu], theta[2 * nx + 2 * nu:]
    lo = batch.lo[i].copy()
    hi = batch.hi[i].copy()
    lo[nx:] = ulo
    hi[nx:] = uhi
    return lti_qp(batch.A[i], batch.B[i], Qd, Rd, Qd, batch.G, lo, hi, x0, batch.N)


def loss_and_grad_x(qp, x):
    xs = x.reshape(qp.N + 1, qp.n)
    u0 = xs[0, qp.nx:]
    xN = xs[qp.N, :qp.nx]
    g = np.zeros_like(xs)
    g[0, qp.nx:] = 2.0 * u0
    g[qp.N, :qp.nx] = 2.0 * xN
    return float(u0 @ u0 + xN @ xN), g.reshape(-1)


def solve_exact(qp, settings=TIGHT, warm=None):
    """ADMM to a tight tolerance followed by the active-set polish."""
    r = admm_solve(qp, settings, warm=warm)
    ok, sol = polish(qp, r.x, r.y_g, eps_solve=max(settings.eps_abs, 1e-8))
    return ok, sol, r


def theta_grad_from_qp_grads(batch, qg):
    """Chain dL/d(QP data) into dL/dtheta for the box-on-all-variables LTI layout
    (G = I, rows nx..n-1 are the controls)."""
    nx, nu = batch.nx, batch.nu
    dD = qg["d_Ddiag"]
    dQ = dD[:, :nx].sum(axis=0)
    dR = dD[:, nx:].sum(axis=0)
    dx0 = qg["d_x_init"]
    dulo = qg["d_lo"][:, nx:].sum(axis=0)
    duhi = qg["d_hi"][:, nx:].sum(axis=0)
    return np.concatenate([dQ, dR, dx0, dulo, duhi])


def implicit_theta_grad(batch, i, sol=None):
    """dL/dtheta by the dense active-set adjoint at the polished solution."""
    theta = theta_of(batch, i)
    qp = qp_of_theta(batch, i, theta)
    if sol is None:
        ok, sol, _ = solve_exact(qp)
        if not ok:
            raise RuntimeError("polish failed")
    L, gx = loss_and_grad_x(qp, sol["x"])
    ex, ef, eg = adjoint_dense(qp, sol["x"], gx, sol["lower"], sol["upper"])
    qg = qp_vjp(qp, sol["x"], ex, ef, eg, sol["lower"], sol["upper"])
    return L, theta_grad_from_qp_grads(batch, qg), sol


def fd_theta_grad(batch, i, h=1e-6, sol=None):
    """Central finite differences of L(theta), each perturbed problem solved
    exactly with the base active set re-certified by the polish step."""
    theta = theta_of(batch, i)
    qp0 = qp_of_theta(batch, i, theta)
    if sol is None:
        ok, sol, _ = solve_exact(qp0)
        if not ok:
            raise RuntimeError("polish failed")
    grad = np.zeros_like(theta)
    for k in range(len(theta)):
        vals = []
        for s in (+1.0, -1.0):
            th = theta.copy()
            th[k] += s * h
            qp = qp_of_theta(batch, i, th)
            ok, sp_, _ = _resolve_same_active(qp, sol)
            if not ok:
                ok, sp_, _ = solve_exact(qp)
                if not ok:
                    raise RuntimeError("perturbed polish failed")
            vals.append(loss_and_grad_x(qp, sp_["x"])[0])
        grad[k] = (vals[0] - vals[1]) / (2 * h)
    return grad


def _resolve_same_active(qp, base_sol):
    """Polish the perturbed QP starting from the base solution's (x, y_g)."""
    ok, sol = polish(qp, base_sol["x"], base_sol["y_g"], eps_solve=1e-8)
    same = ok and np.array_equal(sol["lower"], base_sol["lower"]) and np.array_equal(sol["upper"], base_sol["upper"])
    return same, sol, None
