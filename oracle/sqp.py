"""SQP outer loop of Algorithm 1 with the backtracking line search of
Appendix "Line search" and the stopping test of eq. sqp_stop.

Readings where the paper leaves a choice open:
* each QP is warm-started from the current iterate (x = xbar, z_g = G xbar,
  y = ybar) and the previous rho-bar;
* merit phi = l(x) + slack penalty + mu (||f||_1 + ||[g + xi - g_hi]_+||_1
  + ||[g_lo - g - xi]_+||_1), f including the initial-state row;
* mu_k = max(mu_{k-1}, |grad l' dx| / (0.5 max(viol, eps_c)), 1) (the printed
  ratio can be <= 0, which would defeat the Armijo test);
* the directional derivative of the L1 slack penalty at xi_i = 0 is
  gamma1 |dxi_i|;
* candidates alpha in {1, 1/2, ..., 1/128}; the largest one passing the
  Armijo test (eta = 0.4) wins, otherwise the candidate with the smallest
  finite merit (ties to the larger alpha);
* multipliers move with the same step: y <- ybar + alpha (y* - ybar).

Parity: unpinned as a trajectory (discrete line-search decisions); pinned at
convergence by the NLP KKT test of eq. sqp_stop and, for linear problems, by
one-step convergence (tests/test_oracle_sqp.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .admm import ADMMSettings, admm_solve
from .qp import SOFT_L1, SOFT_L2

ALPHAS = tuple(2.0 ** -j for j in range(8))


@dataclass
class SQPSettings:
    max_sqp: int = 10
    eps_c: float = 1e-4
    armijo_eta: float = 0.4
    fixed_iters: bool = True  # run exactly max_sqp iterations (throughput mode)


@dataclass
class SQPResult:
    z: np.ndarray  # [(N+1), n]
    xi: np.ndarray  # [(N+1), ng]
    y_f: np.ndarray
    y_g: np.ndarray
    rho_bar: float
    sqp_iters: int
    admm_iters: list
    alphas: list
    stop: dict
    converged: bool
    history: list = field(default_factory=list)


def _slack_penalty(ocp, xi):
    kind = np.tile(ocp.soft, ocp.N + 1)
    xi = xi.reshape(-1)
    return ocp.gamma1 * np.sum(np.abs(xi[kind == SOFT_L1])) + 0.5 * np.sum(xi[kind == SOFT_L2] ** 2)


def _violation(ocp, z, xi):
    g = ocp.ineq(z) + xi
    f = ocp.eq_residual(z)
    return (np.sum(np.abs(f)) + np.sum(np.maximum(g - ocp.g_hi, 0.0))
            + np.sum(np.maximum(ocp.g_lo - g, 0.0)))


def merit(ocp, z, xi, mu):
    return ocp.cost(z) + _slack_penalty(ocp, xi) + mu * _violation(ocp, z, xi)


def _penalty_dirderiv(ocp, z, xi, dz, dxi):
    kind = np.tile(ocp.soft, ocp.N + 1)
    x1 = xi.reshape(-1)[kind == SOFT_L1]
    d1 = dxi.reshape(-1)[kind == SOFT_L1]
    l1 = ocp.gamma1 * np.sum(np.where(x1 != 0.0, np.sign(x1) * d1, np.abs(d1)))
    l2 = np.sum(xi.reshape(-1)[kind == SOFT_L2] * dxi.reshape(-1)[kind == SOFT_L2])
    return float(np.sum(ocp.cost_grad(z) * dz)) + l1 + l2


def stop_test(ocp, z, xi, y_f, y_g):
    """The three quantities of eq. sqp_stop."""
    N = ocp.N
    lag = ocp.cost_grad(z) + ocp.eq_jac_T_times(z, y_f)
    yg = y_g.reshape(N + 1, ocp.ng)
    for t in range(N + 1):
        lag[t] += ocp.G_block(t).T @ yg[t]
    g = ocp.ineq(z) + xi.reshape(N + 1, ocp.ng)
    viol = max(float(np.max(g - ocp.g_hi)), float(np.max(ocp.g_lo - g)), 0.0)
    return {"stationarity": float(np.max(np.abs(lag))),
            "eq": float(np.max(np.abs(ocp.eq_residual(z)))), "ineq": viol}


def line_search(ocp, z, xi, dz, dxi, mu_prev, st: SQPSettings):
    """Backtracking line search; returns (alpha, mu)."""
    gdir = _penalty_dirderiv(ocp, z, xi, dz, dxi)
    viol = _violation(ocp, z, xi)
    mu = max(mu_prev, abs(gdir) / (0.5 * max(viol, st.eps_c)), 1.0)
    d_mu = gdir - mu * viol
    phi0 = merit(ocp, z, xi, mu)
    phis = [merit(ocp, z + a * dz, xi + a * dxi, mu) for a in ALPHAS]
    for a, ph in zip(ALPHAS, phis):
        if np.isfinite(ph) and ph <= phi0 + st.armijo_eta * a * d_mu:
            return a, mu
    finite = [(ph, -a) for a, ph in zip(ALPHAS, phis) if np.isfinite(ph)]
    if not finite:
        return 0.0, mu
    return -min(finite)[1], mu


def sqp_solve(ocp, st: SQPSettings = SQPSettings(), admm: ADMMSettings = None, z0=None,
              record=False) -> SQPResult:
    admm = admm or ADMMSettings(max_iter=50, k_check=0)
    N, ng = ocp.N, ocp.ng
    z = ocp.initial_guess() if z0 is None else np.array(z0, float)
    xi = np.zeros((N + 1, ng))
    y_f = np.zeros(ocp.nx * (N + 1))
    y_g = np.zeros(ng * (N + 1))
    rho_bar = admm.rho0
    mu = 0.0
    iters, alphas, hist = [], [], []
    converged = False
    k = 0
    for k in range(1, st.max_sqp + 1):
        qp = ocp.convexify(z)
        warm = {"x": z.reshape(-1), "z_g": np.einsum("tij,tj->ti", qp.G, z).reshape(-1),
                "y_f": y_f, "y_g": y_g, "rho_bar": rho_bar}
        r = admm_solve(qp, admm, warm=warm)
        iters.append(r.iters)
        rho_bar = r.rho_bar
        dz = r.x.reshape(N + 1, -1) - z
        dxi = r.xi.reshape(N + 1, ng) - xi
        a, mu = line_search(ocp, z, xi, dz, dxi, mu, st)
        alphas.append(a)
        z = z + a * dz
        xi = xi + a * dxi
        y_f = y_f + a * (r.y_f - y_f)
        y_g = y_g + a * (r.y_g - y_g)
        s = stop_test(ocp, z, xi, y_f, y_g)
        if record:
            hist.append((z.copy(), s))
        if max(s.values()) <= st.eps_c:
            converged = True
            if not st.fixed_iters:
                break
    return SQPResult(z, xi, y_f, y_g, rho_bar, k, iters, alphas, stop_test(ocp, z, xi, y_f, y_g),
                     converged, hist)
