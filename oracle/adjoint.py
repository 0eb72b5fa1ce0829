"""Active-set identification, polish and implicit-differentiation VJP
(Algorithm 2; Sec. "Backward Pass"; Appendix "Backward Pass: Sensitivities
Computation").

For the QP  min 1/2 x'Px + q'x  s.t.  Cx = c, lo <= Gx <= hi  at a solution
(x, y_f, y_g) with active rows A (lower L, upper U), the active-set KKT map is

    F(w, theta) = [ H x + q + C'y_f + G_A'y_A ;  C x - c ;  G_A x - b_A ]

with b_A = lo on L rows and hi on U rows.  The VJP of a loss with gradient
dL/dx solves  K eta = (dL/dx, 0, 0),  K = [[H, C', G_A'], [C, 0, 0], [G_A, 0, 0]]
(eq. bwd:noslack_kkt_matrix; K is symmetric so its transpose is itself) and
returns  dL/dtheta = -(dF/dtheta)' eta  (eq. loss_gradient):

    dL/dq      = -eta_x
    dL/dc      = +eta_f          (so dL/dx_init = eta_f on the initial rows)
    dL/dD_t[i,i] = -eta_x[t,i] * x[t,i]
    dL/dlo_i   = +eta_A,i on lower-active rows, 0 elsewhere
    dL/dhi_i   = +eta_A,i on upper-active rows, 0 elsewhere

Soft rows: an L1 row whose slack is nonzero has the fixed multiplier
-gamma1 sign(xi) and drops out of the system; an L1 row with xi = 0 is treated
as a hard row.  An active L2-slack row (penalty gamma2/2 xi^2) keeps its slack
through the eliminated slack stationarity gamma2 xi + y = 0, so its active
equation reads G_i x - y_i / gamma2 = b_i (eq. bwd:kkt_active with the slack
toggle on): K carries -1/gamma2 on that row's diagonal.  Eliminating those
rows gives the reduced system of eq. bwd:slack_reduced_system,
[[H + gamma2 G_S'G_S, J'], [J, 0]] with J = [C; hard active rows] and
eta_y = gamma2 G_S eta_x on the slack rows (no loss term on xi), which is the
form the regularised refinement below (the GPU scheme) solves.

Parity: the dense direct solve is the definition; pinned by central finite
differences of polished solutions and by the closed-form LQR gradient
(tests/test_oracle_adjoint.py).  The regularised refinement variant is pinned
against the dense solve.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .qp import HARD, SOFT_L1, SOFT_L2, StageQP


def active_set(qp: StageQP, x, y_g, xi=None, eps_g=None, eps_solve=1e-4):
    """Lower/upper active masks by the rule of Appendix "Active constraints
    identification": the dual sign decides; closeness to a bound only when the
    dual is ambiguous (|y| < eps_g).  The tolerance combines an absolute and a
    relative part on each side: eps_g = 10 eps_solve max(1, ||y_g||_inf) for
    the dual test (relative to the multipliers), 10 eps_solve max(1, |bound|)
    for the proximity test (relative to the bound, as the paper's eps_g |g_i|).
    Rows whose L1 slack is nonzero are returned in neither mask.
    """
    _, _, G, _, _, lo, hi = qp.matrices()
    g = G @ x
    y_g = np.asarray(y_g, float)
    if eps_g is None:
        eps_g = 10.0 * eps_solve * max(1.0, float(np.max(np.abs(y_g))) if y_g.size else 1.0)
    eps_p = 10.0 * eps_solve
    amb = np.abs(y_g) < eps_g
    lower = (y_g < -eps_g) | (amb & (g - lo <= eps_p * np.maximum(1.0, np.abs(lo))))
    upper = (y_g > eps_g) | (amb & (hi - g <= eps_p * np.maximum(1.0, np.abs(hi))))
    both = lower & upper
    lower = lower & ~(both & (y_g > 0))
    upper = upper & ~(both & ~(y_g > 0))
    kind = qp.soft_rows()
    if xi is not None:
        drop = (kind == SOFT_L1) & (np.asarray(xi) != 0.0)
        lower &= ~drop
        upper &= ~drop
    return lower, upper


def _kkt(qp: StageQP, lower, upper, H=None):
    P, C, G, q, c, lo, hi = qp.matrices()
    H = P if H is None else H
    act = lower | upper
    idx = np.flatnonzero(act)
    GA = G[idx]
    # active L2-slack rows: G_i x - y_i / gamma2 = b_i
    dA = np.where(qp.soft_rows()[idx] == SOFT_L2, 1.0 / qp.gamma2, 0.0)
    D = -sp.diags(dA) if np.any(dA) else None
    K = sp.bmat([[H, C.T, GA.T], [C, None, None], [GA, None, D]], format="csc")
    bA = np.where(lower, lo, hi)[act]
    return K, P, C, G, q, c, GA, bA, act


def polish(qp: StageQP, x, y_g, xi=None, eps_solve=1e-4, tol=1e-9):
    """Solve the equality-constrained KKT system on the identified active set
    and certify it: primal feasibility, dual signs and (by construction)
    complementarity.  Returns (ok, sol) with sol = dict(x, y_f, y_g, z_g, xi).
    Soft L1 rows with nonzero slack keep the multiplier -gamma1 sign(xi).
    """
    lower, upper = active_set(qp, x, y_g, xi=xi, eps_solve=eps_solve)
    K, P, C, G, q, c, GA, bA, act = _kkt(qp, lower, upper)
    nv, ne = qp.nvar, qp.neq
    kind = qp.soft_rows()
    fixed = np.zeros(qp.nineq)
    if xi is not None:
        sel = (kind == SOFT_L1) & (np.asarray(xi) != 0.0)
        fixed[sel] = -qp.gamma1 * np.sign(np.asarray(xi)[sel])
    rhs = np.concatenate([-q - G.T @ fixed, c, bA])
    sol = spla.spsolve(K, rhs)
    xs = sol[:nv]
    yf = sol[nv:nv + ne]
    yg = fixed.copy()
    yg[act] = sol[nv + ne:]
    g = G @ xs
    lo, hi = qp.lo.reshape(-1), qp.hi.reshape(-1)
    xis = np.zeros(qp.nineq)
    if xi is not None:
        sel = (kind == SOFT_L1) & (np.asarray(xi) != 0.0)
        xis[sel] = np.clip(g[sel], lo[sel], hi[sel]) - g[sel]
    l2 = (kind == SOFT_L2) & act
    xis[l2] = -yg[l2] / qp.gamma2  # slack stationarity gamma2 xi + y = 0
    gx = g + xis
    feas = np.all(gx >= lo - tol * np.maximum(1, np.abs(lo))) and np.all(gx <= hi + tol * np.maximum(1, np.abs(hi)))
    signs = np.all(yg[lower] <= tol) and np.all(yg[upper] >= -tol)
    ok = bool(feas and signs and np.all(np.isfinite(sol)))
    return ok, {"x": xs, "y_f": yf, "y_g": yg, "z_g": g, "xi": xis, "lower": lower, "upper": upper}


DENSE_LIMIT = 4e7  # entries of the largest J given to the dense rank test (about 320 MB)


def independent_rows(qp: StageQP, lower, upper, rtol=1e-9) -> bool:
    """True if the rows of J = [C; G_A] (hard active rows; active L2-slack
    rows carry their own diagonal and never make K singular) are linearly
    independent (LICQ), by the pivoted QR of J' (rank = number of diagonal
    entries of R above rtol times the largest).  Problems whose J has more
    than DENSE_LIMIT entries (the long horizons) are not tested and taken as
    independent."""
    _, C, G, *_ = qp.matrices()
    act = (lower | upper) & (qp.soft_rows() != SOFT_L2)
    J = sp.vstack([C, G[np.flatnonzero(act)]])
    if J.shape[0] > J.shape[1]:
        return False
    if J.shape[0] * J.shape[1] > DENSE_LIMIT:
        return True  # too large for a dense rank test: taken as independent
    R = sla.qr(J.toarray().T, mode="r", pivoting=True)[0]
    d = np.abs(np.diag(R))
    return bool(d.size == 0 or d.min() > rtol * d.max())


def _slack_rows(qp: StageQP, lower, upper, xi):
    """Rows whose slack is a function of x at the solution: active L2-slack
    rows, and L1-slack rows with nonzero slack (xi_i = bound - G_i x there)."""
    kind = qp.soft_rows()
    l2 = (lower | upper) & (kind == SOFT_L2)
    l1 = np.zeros_like(l2) if xi is None else (kind == SOFT_L1) & (np.asarray(xi) != 0.0)
    return l2, l1


def slack_rhs(qp: StageQP, dL_dx, dL_dxi, lower, upper, xi=None):
    """x-part of the reduced right-hand side with a loss on the slacks
    (eq. bwd:slack_reduced_system): dL/dx - G_S' dL/dxi over the rows whose
    slack moves with x (active L2 rows; L1 rows with nonzero slack, whose
    xi = bound - G x gives the same term)."""
    if dL_dxi is None:
        return np.asarray(dL_dx, float)
    l2, l1 = _slack_rows(qp, lower, upper, xi)
    G = qp.matrices()[2]
    w = np.where(l2 | l1, np.asarray(dL_dxi, float).reshape(-1), 0.0)
    return np.asarray(dL_dx, float) - G.T @ w


def adjoint_dense(qp: StageQP, x, dL_dx, lower, upper, H=None, dL_dxi=None, xi=None):
    """eta = K^{-1} (dL/dx, 0, 0) by a direct sparse LU (the definition).

    With a loss on the slacks (dL_dxi [nineq], `xi` the solution's slacks):
    eq. loss_gradient's right-hand side (dL/dx, dL/dxi, 0) of the slack
    system eq. bwd:slack_adjoint, written on K (slacks of the active L2 rows
    eliminated through their stationarity gamma2 xi + y = 0): the active L2
    row of K reads G_i e_x - e_y,i / gamma2 = -dL/dxi_i / gamma2; an L1 row
    with nonzero slack is not in K and its loss enters through
    xi_i = bound - G_i x as -G_i' dL/dxi_i in the x-part.

    When the active rows are linearly dependent (LICQ fails; at eps 1e-4 this
    happens on unconverged instances; the LU then shows a pivot below 1e-12 of
    the largest, or none at all), K is singular but the system stays
    consistent: eta_x is unique (H is positive definite) and eta_y is
    determined up to the null space of J'.  The result is then the
    minimum-norm solution K^+ (dL/dx, 0, 0) by a dense least-squares solve
    (singular values below 1e-12 of the largest taken as zero),
    whose eta_y lies in the range of J -- the limit of the regularised
    refinement started from zero (its eta_y updates are rho_b (J e_x - r_y)).
    """
    K, *_ , act = _kkt(qp, lower, upper, H)
    nv, ne = qp.nvar, qp.neq
    rhs = np.concatenate([dL_dx, np.zeros(ne + int(act.sum()))])
    if dL_dxi is not None:
        l2, l1 = _slack_rows(qp, lower, upper, xi)
        dxi = np.asarray(dL_dxi, float).reshape(-1)
        G = qp.matrices()[2]
        rhs[:nv] -= G.T @ np.where(l1, dxi, 0.0)
        ry = np.where(l2, -dxi / qp.gamma2, 0.0)
        rhs[nv + ne:] = ry[act]
    lu = None
    try:
        lu = spla.splu(K)
        piv = np.abs(lu.U.diagonal())
        if not (piv.min() > 1e-12 * piv.max()):  # a pivot at rounding level: K is singular
            lu = None
    except RuntimeError:  # exactly singular
        lu = None
    if lu is not None:
        eta = lu.solve(rhs)
    else:
        eta = sla.lstsq(K.toarray(), rhs, cond=1e-12, lapack_driver="gelsd")[0]
    eta_g = np.zeros(qp.nineq)
    eta_g[act] = eta[nv + ne:]
    return eta[:nv], eta[nv:nv + ne], eta_g


def adjoint_refined(qp: StageQP, x, dL_dx, lower, upper, sigma_b=1e-9, rho_b=1e6, sweeps=4, H=None,
                    dL_dxi=None, xi=None):
    """Same eta by iterative refinement on K with the regularised matrix
    K_reg = [[H + sigma_b I, J'], [J, -rho_b^{-1} I]], J = [C; G_A] (active
    L2-slack rows leave J and add gamma2 G_S'G_S to H, their eta_y recovered
    as gamma2 G_S eta_x: eq. bwd:slack_reduced_system):
    e <- e + K_reg^{-1} (r - K e).  Each K_reg solve is one Schur step
    (H + sigma_b I + rho_b J'J) e_x = r_x + rho_b J' r_y, e_y = rho_b (J e_x - r_y).
    Written with dense NumPy algebra (the oracle's plain form of the GPU scheme).
    """
    P, C, G, q, c, lo, hi = qp.matrices()
    H = P if H is None else H
    act = lower | upper
    l2 = act & (qp.soft_rows() == SOFT_L2)  # slack rows: in H (eq. bwd:slack_reduced_system)
    hard = act & ~l2
    J = sp.vstack([C, G[np.flatnonzero(hard)]]).tocsr()
    nv = qp.nvar
    Gs = G[np.flatnonzero(l2)].toarray() if sp.issparse(G) else np.asarray(G)[np.flatnonzero(l2)]
    Hd = H.toarray() + qp.gamma2 * Gs.T @ Gs
    Jd = J.toarray()
    S = Hd + sigma_b * np.eye(nv) + rho_b * Jd.T @ Jd
    Lc = np.linalg.cholesky(S)

    def kreg_solve(rx, ry):
        ex = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rx + rho_b * Jd.T @ ry))
        ey = rho_b * (Jd @ ex - ry)
        return ex, ey

    rx0 = slack_rhs(qp, dL_dx, dL_dxi, lower, upper, xi)  # eq. bwd:slack_reduced_system
    ry0 = np.zeros(Jd.shape[0])
    ex, ey = kreg_solve(rx0, ry0)
    for _ in range(sweeps - 1):
        rx = rx0 - (Hd @ ex + Jd.T @ ey)
        ry = ry0 - Jd @ ex
        dx, dy = kreg_solve(rx, ry)
        ex, ey = ex + dx, ey + dy
    ne = qp.neq
    eta_g = np.zeros(qp.nineq)
    eta_g[hard] = ey[ne:]
    eta_g[l2] = qp.gamma2 * (Gs @ ex)  # eq. bwd:slack:eta_xi_yg
    if dL_dxi is not None:
        eta_g[l2] += np.asarray(dL_dxi, float).reshape(-1)[l2]
    return ex, ey[:ne], eta_g


def qp_vjp(qp: StageQP, x, eta_x, eta_f, eta_g, lower, upper, xi=None, dL_dxi=None):
    """Map eta to gradients of the QP data (eq. loss_gradient).  With the
    slacks `xi` given, also:

    * dL/dgamma2: gamma2 enters only the active slack rows' equation
      G_i x - y_i / gamma2 = b_i, whose derivative y_i / gamma2^2 =
      -xi_i / gamma2 (slack stationarity) with eta_y,i = gamma2 G_i eta_x +
      dL/dxi_i gives dL/dgamma2 = -xi_A' eta_xi = sum_i xi_i (G eta_x)_i over
      those rows (the paper's xi_A' S grad g_A eta_x);
    * dL/dgamma1: an L1 row with nonzero slack carries the fixed multiplier
      -gamma1 sign(xi_i) in the stationarity, so dL/dgamma1 =
      sum_i sign(xi_i) (G eta_x)_i over those rows;
    * eta_xi = -G_i eta_x on the rows whose slack moves with x (eq.
      bwd:slack:eta_xi_yg; active L2 rows, L1 rows with nonzero slack), 0
      elsewhere.

    With a loss on the slacks (dL_dxi), an L1 row with nonzero slack
    xi_i = bound_i - G_i x also passes dL/dxi_i to that bound (lower when
    xi_i > 0, upper when xi_i < 0)."""
    n = qp.n
    xs = np.asarray(x).reshape(qp.N + 1, n)
    ex = np.asarray(eta_x).reshape(qp.N + 1, n)
    d_lo = np.where(lower, eta_g, 0.0)
    d_hi = np.where(upper, eta_g, 0.0)
    d_gamma2 = d_gamma1 = eta_xi = None
    if xi is not None:
        G = qp.matrices()[2]
        gex = G @ np.asarray(eta_x)
        xi = np.asarray(xi, float).reshape(-1)
        l2, l1 = _slack_rows(qp, lower, upper, xi)
        d_gamma2 = float(np.sum(xi[l2] * gex[l2]))
        d_gamma1 = float(np.sum(np.sign(xi[l1]) * gex[l1]))
        eta_xi = np.where(l2 | l1, -gex, 0.0).reshape(qp.N + 1, qp.ng)
        if dL_dxi is not None:
            dxi = np.asarray(dL_dxi, float).reshape(-1)
            d_lo = d_lo + np.where(l1 & (xi > 0), dxi, 0.0)
            d_hi = d_hi + np.where(l1 & (xi < 0), dxi, 0.0)
    return {
        "d_gamma2": d_gamma2,
        "d_gamma1": d_gamma1,
        "eta_xi": eta_xi,
        "d_q": -ex,
        "d_c": np.asarray(eta_f).copy(),
        "d_x_init": np.asarray(eta_f)[: qp.nx].copy(),
        "d_Ddiag": -ex * xs,
        "d_lo": d_lo.reshape(qp.N + 1, qp.ng),
        "d_hi": d_hi.reshape(qp.N + 1, qp.ng),
    }
