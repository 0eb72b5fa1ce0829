"""ADMM QP solver of Algorithm 3 (Sec. "Solving QP via ADMM"; Appendix "ADMM").

One iteration, in the paper's order:

  1. primal update: solve S x~ = eta with S = P + sigma I + C' rho_f C + G' rho_g G,
     eta = sigma x - q + C'(rho_f c - y_f) + G'(rho_g z_g - y_g)   (Schur system);
     z~ = (C x~, G x~);
  2. over-relaxation x^ = a x~ + (1-a) x,  z^_f = a C x~ + (1-a) c,
     z^_g = a G x~ + (1-a) z_g;  x <- x^ (w == 0);
  3. slack update / projection of v = z^_g + y_g / rho_g:
       hard rows  z = Pi(v), xi = 0;
       L2 rows    z = (rho v + g2 Pi v)/(g2 + rho), xi = rho (Pi v - v)/(g2 + rho)
                  (smoothed projection, eq. proj:tilde);
       L1 rows    z = v + clip(Pi v - v, -g1/rho, g1/rho), xi = Pi v - z
                  (the prox of g1 |xi| under z + xi in [lo, hi]; see `project`);
  4. dual update y_f += rho_f (z^_f - c), y_g += rho_g (z^_g - z_g);
  5. residuals (eq. admm:residuals), stop test (eq. admm:termination:slack)
     and the rho-bar adaptation (eq. rho:update), rho_f = 1e3 rho-bar,
     rho_g = rho-bar; at convergence checks that do not stop, the change of
     the multipliers since the previous check is tested as a primal
     infeasibility certificate (status 4; see infeasibility_certificate).

The Schur system is solved with SciPy's banded Cholesky (LAPACK pbtrf/pbtrs)
on the (2n-1)-band storage of S; a failed factorisation is reported as a
factor breakdown.

Parity: projections pinned by brute-force prox minimisation; the Schur step by
a dense LU of the full regularised KKT system; the converged result by a KKT
certificate, by brute-force active-set enumeration on tiny problems and by the
closed-form LQR solution (tests/test_oracle_admm.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np
import scipy.linalg as sla

from .qp import HARD, SOFT_L1, SOFT_L2, StageQP

CONVERGED, MAX_ITER, NON_FINITE, FACTOR_BREAKDOWN, PRIMAL_INFEASIBLE = 0, 1, 2, 3, 4


@dataclass
class ADMMSettings:
    sigma: float = 1e-6
    rho0: float = 0.1
    rho_f_scale: float = 1e3
    rho_min: float = 1e-6
    rho_max: float = 1e6
    k_rho: int = 25
    k_ratio: float = 5.0
    alpha: float = 1.6
    eps_abs: float = 1e-4
    eps_rel: float = 1e-4
    max_iter: int = 1000
    k_check: int = 25  # 0 = never test for convergence (fixed iteration count)
    adapt_rho: bool = True
    eps_pinf: float = 1e-4  # primal-infeasibility certificate tolerance (0 = no test)
    # primal-update solver: "direct" (banded Cholesky) or "pcg" (block-Jacobi
    # preconditioned CG from the current x, oracle.pcg; at most pcg_max_iter
    # iterations, relative residual pcg_tol)
    linsolve: str = "direct"
    pcg_max_iter: int = 50
    pcg_tol: float = 1e-10

    def with_(self, **kw) -> "ADMMSettings":
        return replace(self, **kw)


@dataclass
class ADMMResult:
    x: np.ndarray
    z_g: np.ndarray
    xi: np.ndarray
    y_f: np.ndarray
    y_g: np.ndarray
    rho_bar: float
    iters: int
    status: int
    r_prim: float
    r_dual: float
    n_factor: int
    history: list = field(default_factory=list)
    rho_changes: list = field(default_factory=list)  # (iteration, accepted rho-bar)
    pcg_iters: list = field(default_factory=list)  # CG iterations of each primal update (linsolve "pcg")


def project(v, lo, hi, kind, rho_g, gamma2, gamma1):
    """Slack update for the inequality block: returns (z_g, xi).

    Hard rows: Euclidean projection onto [lo, hi] (xi = 0).
    L2 rows: minimiser of (gamma2/2) xi^2 + (rho/2)(z - v)^2 s.t. z + xi in [lo, hi]
      (Lemma-1 case analysis in Appendix "ADMM with slack variables").
    L1 rows: minimiser of gamma1 |xi| + (rho/2)(z - v)^2 s.t. z + xi in [lo, hi].
      For fixed w = z + xi the inner problem in xi is a soft-threshold, leaving a
      Huber function of (w - v) that is increasing in |w - v|, so w = Pi(v),
      xi = shrink(Pi v - v, gamma1/rho), z = Pi v - xi (= v + clip(Pi v - v, +-gamma1/rho)).
    """
    pv = np.clip(v, lo, hi)
    z = pv.copy()
    xi = np.zeros_like(v)
    l2 = kind == SOFT_L2
    if np.any(l2):
        z[l2] = (rho_g * v[l2] + gamma2 * pv[l2]) / (gamma2 + rho_g)
        xi[l2] = rho_g * (pv[l2] - v[l2]) / (gamma2 + rho_g)
    l1 = kind == SOFT_L1
    if np.any(l1):
        kappa = gamma1 / rho_g
        d = pv[l1] - v[l1]
        xi[l1] = d - np.clip(d, -kappa, kappa)  # soft-threshold: exactly 0 for |d| <= kappa
        z[l1] = pv[l1] - xi[l1]
    return z, xi


def slack_dual_terms(xi, y_g, kind, gamma2, gamma1):
    """Stationarity of the slack variables and the matching scale terms.

    L2 rows: gamma2 xi + y (eq. admm:residuals, second block).
    L1 rows: the distance of -y from gamma1 * subdifferential(|xi|):
      |y + gamma1 sign(xi)| where xi != 0, max(|y| - gamma1, 0) where xi == 0.
    Returns (residual vector, scale vector for the relative test).
    """
    res = np.zeros(0)
    scale = np.zeros(0)
    l2 = kind == SOFT_L2
    if np.any(l2):
        res = np.concatenate([res, gamma2 * xi[l2] + y_g[l2]])
        scale = np.concatenate([scale, np.abs(gamma2 * xi[l2]), np.abs(y_g[l2])])
    l1 = kind == SOFT_L1
    if np.any(l1):
        x1, y1 = xi[l1], y_g[l1]
        r1 = np.where(x1 != 0.0, np.abs(y1 + gamma1 * np.sign(x1)), np.maximum(np.abs(y1) - gamma1, 0.0))
        res = np.concatenate([res, r1])
        scale = np.concatenate([scale, gamma1 * (x1 != 0.0), np.abs(y1)])
    return res, scale


def rho_update(rho_bar, r_prim, r_dual, prim_scale, dual_scale, st: ADMMSettings):
    """Step-size candidate of eq. rho:update and its acceptance rule.

    The candidate scales rho-bar by the square root of the ratio of the
    normalised primal residual r_prim / prim_scale to the normalised dual
    residual r_dual / dual_scale, clipped to [rho_min, rho_max]; every
    normaliser is floored at 1e-30 (reading R7).  It is accepted only when it
    differs from the current value by more than the factor k_ratio in either
    direction.  The caller asks only when the iterate is not converged.
    Returns (candidate, accepted).  Pinned by hand-derived cases in
    tests/golden/rho_update.json.
    """
    num = r_prim / max(prim_scale, 1e-30)
    den = r_dual / max(dual_scale, 1e-30)
    cand = rho_bar * np.sqrt(num / max(den, 1e-30))
    cand = float(np.clip(cand, st.rho_min, st.rho_max))
    return cand, bool(max(cand / rho_bar, rho_bar / cand) > st.k_ratio)


def infeasibility_certificate(M, dy_f, dy_g, eps) -> bool:
    """Primal-infeasibility test of an ADMM multiplier increment (the
    certificate of Banjac, Goulart, Stellato and Boyd for ADMM on convex QPs,
    written from its definition): the constraint set {Cx = c, lo <= Gx <= hi}
    is empty if some dy = (dy_f, dy_g) has A'dy = 0 and a negative support
    value c'dy_f + hi'max(dy_g, 0) + lo'min(dy_g, 0) < 0 (Farkas).  dy is the
    change of the multipliers between two convergence checks: on an infeasible
    problem the multipliers grow along such a direction.  Accepted when
    ||A'dy||_inf <= eps ||dy||_inf and the support value < -eps ||dy||_inf.
    Soft rows never bound the slacked constraint set: any nonzero dy on them
    fails the test."""
    nrm = max(_inf(dy_f), _inf(dy_g))
    if not nrm > 0:
        return False
    if _inf(M.C.T @ dy_f + M.G.T @ dy_g) > eps * nrm:
        return False
    if np.any(dy_g[M.kind != HARD] != 0.0):
        return False
    hi_t = np.where(dy_g > 0, M.hi * dy_g, 0.0)
    lo_t = np.where(dy_g < 0, M.lo * dy_g, 0.0)
    return bool(M.c @ dy_f + np.sum(hi_t) + np.sum(lo_t) < -eps * nrm)


def _inf(v) -> float:
    return float(np.max(np.abs(v))) if v.size else 0.0


class _QPMats:
    def __init__(self, qp: StageQP):
        self.qp = qp
        self.P, self.C, self.G, self.q, self.c, self.lo, self.hi = qp.matrices()
        self.kind = qp.soft_rows()
        self.CtC = (self.C.T @ self.C).tocsr()
        self.GtG = (self.G.T @ self.G).tocsr()
        self.u = 2 * qp.n - 1

    def schur(self, sigma, rho_f, rho_g):
        S = self.P + sigma * _speye(self.P.shape[0]) + rho_f * self.CtC + rho_g * self.GtG
        return S

    def factor(self, sigma, rho_f, rho_g):
        """Banded Cholesky of S (lower band storage, bandwidth 2n-1)."""
        S = self.schur(sigma, rho_f, rho_g).tocsr()
        m, u = S.shape[0], self.u
        ab = np.zeros((u + 1, m))
        for k in range(u + 1):
            ab[k, : m - k] = S.diagonal(-k)
        return sla.cholesky_banded(ab, lower=True)

    def residuals(self, x, z_g, xi, y_f, y_g):
        qp = self.qp
        Cx = self.C @ x
        Gx = self.G @ x
        r_prim = max(_inf(Cx - self.c), _inf(Gx - z_g))
        prim_scale = max(_inf(Cx), _inf(Gx), _inf(self.c), _inf(z_g))
        Px = self.P @ x
        Aty = self.C.T @ y_f + self.G.T @ y_g
        sres, sscale = slack_dual_terms(xi, y_g, self.kind, qp.gamma2, qp.gamma1)
        r_dual = max(_inf(Px + self.q + Aty), _inf(sres))
        dual_scale = max(_inf(Px), _inf(Aty), _inf(self.q), _inf(sscale))
        return r_prim, r_dual, prim_scale, dual_scale


def _speye(m):
    import scipy.sparse as sp

    return sp.identity(m, format="csr")


def admm_solve(qp: StageQP, st: ADMMSettings = ADMMSettings(), warm=None, record=False,
               mats: _QPMats | None = None, scaling=None) -> ADMMResult:
    """Run Algorithm 3 on one QP.

    warm: optional dict with any of x, z_g, y_f, y_g, rho_bar (cold start is
    x = 0, z_g = 0, y = 0, rho_bar = rho0).
    record: keep (x, z_g, xi, y_f, y_g) after every iteration in `history`.
    scaling: an oracle.scaling.Scaling (Remark 4): the iterations run on the
    rescaled QP and the step-size update uses its residuals, while the
    stopping test, the reported residuals, the warm start, the history and
    the result are in the original variables.
    """
    if scaling is not None:
        from .scaling import scale_qp, to_scaled, to_unscaled

        Mg = mats or _QPMats(qp)  # the original problem: stopping test and reported residuals
        qp = scale_qp(qp, scaling)
        M = _QPMats(qp)
        fwd = lambda *v: to_scaled(Mg.qp, scaling, *v)  # noqa: E731
        back = lambda *v: to_unscaled(Mg.qp, scaling, *v)  # noqa: E731
    else:
        M = Mg = mats or _QPMats(qp)
        fwd = back = lambda *v: v  # noqa: E731
    nvar, neq, nin = qp.nvar, qp.neq, qp.nineq
    warm = warm or {}
    x = np.array(warm.get("x", np.zeros(nvar)), dtype=float)
    z_g = np.array(warm.get("z_g", np.zeros(nin)), dtype=float)
    y_f = np.array(warm.get("y_f", np.zeros(neq)), dtype=float)
    y_g = np.array(warm.get("y_g", np.zeros(nin)), dtype=float)
    xi = np.zeros(nin)
    if scaling is not None:
        x, z_g, xi, y_f, y_g = fwd(x, z_g, xi, y_f, y_g)
    rho_bar = float(warm.get("rho_bar", st.rho0))
    a = st.alpha
    kind = M.kind

    def factor(rb):
        if st.linsolve == "pcg":
            from .pcg import diag_block_inverses

            S = M.schur(st.sigma, st.rho_f_scale * rb, rb).tocsr()
            return S, diag_block_inverses(S, qp.n)
        return M.factor(st.sigma, st.rho_f_scale * rb, rb)

    pcg_iters = []

    history = []
    rho_changes = []
    n_factor = 0
    try:
        cf = factor(rho_bar)
        n_factor += 1
    except np.linalg.LinAlgError:
        return ADMMResult(*back(x, z_g, xi, y_f, y_g), rho_bar, 0, FACTOR_BREAKDOWN,
                          np.inf, np.inf, n_factor, history)

    status = MAX_ITER
    r_prim = r_dual = np.inf
    k = 0
    y_prev = None  # multipliers at the previous convergence check (original variables)
    for k in range(1, st.max_iter + 1):
        rho_f, rho_g = st.rho_f_scale * rho_bar, rho_bar
        eta = st.sigma * x - M.q + M.C.T @ (rho_f * M.c - y_f) + M.G.T @ (rho_g * z_g - y_g)
        if st.linsolve == "pcg":
            from .pcg import pcg

            xt, it = pcg(cf[0], eta, x, cf[1], st.pcg_max_iter, st.pcg_tol)
            pcg_iters.append(it)
        else:
            xt = sla.cho_solve_banded((cf, True), eta)
        zt_f = M.C @ xt
        zt_g = M.G @ xt
        x = a * xt + (1.0 - a) * x
        zh_f = a * zt_f + (1.0 - a) * M.c
        zh_g = a * zt_g + (1.0 - a) * z_g
        z_g, xi = project(zh_g + y_g / rho_g, M.lo, M.hi, kind, rho_g, qp.gamma2, qp.gamma1)
        y_f = y_f + rho_f * (zh_f - M.c)
        y_g = y_g + rho_g * (zh_g - z_g)
        if record:
            history.append(tuple(v.copy() for v in back(x, z_g, xi, y_f, y_g)))

        check = st.k_check > 0 and k % st.k_check == 0
        adapt = st.adapt_rho and st.k_rho > 0 and k % st.k_rho == 0
        if check or adapt or k == st.max_iter:
            r_prim, r_dual, ps, ds = Mg.residuals(*back(x, z_g, xi, y_f, y_g))
            if not (np.isfinite(r_prim) and np.isfinite(r_dual)):
                status = NON_FINITE
                break
            conv = (r_prim <= st.eps_abs + st.eps_rel * ps) and (r_dual <= st.eps_abs + st.eps_rel * ds)
            if (check or (st.k_check > 0 and k == st.max_iter)) and conv:
                status = CONVERGED
                break
            if check and st.eps_pinf > 0:
                yo = back(x, z_g, xi, y_f, y_g)
                if y_prev is not None and infeasibility_certificate(Mg, yo[3] - y_prev[0], yo[4] - y_prev[1],
                                                                    st.eps_pinf):
                    status = PRIMAL_INFEASIBLE
                    break
                y_prev = (yo[3].copy(), yo[4].copy())
            if adapt and not conv:
                # the step size balances the residuals of the problem the iterations run on
                rp_i, rd_i, ps_i, ds_i = (r_prim, r_dual, ps, ds) if M is Mg else M.residuals(x, z_g, xi, y_f, y_g)
                cand, accept = rho_update(rho_bar, rp_i, rd_i, ps_i, ds_i, st)
                if accept:
                    # also at the last iteration: the returned rho_bar is the
                    # step size an SQP iteration hands to its next QP
                    rho_bar = cand
                    rho_changes.append((k, rho_bar))
                    if k < st.max_iter:  # the factorisation serves the iterations that follow
                        try:
                            cf = factor(rho_bar)
                            n_factor += 1
                        except np.linalg.LinAlgError:
                            status = FACTOR_BREAKDOWN
                            break
    return ADMMResult(*back(x, z_g, xi, y_f, y_g), rho_bar, k, status, r_prim, r_dual, n_factor, history,
                      rho_changes, pcg_iters)


def kkt_residuals(qp: StageQP, x, z_g, xi, y_f, y_g):
    """(r_prim, r_dual, prim_scale, dual_scale) of eq. admm:residuals in FP64."""
    return _QPMats(qp).residuals(np.asarray(x, float), np.asarray(z_g, float), np.asarray(xi, float),
                                 np.asarray(y_f, float), np.asarray(y_g, float))


def passes_gate(qp: StageQP, sol, eps_abs=1e-4, eps_rel=1e-4, mats=None) -> bool:
    """Stopping test of eq. admm:termination:slack re-evaluated in FP64."""
    M = mats or _QPMats(qp)
    rp, rd, ps, ds = M.residuals(*(np.asarray(sol[k], float) for k in ("x", "z_g", "xi", "y_f", "y_g")))
    return bool(rp <= eps_abs + eps_rel * ps and rd <= eps_abs + eps_rel * ds)
