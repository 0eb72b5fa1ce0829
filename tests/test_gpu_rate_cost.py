"""GPU parity with a control-rate cost (Sec. "Problem formulation": the cost
couples consecutive stages, E_t != 0, which makes the Hessian block
tridiagonal) through the general QP interface: the Schur blocks Theta_t and
Phi_t carry D_t and E_t, the dual residual and the adjoint's H e_x the
cross-stage terms.

A double integrator with cost w/2 ||u_{t+1} - u_t||^2 added (w = 2): D_t
gains w on the control block of stages t and t+1 (interior stages twice),
E_t (block (t+1, t)) holds -w there.

* FP64, fixed rho and iteration count: iterates equal the oracle's (1e-9).
* Adjoint at a tight FP64 solve: eta and the QP-data gradients match the
  oracle's dense KKT solve (1e-6).
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import rel  # noqa: E402
from oracle.adjoint import active_set, adjoint_dense, polish, qp_vjp  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from workloads import double_integrator  # noqa: E402

FP64 = 0
W_RATE = 2.0


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _qps(N=30):
    b = double_integrator(3, N=N, seed=4)
    qps = []
    for i in range(3):
        qp = lti_batch_qp(b, i)
        nx, n = qp.nx, qp.n
        for t in range(N):
            qp.D[t, nx:, nx:] += W_RATE * np.eye(n - nx)
            qp.D[t + 1, nx:, nx:] += W_RATE * np.eye(n - nx)
            qp.E[t, nx:, nx:] = -W_RATE * np.eye(n - nx)
        qps.append(qp)
    return qps


def _solver(qps):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    q0 = qps[0]
    pad = lambda a: np.concatenate([a, np.zeros((1,) + a.shape[1:])])
    cat = lambda f, p=False: np.concatenate([pad(getattr(q, f)) if p else getattr(q, f) for q in qps])
    s = OCPSolver(q0.nx, q0.nu, q0.ng, np.array([q.N for q in qps]), model=A.MODEL_QP, precision=FP64)
    s.set_qp(cat("D"), cat("Am", True), cat("Ap", True), np.stack([q.x_init for q in qps]), cat("G"), cat("lo"),
             cat("hi"), E=cat("E", True), q=cat("q"), b=cat("b", True))
    return s


@pytest.mark.parametrize("seg", [None, 15], ids=["stagewise", "chunked"])
def test_rate_cost_fixed_rho_iterates_fp64(seg):
    qps = _qps()
    s = _solver(qps)
    if seg is not None:
        s.set_segmented(seg)
    out = s.solve(_settings(max_admm=80, k_check=0, adapt_rho=0))
    for i, qp in enumerate(qps):
        ref = admm_solve(qp, ADMMSettings(max_iter=80, k_check=0, adapt_rho=False))
        for k in ("x", "z_g", "y_f", "y_g"):
            got = s.split(out[k], i).cpu().numpy().reshape(-1)
            assert rel(got, getattr(ref, k)) < 1e-9, (i, k, rel(got, getattr(ref, k)))
    s.close()


def test_rate_cost_adjoint_matches_oracle_dense_solve():
    qps = _qps()
    s = _solver(qps)
    s.solve(_settings(eps_abs=1e-10, eps_rel=1e-10, max_admm=40000))
    dl = torch.as_tensor(np.random.default_rng(9).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
    g = s.adjoint(dl, _settings(eps_active=1e-6))
    for i, qp in enumerate(qps):
        r = admm_solve(qp, ADMMSettings(eps_abs=1e-12, eps_rel=1e-12, max_iter=400000))
        ok, sol = polish(qp, r.x, r.y_g, eps_solve=1e-8)
        assert ok, i
        lower, upper = active_set(qp, sol["x"], sol["y_g"], eps_solve=1e-6)
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        assert np.array_equal(act < 0, lower) and np.array_equal(act > 0, upper), i
        dli = s.split(dl, i).cpu().numpy().reshape(-1)
        ex, ef, eg = adjoint_dense(qp, sol["x"], dli, lower, upper)
        assert rel(s.split(g["eta_x"], i).cpu().numpy().reshape(-1), ex) < 1e-6, i
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper)
        flat = lambda a: np.asarray(a).reshape(-1)
        for k in ("d_q", "d_lo", "d_hi"):
            assert rel(flat(s.split(g[k], i).cpu().numpy()), flat(qg[k])) < 1e-6, (i, k)
    s.close()
