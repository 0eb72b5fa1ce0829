"""GPU parity on stage-wise QPs with L2-slack rows (Sec. "Slack update"; the
smoothed projection of the slack ADMM) and their adjoint (eq.
bwd:slack_reduced_system), through the general QP interface (ocp_set_qp,
time-varying layout).

A double integrator whose position rows carry an L2 slack (gamma2 = 4) and a
tightened box, with starts outside it, so that the first stages hold nonzero
slack on the active rows.

* FP64, fixed rho and iteration count: iterates equal the oracle's (1e-9).
* Adjoint at a tight FP64 solve: the active set equals the oracle's at its
  polished optimum (same rule and tolerance), eta and the QP-data gradients
  match the oracle's dense KKT solve with the -1/gamma2 slack diagonal (1e-6),
  and so does the gradient w.r.t. the slack weight, under both launch shapes.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import rel  # noqa: E402
from oracle.adjoint import active_set, adjoint_dense, polish, qp_vjp  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.qp import SOFT_L2, lti_batch_qp  # noqa: E402
from workloads import double_integrator  # noqa: E402

FP64 = 0
GAMMA2 = 4.0


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _qps():
    b = double_integrator(2, N=24, seed=3)
    b.x0[0, :2] = [1.8, -1.6]
    b.x0[1, :2] = [-1.5, 1.7]
    qps = []
    for i in range(2):
        qp = lti_batch_qp(b, i)
        kinds = np.zeros(qp.ng, dtype=np.int64)
        kinds[:2] = SOFT_L2
        qp.soft = kinds
        qp.gamma2 = GAMMA2
        qp.lo[:, :2] = -1.0
        qp.hi[:, :2] = 1.0
        qps.append(qp)
    return qps


def _solver(qps, precision=FP64):
    """Stage-concatenated general QP (dynamics blocks padded at slot N)."""
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    q0 = qps[0]
    nx, n = q0.nx, q0.n
    pad = lambda a: np.concatenate([a, np.zeros((1,) + a.shape[1:])])
    D = np.concatenate([q.D for q in qps])
    Am = np.concatenate([pad(q.Am) for q in qps])
    Ap = np.concatenate([pad(q.Ap) for q in qps])
    bb = np.concatenate([pad(q.b) for q in qps])
    qv = np.concatenate([q.q for q in qps])
    G = np.concatenate([q.G for q in qps])
    lo = np.concatenate([q.lo for q in qps])
    hi = np.concatenate([q.hi for q in qps])
    x0 = np.stack([q.x_init for q in qps])
    s = OCPSolver(nx, q0.nu, q0.ng, np.array([q.N for q in qps]), model=A.MODEL_QP, precision=precision)
    s.set_qp(D, Am, Ap, x0, G, lo, hi, q=qv, b=bb, soft=q0.soft.astype(np.uint8), gamma2=GAMMA2)
    assert D.shape[1:] == (n, n)
    return s


def test_l2_slack_fixed_rho_iterates_fp64():
    qps = _qps()
    s = _solver(qps)
    out = s.solve(_settings(max_admm=80, k_check=0, adapt_rho=0))
    for i, qp in enumerate(qps):
        ref = admm_solve(qp, ADMMSettings(max_iter=80, k_check=0, adapt_rho=False))
        assert np.count_nonzero(ref.xi) > 0
        for k in ("x", "xi", "z_g", "y_f", "y_g"):
            got = s.split(out[k], i).cpu().numpy().reshape(-1)
            assert rel(got, getattr(ref, k)) < 1e-9, (i, k, rel(got, getattr(ref, k)))
    s.close()


@pytest.mark.parametrize("slack_loss", [False, True], ids=["x_loss", "x_and_slack_loss"])
@pytest.mark.parametrize("seg", [None, 15], ids=["stagewise", "chunked"])
def test_l2_slack_adjoint_matches_oracle_dense_solve(seg, slack_loss):
    """slack_loss: a loss term on the slacks too (eq. bwd:slack_reduced_system
    right-hand side, eta_y and eta_xi of eq. bwd:slack:eta_xi_yg)."""
    qps = _qps()
    s = _solver(qps)
    if seg is not None:
        s.set_segmented(seg)
    s.solve(_settings(eps_abs=1e-10, eps_rel=1e-10, max_admm=40000))
    dl = torch.as_tensor(np.random.default_rng(8).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
    dxi = (torch.as_tensor(np.random.default_rng(10).standard_normal((s.S, s.ng)), dtype=torch.float64,
                           device="cuda") if slack_loss else None)
    g = s.adjoint(dl, _settings(eps_active=1e-6), dL_dxi=dxi)
    for i, qp in enumerate(qps):
        r = admm_solve(qp, ADMMSettings(eps_abs=1e-12, eps_rel=1e-12, max_iter=400000))
        ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
        assert ok, i
        lower, upper = active_set(qp, sol["x"], sol["y_g"], xi=sol["xi"], eps_solve=1e-6)
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        assert np.array_equal(act < 0, lower) and np.array_equal(act > 0, upper), i
        assert np.any(((lower | upper) & (qp.soft_rows() == SOFT_L2)))
        dli = s.split(dl, i).cpu().numpy().reshape(-1)
        dxii = s.split(dxi, i).cpu().numpy().reshape(-1) if slack_loss else None
        ex, ef, eg = adjoint_dense(qp, sol["x"], dli, lower, upper, dL_dxi=dxii, xi=sol["xi"])
        assert rel(s.split(g["eta_x"], i).cpu().numpy().reshape(-1), ex) < 1e-6, i
        assert rel(s.split(g["eta_g"], i).cpu().numpy().reshape(-1), eg) < 1e-6, i
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper, xi=sol["xi"], dL_dxi=dxii)
        assert rel(s.split(g["eta_xi"], i).cpu().numpy().reshape(-1), qg["eta_xi"].reshape(-1)) < 1e-6, i
        assert abs(float(g["d_gamma2"][i]) - qg["d_gamma2"]) <= 1e-6 * max(1.0, abs(qg["d_gamma2"])), i
        flat = lambda a: np.asarray(a).reshape(-1)
        assert rel(flat(g["d_x_init"][i].cpu().numpy()), flat(qg["d_x_init"])) < 1e-6, i
        for k in ("d_q", "d_lo", "d_hi"):
            assert rel(flat(s.split(g[k], i).cpu().numpy()), flat(qg[k])) < 1e-6, (i, k)
    s.close()
