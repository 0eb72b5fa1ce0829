"""GPU parity of the implicit-differentiation adjoint (Algorithm 2) on the
kinematic bicycle: time-varying dynamics blocks and the lateral-offset rows
with an L1 slack (rows whose slack is nonzero carry a fixed multiplier and
leave the active set).  One SQP iteration from the initial guess, so the QP
the adjoint differentiates is the oracle's convexification at that guess.

* FP64: the active set equals the oracle's at its polished optimum (same
  rule and tolerance), and eta
  and the QP-data gradients match the oracle's dense KKT solve (1e-6).
* FP32 ADMM iterations: eta matches the dense solve on the active set the
  GPU identified (2e-3; the adjoint itself runs in FP64 over that set).
Both launch shapes: stage-wise and, with the switch lowered, chunked
factorisation and segmented substitutions.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import rel  # noqa: E402
from oracle.adjoint import active_set, adjoint_dense, polish, qp_vjp  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.models import BicycleOCP  # noqa: E402
from workloads import bicycle_batch  # noqa: E402

FP64, MIXED = 0, 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


@pytest.mark.parametrize("slack_loss", [False, True], ids=["x_loss", "x_and_slack_loss"])
@pytest.mark.parametrize("seg", [None, 15], ids=["stagewise", "chunked"])
@pytest.mark.parametrize("precision", [FP64, MIXED])
def test_bicycle_adjoint_matches_oracle_dense_solve(precision, seg, slack_loss):
    """slack_loss: the loss also has a term on the slacks (dL/dxi, eq.
    loss_gradient with the slack block): the L1 rows with nonzero slack pass
    it to the right-hand side and to their bound; eta_xi and dL/dgamma1 are
    compared too.  The adjoint runs in FP64 in both precisions and the
    linearisation point is the shared initial guess, so the oracle's dense
    solve at the GPU's active set is matched to 1e-6 in both."""
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(3, N=40, seed=6)
    # instance 1 starts 2.6 m off the reference (track half-width 2): the first
    # ten lateral rows then carry nonzero L1 slack and leave the active set
    o = b.stage_off[1]
    b.x0[1, :2] = b.ref[o, :2] + 2.6 * b.normal[o]
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=precision)
    s.set_bicycle(b)
    if seg is not None:
        s.set_segmented(seg)
    eps = 1e-10 if precision == FP64 else 1e-6
    s.solve(_settings(max_sqp=1, fixed_sqp=1, eps_abs=eps, eps_rel=eps, max_admm=20000))
    dl = torch.as_tensor(np.random.default_rng(7).standard_normal((s.S, 6)), dtype=torch.float64, device="cuda")
    dxi = (torch.as_tensor(np.random.default_rng(9).standard_normal((s.S, 3)), dtype=torch.float64, device="cuda")
           if slack_loss else None)
    g = s.adjoint(dl, _settings(eps_active=1e-6), dL_dxi=dxi)
    for i in range(b.batch):
        ocp = BicycleOCP(b, i)
        qp = ocp.convexify(ocp.initial_guess())
        r = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=200000))
        ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-8)
        assert ok, i
        if i == 1:
            assert np.count_nonzero(r.xi) > 0
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        lower, upper = act < 0, act > 0
        if precision == FP64:
            # the same identification rule and tolerance as the GPU's
            # (eps_active = 1e-6): weakly active rows (zero multiplier, value
            # within the tolerance of its bound) count on both sides
            ref_lo, ref_up = active_set(qp, sol["x"], sol["y_g"], xi=r.xi, eps_solve=1e-6)
            assert np.array_equal(lower, ref_lo) and np.array_equal(upper, ref_up), i
        dli = s.split(dl, i).cpu().numpy().reshape(-1)
        # which L1 rows hold a nonzero slack (they leave the active set): the
        # oracle's converged ADMM slacks of the same QP
        xi_gpu = r.xi
        dxii = s.split(dxi, i).cpu().numpy().reshape(-1) if slack_loss else None
        ex, ef, eg = adjoint_dense(qp, sol["x"], dli, lower, upper, dL_dxi=dxii, xi=xi_gpu)
        tol = 1e-6
        assert rel(s.split(g["eta_x"], i).cpu().numpy().reshape(-1), ex) < tol, i
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper, xi=xi_gpu, dL_dxi=dxii)
        flat = lambda a: np.asarray(a).reshape(-1)
        assert rel(flat(g["d_x_init"][i].cpu().numpy()), flat(qg["d_x_init"])) < tol, i
        for k in ("d_q", "d_lo", "d_hi", "eta_xi"):
            assert rel(flat(s.split(g[k], i).cpu().numpy()), flat(qg[k])) < tol, (i, k)
        assert rel(flat(s.split(g["eta_g"], i).cpu().numpy()), flat(eg)) < tol, i
        assert abs(float(g["d_gamma1"][i]) - qg["d_gamma1"]) <= tol * max(1.0, abs(qg["d_gamma1"])), i
        if i == 1:
            assert abs(qg["d_gamma1"]) > 1e-6
    s.close()
