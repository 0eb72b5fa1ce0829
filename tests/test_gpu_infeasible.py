"""GPU primal-infeasibility status (OCP_INFEASIBLE = 4) against the oracle.

* Double integrator started at 4.9 m with 3 m/s towards the 5 m wall: with
  |a| <= 1 it needs 4.5 m to stop, so the constraint set is empty.  Those
  instances end with status 4, the feasible ones converge; in FP64 status and
  iteration count equal the oracle's, FP32 iterations reach the same status.
* The random-LTI batch at the benchmark setting (eps 1e-4, cap 1000): on
  instances the oracle declares infeasible and on converged ones, the FP64
  status and iteration count equal the oracle's, with and without the box
  rescaling.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from oracle.scaling import box_scaling  # noqa: E402
from workloads import double_integrator, random_lti  # noqa: E402

FP64, MIXED = 0, 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_double_integrator_towards_the_wall(precision):
    b = double_integrator(4, N=40, seed=1)
    b.x0[0] = [4.9, 0.0, 3.0, 0.0]
    b.x0[2] = [-4.9, 1.0, -3.0, 0.5]
    s = lti_solver(b, precision)
    out = s.solve(_settings(eps_abs=1e-5, eps_rel=1e-5, max_admm=4000))
    st = ADMMSettings(eps_abs=1e-5, eps_rel=1e-5, max_iter=4000)
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), st)
        assert ref.status == (4 if i in (0, 2) else 0)
        assert int(out["status"][i]) == ref.status, (i, int(out["status"][i]), ref.status)
        if precision == FP64:
            assert int(out["admm_iters"][i]) == ref.iters, (i, int(out["admm_iters"][i]), ref.iters)
    s.close()


@pytest.mark.parametrize("scaled", [False, True], ids=["plain", "rescaled"])
def test_random_lti_batch_statuses(scaled):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = random_lti(1024, N=50, seed=2)
    s = OCPSolver(b.nx, b.nu, b.ng, np.full(b.batch, b.N), model=A.MODEL_LTI, precision=FP64)
    if scaled:
        s.set_scaling_box(0.6)
    s.set_lti(b.A, b.B, b.Qd, b.Rd, b.Qfd, b.G, b.lo, b.hi, b.x0)
    out = s.solve(_settings(eps_abs=1e-4, eps_rel=1e-4, max_admm=1000, k_check=25, k_rho=25))
    status = out["status"].cpu().numpy()
    iters = out["admm_iters"].cpu().numpy()
    st = ADMMSettings(eps_abs=1e-4, eps_rel=1e-4, max_iter=1000)
    # instances the oracle declares infeasible (checked there against a linear-programming feasibility test)
    # and converged ones
    for i in (76, 280, 463, 598, 621, 661, 908, 0, 1, 2, 3):
        qp = lti_batch_qp(b, i)
        ref = admm_solve(qp, st, scaling=box_scaling(qp, 0.6) if scaled else None)
        assert int(status[i]) == ref.status and int(iters[i]) == ref.iters, (i, int(status[i]), ref.status,
                                                                              int(iters[i]), ref.iters)
    assert (status == 4).sum() >= 5
    s.close()
