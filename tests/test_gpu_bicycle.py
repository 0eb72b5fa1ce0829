"""GPU parity of the SQP path (Algorithm 1) on the kinematic-bicycle
workload: convexification at the iterate, warm-started ADMM, backtracking
line search, stopping quantities of eq. sqp_stop.

* Fixed SQP x ADMM iteration counts in FP64: the GPU follows the oracle's
  trajectory (identical algorithm; only rounding order differs).
* Run to convergence: the GPU and the oracle reach the same NLP KKT point.
* FP32 ADMM iterations: the final iterate stays within the FP32 tolerance of
  the oracle's and its NLP KKT residuals are reported.
* Ragged horizons in one batch.
* Horizons past the line search's 512-stage chunks (merit sums, step and
  stopping quantities spread over one wavefront per chunk) follow the
  oracle's trajectory in FP64.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import rel  # noqa: E402
from oracle.admm import ADMMSettings  # noqa: E402
from oracle.models import BicycleOCP  # noqa: E402
from oracle.sqp import SQPSettings, sqp_solve  # noqa: E402
from workloads import bicycle_batch, bicycle_long_and_ragged  # noqa: E402

FP64, MIXED = 0, 1


def _solver(batch, precision):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    s = OCPSolver(4, 2, 3, batch.horizons, model=A.MODEL_BICYCLE, precision=precision)
    s.set_bicycle(batch)
    return s


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def test_fixed_iterations_follow_the_oracle_fp64():
    b = bicycle_batch(4, N=40, seed=3)
    s = _solver(b, FP64)
    out = s.solve(_settings(max_sqp=10, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=10, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, rel(z, ref.z)
        kkt = out["sqp_kkt"][i].cpu().numpy()
        assert abs(kkt[0] - ref.stop["stationarity"]) < 1e-7 * max(1, ref.stop["stationarity"])
        assert abs(kkt[1] - ref.stop["eq"]) < 1e-9 + 1e-7 * ref.stop["eq"]
        assert int(out["sqp_iters"][i]) == 10


def test_chunked_line_search_follows_the_oracle_fp64():
    """Horizons 1183, 610 and 505: three, two and one 512-stage chunks."""
    _, rag = bicycle_long_and_ragged(seed=13, long_N=16, ragged=3, n_lo=480, n_hi=1200)
    assert list(rag.horizons) == [1183, 610, 505]
    s = _solver(rag, FP64)
    out = s.solve(_settings(max_sqp=3, max_admm=25, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(rag.batch):
        ref = sqp_solve(BicycleOCP(rag, i), SQPSettings(max_sqp=3, fixed_iters=True),
                        admm=ADMMSettings(max_iter=25, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, (i, rel(z, ref.z))
        kkt = out["sqp_kkt"][i].cpu().numpy()
        assert abs(kkt[0] - ref.stop["stationarity"]) < 1e-7 * max(1, ref.stop["stationarity"]), (i, kkt, ref.stop)
        assert abs(kkt[1] - ref.stop["eq"]) < 1e-9 + 1e-7 * ref.stop["eq"], (i, kkt, ref.stop)
        assert abs(kkt[2] - ref.stop["ineq"]) < 1e-9 + 1e-7 * ref.stop["ineq"], (i, kkt, ref.stop)
        assert int(out["sqp_iters"][i]) == 3


def test_converged_sqp_reaches_the_oracle_kkt_point():
    b = bicycle_batch(3, N=40, seed=3, first=10)
    s = _solver(b, FP64)
    tight = dict(eps_abs=1e-10, eps_rel=1e-10, max_admm=20000, k_check=25)
    out = s.solve(_settings(max_sqp=25, fixed_sqp=1, **tight))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=25, fixed_iters=True),
                        admm=ADMMSettings(eps_abs=1e-10, eps_rel=1e-10, max_iter=20000))
        z = s.split(out["x"], i).cpu().numpy()
        assert max(ref.stop.values()) < 1e-6
        assert rel(z, ref.z) < 1e-6
        assert float(out["sqp_kkt"][i].max()) < 1e-6


def test_mixed_precision_sqp_close_to_oracle():
    b = bicycle_batch(4, N=40, seed=3)
    s = _solver(b, MIXED)
    out = s.solve(_settings(max_sqp=10, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=10, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-3
        assert np.all(np.isfinite(out["sqp_kkt"][i].cpu().numpy()))


def test_ragged_bicycle_batch():
    _, rag = bicycle_long_and_ragged(seed=5, long_N=64, ragged=6, n_lo=32, n_hi=96)
    s = _solver(rag, FP64)
    out = s.solve(_settings(max_sqp=4, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(rag.batch):
        ref = sqp_solve(BicycleOCP(rag, i), SQPSettings(max_sqp=4, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert z.shape == (rag.horizons[i] + 1, 6)
        assert rel(z, ref.z) < 1e-8


@pytest.mark.parametrize("seg", [None, 15], ids=["stagewise", "chunked"])
def test_trapezoidal_rule_follows_the_oracle_fp64(seg):
    """The trapezoidal discretisation (Remark A1): linearisation, line-search
    merit and stopping quantities all evaluate the same rule as the oracle."""
    b = bicycle_batch(3, N=40, seed=3, first=20)
    b.integrator = 1
    s = _solver(b, FP64)
    if seg is not None:
        s.set_segmented(seg)
    out = s.solve(_settings(max_sqp=8, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=8, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, rel(z, ref.z)
        kkt = out["sqp_kkt"][i].cpu().numpy()
        assert abs(kkt[0] - ref.stop["stationarity"]) < 1e-7 * max(1, ref.stop["stationarity"])
        assert abs(kkt[1] - ref.stop["eq"]) < 1e-9 + 1e-7 * ref.stop["eq"]
    s.close()


def test_unknown_discretisation_rule_is_rejected():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(1, N=10, seed=3)
    b.integrator = 2
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
    with pytest.raises(A.OCPError) as e:
        s.set_bicycle(b)
    assert e.value.code == A.OCP_E_ARG
    s.close()
