"""GPU parity of the PCG primal updates (ocp_set_linsolve): block-Jacobi
preconditioned CG on the Schur system from the current primal iterate,
stage-parallel on one wavefront per instance.

* A fixed number of CG iterations (tolerance 0) per ADMM iteration: the FP64
  iterates equal the oracle's ADMM with the same PCG (oracle.pcg), 1e-6
  after 20 ADMM iterations, on random linear MPC (box-selection structure)
  and on the bicycle SQP (time-varying blocks, L1-slack rows).  A truncated
  CG on the ill-conditioned Schur system (rho_f = 1e3 rho) amplifies the
  different summation order of its inner products (wavefront sums against
  NumPy's), ~1e-8 per solve; a wrong start, preconditioner or iteration
  count shows at 1e-2.  A converged inner solve (below) matches the direct
  iterates to 1e-8.
* A tight tolerance: the FP64 iterates equal the oracle's direct ADMM, 1e-8.
* FP32 iterations with convergence checks reach the polished optimum.
* Switching back to the direct solver gives the direct solve bit for bit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.adjoint import polish  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.models import BicycleOCP  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from oracle.sqp import SQPSettings, sqp_solve  # noqa: E402
from workloads import bicycle_batch, random_lti  # noqa: E402

FP64, MIXED = 0, 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def test_pcg_fixed_count_iterates_lti_fp64():
    b = random_lti(3, N=20, seed=41)
    s = lti_solver(b, FP64)
    s.set_linsolve(True, max_iter=8, tol=0.0)
    out = s.solve(_settings(max_admm=20, k_check=0, adapt_rho=0))
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), ADMMSettings(max_iter=20, k_check=0, adapt_rho=False,
                                                          linsolve="pcg", pcg_max_iter=8, pcg_tol=0.0))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-6, (i, k, rel(got[k], getattr(ref, k)))
    s.close()


def test_pcg_fixed_count_bicycle_sqp_fp64():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(2, N=30, seed=3, first=7)
    o = b.stage_off[1]
    b.x0[1, :2] = b.ref[o, :2] + 2.6 * b.normal[o]  # lateral rows with L1 slack
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
    s.set_linsolve(True, max_iter=6, tol=0.0)
    s.set_bicycle(b)
    out = s.solve(_settings(max_sqp=2, max_admm=20, k_check=0, adapt_rho=0, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=2, fixed_iters=True),
                        admm=ADMMSettings(max_iter=20, k_check=0, adapt_rho=False, linsolve="pcg",
                                          pcg_max_iter=6, pcg_tol=0.0))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-6, (i, rel(z, ref.z))
    s.close()


def test_pcg_tight_tolerance_equals_direct_fp64():
    b = random_lti(2, N=30, seed=42)
    s = lti_solver(b, FP64)
    s.set_linsolve(True, max_iter=600, tol=1e-13)
    out = s.solve(_settings(max_admm=150, k_check=0, k_rho=25))
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), ADMMSettings(max_iter=150, k_check=0, k_rho=25))
        got = per_instance(s, out, i)
        assert int(out["n_factor"][i]) == ref.n_factor
        assert rel(got["x"], ref.x) < 1e-8, (i, rel(got["x"], ref.x))
    s.close()


def test_pcg_fp32_converges_and_direct_is_restored():
    b = random_lti(4, N=20, seed=43)
    s = lti_solver(b, MIXED)
    st = _settings(eps_abs=1e-4, eps_rel=1e-4, max_admm=4000)
    direct = s.solve(st)
    direct = {k: v.clone() for k, v in direct.items()}
    s.set_linsolve(True, max_iter=30, tol=1e-5)
    out = s.solve(st)
    for i in range(b.batch):
        if int(direct["status"][i]) != 0:
            continue
        assert int(out["status"][i]) == 0, i
        qp = lti_batch_qp(b, i)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=80000))
        ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-8)
        assert ok
        assert rel(per_instance(s, out, i)["x"], exact["x"]) < 2e-3, i
    s.set_linsolve(False)
    again = s.solve(st)
    for k in ("x", "y_g", "status", "admm_iters"):
        assert bool((again[k] == direct[k]).all()), k
    s.close()
