"""GPU parity of the segmented substitutions (horizons of 128 stages and more):
the horizon is cut into four quarters whose chains run side by side and are
joined through the quarters' transfer blocks.  In exact arithmetic this is the
same solve of the Schur system, so the FP64 iterates follow the oracle's as
closely as the interleaved iteration does.

* Linear MPC (time-invariant, box-selection structure): fixed-rho FP64
  iterates against the oracle for horizons on both sides of the switch and
  with every residue of N + 1 mod 4 (quarter lengths); FP32 iterations over
  the FP64 factor converge to the oracle's polished optimum.
* Kinematic bicycle (time-varying data): fixed SQP x ADMM trajectory in FP64.
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
# 126, 127: interleaved; 128 .. 131: segmented with N + 1 = 1, 2, 3, 0 mod 4; 203: uneven quarters
HORIZONS = np.array([126, 127, 128, 129, 130, 131, 203])


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _sub(b, i, N):
    bi = b.subset([i])
    bi.N = int(N)
    return bi


def test_segmented_fixed_rho_iterates_fp64():
    b = random_lti(len(HORIZONS), N=int(HORIZONS.max()), seed=21)
    s = lti_solver(b, FP64, horizons=HORIZONS)
    out = s.solve(_settings(max_admm=60, k_check=0, adapt_rho=0))
    for i, N in enumerate(HORIZONS):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=60, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        assert got["x"].size == (N + 1) * b.n
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, (int(N), k, rel(got[k], getattr(ref, k)))
    s.close()


def test_segmented_rho_adaptation_and_refactorisation_fp64():
    """rho changes refactor inside the launch; the transfer blocks follow."""
    hz = HORIZONS[2:5]
    b = random_lti(len(hz), N=int(hz.max()), seed=22)
    s = lti_solver(b, FP64, horizons=hz)
    out = s.solve(_settings(max_admm=150, k_check=0, k_rho=25))
    for i, N in enumerate(hz):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=150, k_check=0, k_rho=25))
        got = per_instance(s, out, i)
        assert int(out["n_factor"][i]) == ref.n_factor, (int(N), int(out["n_factor"][i]), ref.n_factor)
        assert rel(got["x"], ref.x) < 1e-8, int(N)
    s.close()


def test_segmented_mixed_precision_converges():
    hz = HORIZONS[2:]
    b = random_lti(len(hz), N=int(hz.max()), seed=23)
    s = lti_solver(b, MIXED, horizons=hz)
    out = s.solve(_settings(eps_abs=1e-6, eps_rel=1e-6, max_admm=6000))
    for i, N in enumerate(hz):
        qp = lti_batch_qp(_sub(b, i, N), 0)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=80000))
        ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-8)
        assert ok
        got = per_instance(s, out, i)
        assert rel(got["x"], exact["x"]) < 1e-4, (int(N), rel(got["x"], exact["x"]))
    s.close()


def test_segmented_bicycle_trajectory_fp64():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(2, N=150, seed=3, first=40)
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
    s.set_bicycle(b)
    out = s.solve(_settings(max_sqp=6, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=6, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, rel(z, ref.z)
    s.close()
