"""GPU parity of the chunked factorisation of long horizons: the horizon is cut
into five chunks, chunks 1..3 are first summarised as functions of their
entering Schur state (Woodbury identity), the entering states are chained
through the summaries, and every chunk is then factored from its true entering
state.  The blocks equal those of the stage-by-stage recurrence up to
rounding, so the FP64 iterates follow the oracle's as closely as before.

The switch horizon is lowered with ``set_segmented`` so that short horizons
(chunks of three or four stages, every residue of N + 1 mod 5) take the
chunked path; it covers the time-invariant products (random LTI, double
integrator) and the time-varying stage loads (kinematic bicycle), both
precisions' factor forms, and refactorisation after rho changes.
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
from workloads import bicycle_batch, double_integrator, random_lti  # noqa: E402

FP64, MIXED = 0, 1
# shortest chunked horizon (15) and the next four residues of N + 1 mod 5, two longer ones
HORIZONS = np.array([15, 16, 17, 18, 19, 57, 130])


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _sub(b, i, N):
    bi = b.subset([i])
    bi.N = int(N)
    return bi


def test_chunked_fixed_rho_iterates_fp64():
    b = random_lti(len(HORIZONS), N=int(HORIZONS.max()), seed=31)
    s = lti_solver(b, FP64, horizons=HORIZONS)
    s.set_segmented(15)
    out = s.solve(_settings(max_admm=60, k_check=0, adapt_rho=0))
    for i, N in enumerate(HORIZONS):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=60, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, (int(N), k, rel(got[k], getattr(ref, k)))
    s.close()


def test_chunked_matches_stage_recurrence_fp64():
    """Chunked and stage-by-stage factorisations give the same iterates."""
    b = random_lti(len(HORIZONS), N=int(HORIZONS.max()), seed=32)
    st = _settings(max_admm=40, k_check=0, adapt_rho=0)
    outs = []
    for seg in (15, 1 << 30):
        s = lti_solver(b, FP64, horizons=HORIZONS)
        s.set_segmented(seg)
        o = s.solve(st)
        outs.append([per_instance(s, o, i)["x"] for i in range(len(HORIZONS))])
        s.close()
    for i, N in enumerate(HORIZONS):
        assert rel(outs[0][i], outs[1][i]) < 1e-11, (int(N), rel(outs[0][i], outs[1][i]))


def test_chunked_refactorisation_fp64():
    hz = np.array([16, 40, 131])
    b = random_lti(len(hz), N=int(hz.max()), seed=33)
    s = lti_solver(b, FP64, horizons=hz)
    s.set_segmented(15)
    out = s.solve(_settings(max_admm=150, k_check=0, k_rho=25))
    for i, N in enumerate(hz):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=150, k_check=0, k_rho=25))
        got = per_instance(s, out, i)
        assert int(out["n_factor"][i]) == ref.n_factor, (int(N), int(out["n_factor"][i]), ref.n_factor)
        assert rel(got["x"], ref.x) < 1e-8, int(N)
    s.close()


def test_chunked_mixed_precision_converges():
    b = random_lti(len(HORIZONS), N=int(HORIZONS.max()), seed=34)
    s = lti_solver(b, MIXED, horizons=HORIZONS)
    s.set_segmented(15)
    out = s.solve(_settings(eps_abs=1e-6, eps_rel=1e-6, max_admm=6000))
    for i, N in enumerate(HORIZONS):
        qp = lti_batch_qp(_sub(b, i, N), 0)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=80000))
        ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-8)
        assert ok
        got = per_instance(s, out, i)
        assert rel(got["x"], exact["x"]) < 1e-4, (int(N), rel(got["x"], exact["x"]))
    s.close()


def test_chunked_double_integrator_fp64():
    hz = np.array([15, 99, 200])
    b = double_integrator(len(hz), N=int(hz.max()), seed=1)
    s = lti_solver(b, FP64, horizons=hz)
    s.set_segmented(15)
    out = s.solve(_settings(max_admm=200, k_check=0, adapt_rho=0))
    for i, N in enumerate(hz):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=200, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        assert rel(got["x"], ref.x) < 1e-10, (int(N), rel(got["x"], ref.x))
    s.close()


@pytest.mark.parametrize("N", [19, 64])
def test_chunked_bicycle_trajectory_fp64(N):
    """Time-varying blocks: the stage loads of every chunk start at its own stage."""
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    b = bicycle_batch(2, N=N, seed=4, first=10)
    s = OCPSolver(4, 2, 3, b.horizons, model=A.MODEL_BICYCLE, precision=FP64)
    s.set_bicycle(b)
    s.set_segmented(15)
    out = s.solve(_settings(max_sqp=5, max_admm=50, k_check=0, k_rho=25, fixed_sqp=1))
    for i in range(b.batch):
        ref = sqp_solve(BicycleOCP(b, i), SQPSettings(max_sqp=5, fixed_iters=True),
                        admm=ADMMSettings(max_iter=50, k_check=0, k_rho=25))
        z = s.split(out["x"], i).cpu().numpy()
        assert rel(z, ref.z) < 1e-8, rel(z, ref.z)
    s.close()
