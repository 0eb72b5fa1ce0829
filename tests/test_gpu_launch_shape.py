"""GPU parity under every launch shape the scheduler can pick: the
segmented substitutions forced on short horizons, and kept off on long
ones, give the oracle's FP64 iterates; the autotuner returns one of its
candidates and the solves that follow stay correct."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve, passes_gate  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from workloads import random_lti  # noqa: E402

FP64, MIXED = 0, 1
NEVER = 2**31 - 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _sub(b, i, N):
    bi = b.subset([i])
    bi.N = int(N)
    return bi


@pytest.mark.parametrize("seg_min_n,after,horizons", [(15, NEVER, [15, 16, 17, 18, 50]), (NEVER, NEVER, [130, 203]),
                                                     (NEVER, 30, [15, 16, 17, 18, 50, 130])])
def test_forced_launch_shape_fixed_rho_iterates_fp64(seg_min_n, after, horizons):
    """after = 30: every instance switches to the segmented sweeps at iteration 30 (the tail switch)."""
    hz = np.array(horizons)
    b = random_lti(len(hz), N=int(hz.max()), seed=31)
    s = lti_solver(b, FP64, horizons=hz)
    s.set_segmented(seg_min_n)
    s.set_segmented_after(after)
    out = s.solve(_settings(max_admm=60, k_check=0, adapt_rho=0))
    for i, N in enumerate(hz):
        ref = admm_solve(lti_batch_qp(_sub(b, i, N), 0), ADMMSettings(max_iter=60, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, (int(N), k)
    s.close()


def test_autotune_picks_a_candidate_and_solves_stay_correct():
    b = random_lti(64, N=50, seed=2)
    for precision in (MIXED, FP64):
        s = lti_solver(b, precision)
        chosen = s.autotune(_settings(), reps=1)
        cand = [(15, NEVER, 0), (128, NEVER, 0), (NEVER, NEVER, 0), (128, 150, 0), (128, 300, 0), (128, 500, 0)]
        if precision == MIXED:
            cand += [(128, NEVER, 200), (128, NEVER, 300), (128, 150, 200)]
        assert chosen in cand, chosen
        out = s.solve(_settings())
        st = out["status"].cpu().numpy()
        assert (st == 0).mean() >= 0.85
        for i in np.flatnonzero(st == 0)[:16]:
            assert passes_gate(lti_batch_qp(b, int(i)), per_instance(s, out, int(i))), int(i)
        s.close()
