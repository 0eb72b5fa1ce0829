"""GPU parity of the ADMM path (Algorithm 3) on linear-quadratic OCPs against
the FP64 oracle.

* Fixed rho, fixed iteration count: the FP64 GPU path reproduces the oracle's
  iterates (same arithmetic, different rounding order).
* Converged solves: the FP64 path matches the oracle's polished optimum to
  1e-6 relative, the FP32-iteration / FP64-factor path to 1e-4.
* Ragged horizons, the shortest horizon N = 1, and the per-instance status
  codes (non-finite data, factor breakdown, iteration limit).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve, passes_gate  # noqa: E402
from oracle.adjoint import polish  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from workloads import double_integrator, random_lti  # noqa: E402

FP64, MIXED = 0, 1


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def test_double_integrator_fixed_rho_iterates_match_oracle():
    b = double_integrator(4)
    s = lti_solver(b, FP64)
    out = s.solve(_settings(max_admm=200, k_check=0, adapt_rho=0))
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), ADMMSettings(max_iter=200, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-10, k
        assert int(out["status"][i]) == 1 and int(out["admm_iters"][i]) == 200
        assert abs(float(out["r_prim"][i]) - ref.r_prim) < 1e-9 * max(1, ref.r_prim)


def test_double_integrator_mixed_precision_iterates():
    b = double_integrator(4)
    s = lti_solver(b, MIXED)
    out = s.solve(_settings(max_admm=200, k_check=0, adapt_rho=0))
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), ADMMSettings(max_iter=200, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-4, k


def test_random_lti_fixed_rho_iterates_match_oracle():
    b = random_lti(8, N=50, seed=2)
    s = lti_solver(b, FP64)
    out = s.solve(_settings(max_admm=60, k_check=0, adapt_rho=0))
    for i in range(b.batch):
        ref = admm_solve(lti_batch_qp(b, i), ADMMSettings(max_iter=60, k_check=0, adapt_rho=False))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, k


@pytest.mark.parametrize("precision,tol,eps", [(FP64, 1e-6, 1e-9), (MIXED, 1e-4, 1e-6)])
def test_random_lti_converges_to_the_qp_optimum(precision, tol, eps):
    b = random_lti(16, N=50, seed=2)
    s = lti_solver(b, precision)
    out = s.solve(_settings(eps_abs=eps, eps_rel=eps, max_admm=4000))
    st = out["status"].cpu().numpy()
    for i in range(b.batch):
        qp = lti_batch_qp(b, i)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=50000))
        ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-8)
        assert ok
        got = per_instance(s, out, i)
        if precision == FP64:
            assert st[i] == 0
        # primal and dual solutions at the stated tolerance (1e-6 relative in
        # FP64, 1e-4 in FP32; measured: 3e-8 and 3e-5)
        assert rel(got["x"], exact["x"]) < tol
        assert rel(got["y_f"], exact["y_f"]) < tol
        assert rel(got["y_g"], exact["y_g"]) < tol


def test_random_lti_gate_at_1e4_matches_oracle_solution():
    """The metric's setting: eps = 1e-4, FP64 re-evaluated gate."""
    b = random_lti(16, N=50, seed=2)
    for precision in (FP64, MIXED):
        s = lti_solver(b, precision)
        out = s.solve(_settings())
        st = out["status"].cpu().numpy()
        for i in range(b.batch):
            qp = lti_batch_qp(b, i)
            got = per_instance(s, out, i)
            if st[i] == 0:
                assert passes_gate(qp, got)
            ref = admm_solve(qp, ADMMSettings())
            assert ref.status == 0
            ok, exact = polish(qp, ref.x, ref.y_g, eps_solve=1e-6)
            # both approximate the same optimum to the tolerance's accuracy
            assert rel(got["x"], ref.x) < 5e-3
        assert (st == 0).mean() >= 0.9


def test_ragged_horizons_and_shortest_horizon():
    base = random_lti(6, N=40, seed=12)
    hz = np.array([40, 1, 17, 33, 2, 40])
    s = lti_solver(base, FP64, horizons=hz)
    out = s.solve(_settings(eps_abs=1e-9, eps_rel=1e-9, max_admm=4000))
    for i in range(base.batch):
        bi = base.subset([i])
        bi.N = int(hz[i])
        qp = lti_batch_qp(bi, 0)
        ref = admm_solve(qp, ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=50000))
        got = per_instance(s, out, i)
        assert got["x"].size == (hz[i] + 1) * base.n
        assert rel(got["x"], ref.x) < 1e-6


def test_status_codes():
    b = random_lti(4, N=20, seed=13)
    b.x0[1, 0] = np.nan          # non-finite data
    b.Rd[2, :] = -1e4            # indefinite cost: the Schur factor breaks down
    s = lti_solver(b, FP64)
    out = s.solve(_settings())
    st = out["status"].cpu().numpy()
    assert st[0] == 0 and st[3] == 0
    assert st[1] == 2
    assert st[2] == 3
    out = s.solve(_settings(max_admm=1))
    assert out["status"].cpu().numpy()[0] == 1 and int(out["admm_iters"][0]) == 1


def test_deterministic_across_runs():
    b = random_lti(8, N=50, seed=2)
    s = lti_solver(b, MIXED)
    o1 = {k: v.clone() for k, v in s.solve(_settings()).items()}
    o2 = s.solve(_settings())
    for k in ("x", "y_f", "y_g", "z_g"):
        assert np.array_equal(o1[k].cpu().numpy(), o2[k].cpu().numpy())


def test_kernel_timing_counts_launches():
    """The library's event timing sees the launches of a solve: the
    per-solve initialisation and one persistent solve launch."""
    b = random_lti(8, N=20, seed=2)
    s = lti_solver(b, MIXED)
    s.profile(True)
    st = _settings(max_admm=100, k_check=25, k_rho=25)
    s.solve(st)
    t = s.profile_read()
    assert t["solve"][1] == 1 and t["other"][1] == 1
    assert all(ms >= 0.0 for ms, _ in t.values()) and t["solve"][0] > 0.0
    s.profile(False)
    s.solve(st)
    t2 = s.profile_read()
    assert all(c == 0 for _, c in t2.values())
