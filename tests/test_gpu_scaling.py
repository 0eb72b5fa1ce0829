"""GPU parity of the rescaled ADMM solve (Remark 4, "Rescaling") against the
oracle's rescaled Algorithm 3 (oracle.scaling; the same transform, the
stopping test on the original problem, the step size from the rescaled
residuals).

* Box normalisation derived on the device (ocp_set_scaling_box, p = 0.6):
  FP64 iterates at fixed rho, and with rho adaptation, equal the oracle's
  (1e-9 / 1e-8) on the random LTI and double-integrator workloads -- which
  also pins the device-computed factors to the oracle's box_scaling.
* Caller-given factors (ocp_set_scaling, arbitrary positive values) on the
  general QP interface with time-varying blocks and a control-rate cost
  (E_t != 0): FP64 iterates 1e-9.
* FP32 iterations to their noise floor: the primal solution within 1e-4 and
  the multipliers within 1e-3 of the polished optimum of the original problem.
* Adjoint on a rescaled solve: active set, eta and the QP-data gradients in
  the original variables within 1e-6 of the oracle's dense solve.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.adjoint import active_set, adjoint_dense, polish, qp_vjp  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from oracle.scaling import Scaling, box_scaling  # noqa: E402
from workloads import double_integrator, random_lti  # noqa: E402

FP64, MIXED = 0, 1
P = 0.6


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


def _scaled_lti(b, precision):
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    s = OCPSolver(b.nx, b.nu, b.ng, np.full(b.batch, b.N), model=A.MODEL_LTI, precision=precision)
    s.set_scaling_box(P)
    s.set_lti(b.A, b.B, b.Qd, b.Rd, b.Qfd, b.G, b.lo, b.hi, b.x0)
    return s


@pytest.mark.parametrize("workload", ["random_lti", "double_integrator"])
@pytest.mark.parametrize("adapt", [False, True], ids=["fixed_rho", "adaptive_rho"])
def test_box_scaled_iterates_match_oracle(workload, adapt):
    b = random_lti(6, N=20, seed=2) if workload == "random_lti" else double_integrator(4, N=20, seed=1)
    s = _scaled_lti(b, FP64)
    K = 150
    out = s.solve(_settings(max_admm=K, k_check=0, adapt_rho=int(adapt)))
    tol = 1e-8 if adapt else 1e-9
    for i in range(b.batch):
        qp = lti_batch_qp(b, i)
        ref = admm_solve(qp, ADMMSettings(max_iter=K, k_check=0, adapt_rho=adapt), scaling=box_scaling(qp, P))
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < tol, (i, k, rel(got[k], getattr(ref, k)))
        assert int(out["n_factor"][i]) == ref.n_factor
        assert abs(float(out["r_prim"][i]) - ref.r_prim) <= 1e-8 * max(1.0, ref.r_prim)
        assert abs(float(out["r_dual"][i]) - ref.r_dual) <= 1e-8 * max(1.0, ref.r_dual)
    s.close()


def _rate_cost_qps(N=24, w=2.0):
    b = double_integrator(3, N=N, seed=4)
    qps = []
    for i in range(3):
        qp = lti_batch_qp(b, i)
        nx, n = qp.nx, qp.n
        for t in range(N):
            qp.D[t, nx:, nx:] += w * np.eye(n - nx)
            qp.D[t + 1, nx:, nx:] += w * np.eye(n - nx)
            qp.E[t, nx:, nx:] = -w * np.eye(n - nx)
        qp.q[:] = np.random.default_rng(i).normal(scale=0.3, size=qp.q.shape)
        qps.append(qp)
    return qps


def test_caller_scaling_on_time_varying_qp_with_rate_cost():
    from paper_2606_24039_amd import _abi as A
    from paper_2606_24039_amd.solver import OCPSolver

    qps = _rate_cost_qps()
    q0 = qps[0]
    rng = np.random.default_rng(7)
    scs = [Scaling(rng.uniform(0.3, 3.0, q0.n), rng.uniform(0.3, 3.0, q0.ng), float(rng.uniform(0.05, 5.0)))
           for _ in qps]
    pad = lambda a: np.concatenate([a, np.zeros((1,) + a.shape[1:])])  # noqa: E731
    cat = lambda f, p=False: np.concatenate([pad(getattr(q, f)) if p else getattr(q, f) for q in qps])  # noqa: E731
    s = OCPSolver(q0.nx, q0.nu, q0.ng, np.array([q.N for q in qps]), model=A.MODEL_QP, precision=FP64)
    s.set_scaling(np.stack([c.d for c in scs]), np.stack([c.e_g for c in scs]), np.array([c.c for c in scs]))
    s.set_qp(cat("D"), cat("Am", True), cat("Ap", True), np.stack([q.x_init for q in qps]), cat("G"), cat("lo"),
             cat("hi"), E=cat("E", True), q=cat("q"), b=cat("b", True))
    K = 120
    out = s.solve(_settings(max_admm=K, k_check=0, adapt_rho=0))
    for i, (qp, sc) in enumerate(zip(qps, scs)):
        ref = admm_solve(qp, ADMMSettings(max_iter=K, k_check=0, adapt_rho=False), scaling=sc)
        got = per_instance(s, out, i)
        for k in ("x", "z_g", "y_f", "y_g"):
            assert rel(got[k], getattr(ref, k)) < 1e-9, (i, k, rel(got[k], getattr(ref, k)))
    s.close()


def test_fp32_rescaled_converges_to_the_original_optimum():
    b = random_lti(8, N=50, seed=2)
    s = _scaled_lti(b, MIXED)
    out = s.solve(_settings(eps_abs=1e-6, eps_rel=1e-6, max_admm=5000))
    tight = ADMMSettings(eps_abs=1e-11, eps_rel=1e-11, max_iter=50000)
    for i in range(b.batch):
        qp = lti_batch_qp(b, i)
        r = admm_solve(qp, tight)
        ok, ref = polish(qp, r.x, r.y_g, eps_solve=1e-8)
        assert ok
        got = per_instance(s, out, i)
        # FP32 iterations stop at their noise floor (status 1 at eps 1e-6 is
        # allowed, as unscaled); the solution must still be the optimum
        assert rel(got["x"], ref["x"]) < 1e-4, (i, rel(got["x"], ref["x"]))
        assert rel(got["y_f"], ref["y_f"]) < 1e-3, (i, rel(got["y_f"], ref["y_f"]))
        assert rel(got["y_g"], ref["y_g"]) < 1e-3, (i, rel(got["y_g"], ref["y_g"]))
    s.close()


@pytest.mark.parametrize("precision", [FP64, MIXED], ids=["fp64", "mixed"])
def test_adjoint_of_a_rescaled_solve(precision):
    b = random_lti(8, N=30, seed=4)
    s = _scaled_lti(b, precision)
    eps = 1e-9 if precision == FP64 else 1e-6
    st = _settings(eps_abs=eps, eps_rel=eps, max_admm=5000, eps_active=1e-6)
    out = s.solve(st)
    dl = torch.as_tensor(np.random.default_rng(3).standard_normal((s.S, s.n)), dtype=torch.float64, device="cuda")
    g = s.adjoint(dl, st)
    for i in range(b.batch):
        qp = lti_batch_qp(b, i)
        sol = per_instance(s, out, i)
        lower, upper = active_set(qp, sol["x"], sol["y_g"], sol["xi"], eps_solve=1e-6)
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        assert np.array_equal(act < 0, lower) and np.array_equal(act > 0, upper), i
        gx = s.split(dl, i).cpu().numpy().reshape(-1)
        ex, ef, eg = adjoint_dense(qp, sol["x"], gx, lower, upper)
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper)
        errs = {k: rel(s.split(g[k], i).cpu().numpy().reshape(-1), ref)
                for k, ref in (("eta_x", ex), ("eta_f", ef), ("eta_g", eg))}
        errs.update({k: rel(s.split(g[k], i).cpu().numpy(), qg[k]) for k in ("d_q", "d_Ddiag", "d_lo", "d_hi")})
        errs["d_x_init"] = rel(g["d_x_init"][i].cpu().numpy(), qg["d_x_init"])
        assert max(errs.values()) < 1e-6, (i, errs)
        assert int(g["adj_status"][i]) == 0
    s.close()
