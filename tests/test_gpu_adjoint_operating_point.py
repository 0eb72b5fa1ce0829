"""GPU adjoint at the setting the benchmark times: ADMM solves stopped at
eps_abs = eps_rel = 1e-4 (cap 1000 iterations, test every 25) and the active
set taken with eps_active = 1e-4, on the full batched workloads
(1024 random LTI instances of N = 50; 512 of N = 64), both precisions.

For 64 sampled instances of each batch the oracle takes the GPU's returned
solution, identifies the active set by the same rule (Appendix "Active
constraints identification") and solves the active-set KKT system K eta =
(dL/dx, 0, 0) directly (eq. bwd:noslack_kkt_matrix; the minimum-norm solution
where the active rows are dependent).  Checked:

* the active set equals the oracle's, row by row;
* every instance the GPU flags OCP_ADJ_OK has eta_x, eta_f, eta_g and the
  QP-data gradients within 1e-6 (relative, ||a-b||_inf / max(||b||_inf, 1))
  of the oracle's -- the adjoint runs in FP64 in both precisions;
* every instance flagged OCP_ADJ_OK reports a residual at most the
  tolerance, and at most 1 % of the converged instances are flagged;
* flagged instances (and every flagged converged one) are reported with
  their error against the oracle, never silently compared.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gpu_helpers import lti_solver, per_instance, rel  # noqa: E402
from oracle.adjoint import active_set, adjoint_dense, qp_vjp  # noqa: E402
from oracle.qp import lti_batch_qp  # noqa: E402
from workloads import random_lti  # noqa: E402

FP64, MIXED = 0, 1
WORKLOADS = {"lti1024_n50": (1024, 50, 2), "lti512_n64": (512, 64, 4)}


def _settings(**kw):
    from paper_2606_24039_amd import default_settings

    return default_settings(**kw)


@pytest.mark.parametrize("precision", [MIXED, FP64], ids=["mixed", "fp64"])
@pytest.mark.parametrize("workload", list(WORKLOADS))
def test_adjoint_at_the_benchmark_setting(workload, precision):
    from paper_2606_24039_amd import _abi as A

    B, N, seed = WORKLOADS[workload]
    b = random_lti(B, N=N, seed=seed)
    s = lti_solver(b, precision)
    st = _settings(eps_abs=1e-4, eps_rel=1e-4, max_admm=1000, k_check=25, k_rho=25, eps_active=1e-4)
    out = s.solve(st)
    rng = np.random.default_rng(11)
    dl = torch.as_tensor(rng.standard_normal((s.S, s.n)), dtype=torch.float64, device="cuda")
    g = s.adjoint(dl, st)
    status = out["status"].cpu().numpy()
    astat = g["adj_status"].cpu().numpy()
    ares = g["adj_resid"].cpu().numpy()
    conv = status == A.SOLVED
    assert np.all(ares[astat == A.ADJ_OK] <= st.adj_tol)
    conv_flagged = np.flatnonzero(conv & (astat != A.ADJ_OK))
    # the flag marks exceptions among the converged instances, not the rule
    assert conv_flagged.size <= max(2, conv.sum() // 100), conv_flagged
    flagged = []
    sample = sorted(set(range(0, B, B // 64)) | set(conv_flagged.tolist()))
    for i in sample:
        qp = lti_batch_qp(b, i)
        sol = per_instance(s, out, i)
        lower, upper = active_set(qp, sol["x"], sol["y_g"], sol["xi"], eps_solve=1e-4)
        act = s.split(g["active"], i).cpu().numpy().reshape(-1)
        assert np.array_equal(act < 0, lower) and np.array_equal(act > 0, upper), i
        gx = s.split(dl, i).cpu().numpy().reshape(-1)
        ex, ef, eg = adjoint_dense(qp, sol["x"], gx, lower, upper)
        qg = qp_vjp(qp, sol["x"], ex, ef, eg, lower, upper)
        errs = {k: rel(s.split(g[k], i).cpu().numpy().reshape(-1), ref)
                for k, ref in (("eta_x", ex), ("eta_f", ef), ("eta_g", eg))}
        errs.update({k: rel(s.split(g[k], i).cpu().numpy(), qg[k]) for k in ("d_q", "d_Ddiag", "d_lo", "d_hi")})
        errs["d_x_init"] = rel(g["d_x_init"][i].cpu().numpy(), qg["d_x_init"])
        worst = max(errs.values())
        if astat[i] != A.ADJ_OK:  # reported, not compared
            flagged.append((i, int(status[i]), int(astat[i]), float(ares[i]), worst))
            continue
        assert worst < 1e-6, (i, float(ares[i]), errs)
    print(f"[{workload} prec={precision}] flagged instances (i, solve status, adj status, resid, "
          f"error vs oracle): {flagged}", flush=True)
    assert len(flagged) <= 64 // 8  # the flag marks exceptions, not the rule
    s.close()
