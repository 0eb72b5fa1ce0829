"""Writes bicycle_qp_initial_linearisation.json: the oracle's exact solution
of the QP of the single long bicycle instance (N = 8192, seed 5) convexified
at the initial guess (the reference trajectory with zero controls; Appendix
"QP Approximation"), solved by the oracle's ADMM (Algorithm 3, eps 1e-7) and
polished on its active set.  Stored: the solution at every 64th stage and the
last one, and the QP objective value.  Calls only oracle/ and workloads/;
takes about two minutes.

    python tests/golden/make_bicycle_qp_reference.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.adjoint import polish  # noqa: E402
from oracle.admm import ADMMSettings, admm_solve  # noqa: E402
from oracle.models import BicycleOCP  # noqa: E402
from workloads import bicycle_long_and_ragged  # noqa: E402

STRIDE = 64


def main():
    lng, _ = bicycle_long_and_ragged(seed=5, ragged=1)
    ocp = BicycleOCP(lng, 0)
    qp = ocp.convexify(ocp.initial_guess())
    r = admm_solve(qp, ADMMSettings(eps_abs=1e-7, eps_rel=1e-7, max_iter=20000))
    ok, sol = polish(qp, r.x, r.y_g, xi=r.xi, eps_solve=1e-7)
    assert r.status == 0 and ok
    x = sol["x"].reshape(qp.N + 1, qp.n)
    P, C, G, q, c, lo, hi = qp.matrices()
    xs = sol["x"]
    obj = 0.5 * xs @ (P @ xs) + q @ xs + qp.gamma1 * np.sum(np.abs(sol["xi"]))
    stages = list(range(0, qp.N + 1, STRIDE)) + ([qp.N] if qp.N % STRIDE else [])
    out = {
        "_source": "oracle ADMM (Algorithm 3) + active-set polish of the QP of the N = 8192 bicycle instance "
                   "(seed 5) convexified at the reference trajectory with zero controls; written by "
                   "make_bicycle_qp_reference.py",
        "N": qp.N, "stride": STRIDE, "stages": stages, "x": x[stages].tolist(),
        "x_inf_norm": float(np.max(np.abs(xs))), "objective": float(obj), "admm_iters": int(r.iters),
    }
    with open(os.path.join(HERE, "bicycle_qp_initial_linearisation.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("written", len(stages), "stages; objective", obj)


if __name__ == "__main__":
    main()
