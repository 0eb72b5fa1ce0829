"""Pins for the step-size adaptation of eq. rho:update (Sec. "Solving QP via
ADMM", step-size parameters selection).

* The candidate and its acceptance against hand-derived cases
  (tests/golden/rho_update.json): an inverted ratio, a dropped scale, a
  missing clip or a wrong threshold each fails one of them.
* Wiring inside Algorithm 3: the adaptation runs at multiples of k_rho on the
  residuals of that iterate, is skipped while the iterate passes the stopping
  test (even when the candidate would be accepted), and every accepted change
  refactors the Schur matrix.
"""
import json
import os

import numpy as np
import pytest

from oracle.admm import ADMMSettings, admm_solve, kkt_residuals, rho_update
from oracle.qp import lti_batch_qp
from workloads import random_lti

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rho_update.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: c["derivation"][:40])
def test_rho_candidate_matches_hand_derivation(case):
    st = ADMMSettings(**_golden()["settings"])
    cand, accept = rho_update(case["rho"], case["r_prim"], case["r_dual"], case["prim_scale"], case["dual_scale"], st)
    assert cand == pytest.approx(case["cand"], rel=1e-7)
    assert accept == case["accept"]


def _qp(i):
    return lti_batch_qp(random_lti(4, N=10, seed=2), i)


def test_adaptation_runs_at_k_rho_on_that_iterate_and_refactors():
    st = ADMMSettings(eps_abs=1e-9, eps_rel=1e-9, max_iter=60, k_check=0)
    qp = _qp(2)
    r = admm_solve(qp, st, record=True)
    assert r.rho_changes and r.rho_changes[0][0] == st.k_rho
    assert all(k % st.k_rho == 0 for k, _ in r.rho_changes)
    assert r.n_factor == 1 + len(r.rho_changes)
    # the accepted value is the candidate formed from the residuals of iterate k_rho
    x, z_g, xi, y_f, y_g = r.history[st.k_rho - 1]
    rp, rd, ps, ds = kkt_residuals(qp, x, z_g, xi, y_f, y_g)
    cand, accept = rho_update(st.rho0, rp, rd, ps, ds, st)
    assert accept and r.rho_changes[0][1] == cand


def test_no_adaptation_while_converged():
    # a loose tolerance: the iterate at k_rho passes the stopping test, so the
    # candidate is not taken even though its change would exceed the threshold
    st = ADMMSettings(eps_abs=1.0, eps_rel=1.0, max_iter=60, k_check=0)
    qp = _qp(2)
    r = admm_solve(qp, st, record=True)
    x, z_g, xi, y_f, y_g = r.history[st.k_rho - 1]
    rp, rd, ps, ds = kkt_residuals(qp, x, z_g, xi, y_f, y_g)
    assert rp <= st.eps_abs + st.eps_rel * ps and rd <= st.eps_abs + st.eps_rel * ds
    assert rho_update(st.rho0, rp, rd, ps, ds, st)[1]
    assert r.rho_changes == [] and r.n_factor == 1 and r.rho_bar == st.rho0


def test_no_adaptation_when_disabled():
    st = ADMMSettings(eps_abs=1e-9, eps_rel=1e-9, max_iter=60, k_check=0, adapt_rho=False)
    r = admm_solve(_qp(2), st)
    assert r.rho_changes == [] and r.n_factor == 1
