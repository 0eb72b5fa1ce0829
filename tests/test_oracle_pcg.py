"""Pins for the preconditioned-CG primal update (oracle.pcg) and ADMM with it.

* Block-diagonal S: the block-Jacobi preconditioner is S^-1, so PCG is
  exact after one iteration.
* SPD block-tridiagonal S (a random-LTI Schur matrix): PCG reaches the
  direct solution (relative 1e-10) within n (N + 1) iterations, and the
  S-norm of the error never increases (the CG optimality property).
* ADMM with PCG at a tight tolerance follows the direct ADMM iterates; with
  a loose one it still converges to the polished optimum.
"""
import numpy as np
import scipy.sparse as sp

from oracle.admm import ADMMSettings, admm_solve, _QPMats
from oracle.pcg import diag_block_inverses, pcg
from oracle.qp import lti_batch_qp
from workloads import random_lti


def _schur(N=12, seed=3):
    b = random_lti(1, N=N, seed=seed)
    qp = lti_batch_qp(b, 0)
    S = _QPMats(qp).schur(1e-6, 100.0, 0.1).tocsr()
    return qp, S


def test_block_diagonal_exact_in_one_iteration():
    rng = np.random.default_rng(1)
    n, m = 6, 5
    blocks = []
    for _ in range(m):
        a = rng.standard_normal((n, n))
        blocks.append(a @ a.T + n * np.eye(n))
    S = sp.block_diag(blocks).tocsr()
    b = rng.standard_normal(n * m)
    x, k = pcg(S, b, np.zeros(n * m), diag_block_inverses(S, n), 5, 0.0)
    assert k == 5  # tol 0: runs the cap, but the first iteration is already exact
    x1, _ = pcg(S, b, np.zeros(n * m), diag_block_inverses(S, n), 1, 0.0)
    np.testing.assert_allclose(S @ x1, b, rtol=1e-12, atol=1e-12)


def test_converges_to_the_direct_solution_with_monotone_energy_error():
    qp, S = _schur()
    n = qp.n
    rng = np.random.default_rng(2)
    b = rng.standard_normal(S.shape[0])
    xs = np.linalg.solve(S.toarray(), b)
    Binv = diag_block_inverses(S, n)
    x, k = pcg(S, b, np.zeros_like(b), Binv, S.shape[0], 1e-13)
    assert k <= S.shape[0]
    assert np.max(np.abs(x - xs)) <= 1e-9 * max(1.0, np.max(np.abs(xs)))
    errs = []
    for it in range(0, 40, 4):
        xi, _ = pcg(S, b, np.zeros_like(b), Binv, it, 0.0)
        e = xi - xs
        errs.append(float(e @ (S @ e)))
    assert all(errs[j + 1] <= errs[j] * (1 + 1e-9) for j in range(len(errs) - 1)), errs


def test_admm_with_pcg_tracks_the_direct_iterates():
    b = random_lti(1, N=20, seed=5)
    qp = lti_batch_qp(b, 0)
    st = dict(max_iter=60, k_check=0, adapt_rho=False)
    ref = admm_solve(qp, ADMMSettings(**st))
    got = admm_solve(qp, ADMMSettings(**st, linsolve="pcg", pcg_max_iter=500, pcg_tol=1e-13))
    assert np.max(np.abs(got.x - ref.x)) <= 1e-8 * max(1.0, np.max(np.abs(ref.x)))
    assert len(got.pcg_iters) == 60 and max(got.pcg_iters) > 1
    # a looser tolerance still converges (the outer iteration corrects the
    # inexact solves), in more ADMM iterations than the direct solve
    loose = admm_solve(qp, ADMMSettings(eps_abs=1e-6, eps_rel=1e-6, max_iter=5000, linsolve="pcg",
                                        pcg_max_iter=50, pcg_tol=1e-7))
    direct = admm_solve(qp, ADMMSettings(eps_abs=1e-6, eps_rel=1e-6, max_iter=5000))
    assert loose.status == 0 and direct.status == 0 and loose.iters >= direct.iters
    assert np.max(np.abs(loose.x - direct.x)) <= 1e-3 * max(1.0, np.max(np.abs(direct.x)))
