"""Preconditioned conjugate gradients for the ADMM primal update (the PCG
backends of the paper's table of QP solver backends; the hybrid direct /
PCG design of its discussion section), written from the textbook method
(Hestenes and Stiefel's conjugate gradients with a left preconditioner, as
in Saad, "Iterative Methods for Sparse Linear Systems", Algorithm 9.1).

Test infrastructure: only tests, the package's smoke check and the
benchmark's CPU leg use it.

The system is the Schur system S x~ = eta of the primal update (eq.
admm:schur), S symmetric positive definite and block tridiagonal over the
stages.  The preconditioner is block Jacobi: the inverses of S's n x n
diagonal blocks Theta_t.  Stopping rule: before each iteration, stop when
||r||_2 <= tol ||eta||_2 or after max_iter iterations.  The start x0 is the
caller's (ADMM passes its current primal iterate x).

Parity: exact in one iteration on block-diagonal S (the preconditioner is
S^-1); the direct solution within n (N+1) iterations on SPD block-tridiagonal
S; the S-norm of the error never increases (tests/test_oracle_pcg.py).
"""
from __future__ import annotations

import numpy as np


def diag_block_inverses(S, n):
    """Inverses of the n x n diagonal blocks of the (sparse or dense) S."""
    Sd = S.toarray() if hasattr(S, "toarray") else np.asarray(S)
    m = Sd.shape[0] // n
    return np.stack([np.linalg.inv(Sd[t * n:(t + 1) * n, t * n:(t + 1) * n]) for t in range(m)])


def apply_block_diag(Binv, r):
    n = Binv.shape[1]
    return np.einsum("tij,tj->ti", Binv, r.reshape(-1, n)).reshape(-1)


def pcg(S, b, x0, Binv, max_iter: int, tol: float):
    """Solve S x = b from x0 with the block-Jacobi preconditioner Binv.
    Returns (x, iterations taken)."""
    x = np.array(x0, dtype=float)
    r = b - S @ x
    z = apply_block_diag(Binv, r)
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.linalg.norm(b))
    k = 0
    while k < max_iter and float(np.linalg.norm(r)) > tol * bnorm:
        Sp = S @ p
        alpha = rz / float(p @ Sp)
        x = x + alpha * p
        r = r - alpha * Sp
        z = apply_block_diag(Binv, r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
    return x, k
