"""Stage-wise QP of an optimal-control problem (Sec. "QP Approximation of OCP";
Appendix "QP Approximation").

Decision vector x = (x_0, u_0, x_1, u_1, ..., x_N, u_N), n = nx + nu per stage.

    min  1/2 x'Px + q'x + slack penalty
    s.t. C x = c,   lo <= G x + xi <= hi   (xi only on soft rows)

P is block-tridiagonal with diagonal blocks D_t and sub-diagonal blocks E_t
(block (t+1, t)); C stacks the initial-state row block A_init = [I 0] and the
dynamics row blocks [A_t^-  A_t^+] acting on stages (t, t+1); G is
block-diagonal with blocks G_t.  c = (x_init, b_0, ..., b_{N-1}).

Row ordering of the constraint multipliers: y_f = (y_init, y_dyn_0 .. y_dyn_{N-1}),
y_g = (rows of G_0, ..., rows of G_N).

Parity: assembly pinned by tests that evaluate the OCP cost and constraints
directly (test_oracle_qp.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

HARD, SOFT_L2, SOFT_L1 = 0, 1, 2


@dataclass
class StageQP:
    nx: int
    nu: int
    N: int
    D: np.ndarray  # [N+1, n, n]
    E: np.ndarray  # [N, n, n]
    q: np.ndarray  # [N+1, n]
    Am: np.ndarray  # [N, nx, n]
    Ap: np.ndarray  # [N, nx, n]
    b: np.ndarray  # [N, nx]
    x_init: np.ndarray  # [nx]
    G: np.ndarray  # [N+1, ng, n]
    lo: np.ndarray  # [N+1, ng]
    hi: np.ndarray  # [N+1, ng]
    soft: np.ndarray = field(default=None)  # [ng] HARD / SOFT_L2 / SOFT_L1
    gamma2: float = 1.0  # L2 slack weight: (gamma2/2) ||xi||^2
    gamma1: float = 1.0  # L1 slack weight: gamma1 ||xi||_1

    def __post_init__(self):
        if self.soft is None:
            self.soft = np.zeros(self.ng, dtype=np.int64)

    @property
    def n(self) -> int:
        return self.nx + self.nu

    @property
    def ng(self) -> int:
        return self.G.shape[1]

    @property
    def nvar(self) -> int:
        return (self.N + 1) * self.n

    @property
    def neq(self) -> int:
        return self.nx * (self.N + 1)

    @property
    def nineq(self) -> int:
        return self.ng * (self.N + 1)

    def soft_rows(self) -> np.ndarray:
        """Soft-row kind for every stacked inequality row."""
        return np.tile(self.soft, self.N + 1)

    def matrices(self):
        """Sparse P, C, G and stacked q, c, lo, hi."""
        n, nx, N = self.n, self.nx, self.N
        Pb = [[None] * (N + 1) for _ in range(N + 1)]
        for t in range(N + 1):
            Pb[t][t] = sp.csr_matrix(self.D[t])
        for t in range(N):
            Pb[t + 1][t] = sp.csr_matrix(self.E[t])
            Pb[t][t + 1] = sp.csr_matrix(self.E[t].T)
        P = sp.bmat(Pb, format="csr")
        Cb = [[None] * (N + 1) for _ in range(N + 1)]
        A_init = np.hstack([np.eye(nx), np.zeros((nx, self.nu))])
        Cb[0][0] = sp.csr_matrix(A_init)
        for t in range(N):
            Cb[t + 1][t] = sp.csr_matrix(self.Am[t])
            Cb[t + 1][t + 1] = sp.csr_matrix(self.Ap[t])
        # make sure empty block columns still have a width
        for t in range(N + 1):
            if all(Cb[r][t] is None for r in range(N + 1)):
                Cb[0][t] = sp.csr_matrix((nx, n))
        C = sp.bmat(Cb, format="csr")
        G = sp.block_diag([sp.csr_matrix(self.G[t]) for t in range(N + 1)], format="csr")
        q = self.q.reshape(-1)
        c = np.concatenate([self.x_init, self.b.reshape(-1)])
        return P, C, G, q, c, self.lo.reshape(-1), self.hi.reshape(-1)


def lti_qp(A, B, Qd, Rd, Qfd, G, lo, hi, x0, N, c_dyn=None) -> StageQP:
    """QP of a linear-quadratic OCP (exact: the convexification of a linear
    problem is the problem itself).

    Cost 1/2 (x_t'Q x_t + u_t'R u_t) for t < N and 1/2 (x_N'Q_f x_N + u_N'R u_N);
    dynamics f_t = A x_t + B u_t + c_dyn - x_{t+1} = 0, so that
    A_t^- = [A B], A_t^+ = [-I 0], b_t = -c_dyn; bounds lo <= G_t (x_t,u_t) <= hi.
    """
    nx, nu = B.shape
    n = nx + nu
    D = np.zeros((N + 1, n, n))
    for t in range(N):
        D[t] = np.diag(np.concatenate([Qd, Rd]))
    D[N] = np.diag(np.concatenate([Qfd, Rd]))
    Am = np.tile(np.hstack([A, B]), (N, 1, 1))
    Ap = np.tile(np.hstack([-np.eye(nx), np.zeros((nx, nu))]), (N, 1, 1))
    b = np.zeros((N, nx)) if c_dyn is None else np.tile(-np.asarray(c_dyn, float), (N, 1))
    ng = G.shape[0]
    return StageQP(
        nx=nx, nu=nu, N=N, D=D, E=np.zeros((N, n, n)), q=np.zeros((N + 1, n)),
        Am=Am, Ap=Ap, b=b, x_init=np.asarray(x0, float).copy(),
        G=np.tile(G, (N + 1, 1, 1)), lo=np.tile(lo, (N + 1, 1)), hi=np.tile(hi, (N + 1, 1)),
        soft=np.zeros(ng, dtype=np.int64),
    )


def lti_batch_qp(batch, i: int) -> StageQP:
    """QP of instance i of a workloads.LTIBatch."""
    return lti_qp(batch.A[i], batch.B[i], batch.Qd[i], batch.Rd[i], batch.Qfd[i],
                  batch.G, batch.lo[i], batch.hi[i], batch.x0[i], batch.N)
