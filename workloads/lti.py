"""Linear time-invariant MPC workloads (seeded, synthetic).

Each instance is a discrete-time system x_{t+1} = A x_t + B u_t with
quadratic stage cost 1/2 (x'Qx + u'Ru), terminal weight Q_f on x_N (and R on
u_N, which is a decision variable of the problem class), and box bounds on a
selection of the stage variables, written as  lo <= G (x_t, u_t) <= hi  with
G a 0/1 selection matrix that is the same at every stage t = 0..N.

The shapes follow the paper's linear-system experiments (Sec. "Linear-System
RL Scaling"); the concrete recipes are stated per generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LTIBatch:
    """A batch of LTI optimal-control problems sharing (nx, nu, N, G)."""

    name: str
    nx: int
    nu: int
    N: int
    A: np.ndarray  # [B, nx, nx]
    B: np.ndarray  # [B, nx, nu]
    Qd: np.ndarray  # [B, nx]   diagonal of Q
    Rd: np.ndarray  # [B, nu]   diagonal of R
    Qfd: np.ndarray  # [B, nx]  diagonal of the terminal state weight
    G: np.ndarray  # [ng, nx+nu] selection rows, shared by all stages and instances
    lo: np.ndarray  # [B, ng]
    hi: np.ndarray  # [B, ng]
    x0: np.ndarray  # [B, nx]
    dt: float = 0.1
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.nx + self.nu

    @property
    def ng(self) -> int:
        return self.G.shape[0]

    def subset(self, idx) -> "LTIBatch":
        idx = np.atleast_1d(np.asarray(idx))
        return LTIBatch(
            name=self.name, nx=self.nx, nu=self.nu, N=self.N,
            A=self.A[idx].copy(), B=self.B[idx].copy(), Qd=self.Qd[idx].copy(),
            Rd=self.Rd[idx].copy(), Qfd=self.Qfd[idx].copy(), G=self.G.copy(),
            lo=self.lo[idx].copy(), hi=self.hi[idx].copy(), x0=self.x0[idx].copy(),
            dt=self.dt, meta=dict(self.meta),
        )


def paper_point_mass_matrices(dim: int, dt: float):
    """Forward-Euler unit-mass double integrator in `dim` spatial dimensions.

    State (p, v), control u:  p+ = p + dt v,  v+ = v + dt u  (appendix
    "Neural Network Training", point-mass dynamics).
    """
    I = np.eye(dim)
    Z = np.zeros((dim, dim))
    A = np.block([[I, dt * I], [Z, I]])
    B = np.vstack([Z, dt * I])
    return A, B


def double_integrator(batch: int = 1, N: int = 20, seed: int = 1) -> LTIBatch:
    """2-D double integrator: nx=4 (px, py, vx, vy), nu=2, dt=0.1.

    Q = I, R = 0.1 I, Q_f = 10 I; controls boxed to [-1, 1], positions to
    [-5, 5]; x0 ~ U[-2, 2]^4 drawn from default_rng([seed, i]).
    """
    nx, nu = 4, 2
    A, Bm = paper_point_mass_matrices(2, 0.1)
    G = np.zeros((4, nx + nu))
    G[0, 0] = G[1, 1] = 1.0  # positions
    G[2, 4] = G[3, 5] = 1.0  # controls
    x0 = np.empty((batch, nx))
    for i in range(batch):
        rng = np.random.default_rng([seed, i])
        x0[i] = rng.uniform(-2.0, 2.0, size=nx)
    lo = np.tile(np.array([-5.0, -5.0, -1.0, -1.0]), (batch, 1))
    hi = -lo
    return LTIBatch(
        name="double_integrator", nx=nx, nu=nu, N=N,
        A=np.tile(A, (batch, 1, 1)), B=np.tile(Bm, (batch, 1, 1)),
        Qd=np.ones((batch, nx)), Rd=np.full((batch, nu), 0.1), Qfd=np.full((batch, nx), 10.0),
        G=G, lo=lo, hi=hi, x0=x0, dt=0.1,
    )


def random_lti(batch: int = 1024, N: int = 50, nx: int = 12, nu: int = 4, seed: int = 2,
               spectral_radius: float = 1.05, x_bound: float = 10.0, u_bound: float = 1.0,
               first: int = 0) -> LTIBatch:
    """Random LTI systems, all stage variables boxed.

    Per instance i (default_rng([seed, first + i]), draws in this order):
      Gm ~ N(0,1)^{nx x nx}, rescaled so its spectral radius is `spectral_radius`;
      A = I + 0.1 Gm;  B ~ N(0,1)^{nx x nu} / sqrt(nx);  Q = diag(U[0.5, 2]^nx);
      x0 ~ N(0, I).
    R = 0.1 I, Q_f = Q, x in [-x_bound, x_bound], u in [-u_bound, u_bound].
    """
    n = nx + nu
    A = np.empty((batch, nx, nx))
    Bm = np.empty((batch, nx, nu))
    Qd = np.empty((batch, nx))
    x0 = np.empty((batch, nx))
    for i in range(batch):
        rng = np.random.default_rng([seed, first + i])
        Gm = rng.standard_normal((nx, nx))
        Gm *= spectral_radius / np.max(np.abs(np.linalg.eigvals(Gm)))
        A[i] = np.eye(nx) + 0.1 * Gm
        Bm[i] = rng.standard_normal((nx, nu)) / np.sqrt(nx)
        Qd[i] = rng.uniform(0.5, 2.0, size=nx)
        x0[i] = rng.standard_normal(nx)
    lo_row = np.concatenate([np.full(nx, -x_bound), np.full(nu, -u_bound)])
    return LTIBatch(
        name="random_lti", nx=nx, nu=nu, N=N, A=A, B=Bm, Qd=Qd,
        Rd=np.full((batch, nu), 0.1), Qfd=Qd.copy(), G=np.eye(n),
        lo=np.tile(lo_row, (batch, 1)), hi=np.tile(-lo_row, (batch, 1)), x0=x0, dt=0.1,
        meta={"seed": seed, "first": first},
    )
