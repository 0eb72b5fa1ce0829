"""Kinematic-bicycle racing-style workloads (seeded, synthetic).

State (px, py, yaw, v), control (acceleration a, steering angle delta).
Each instance tracks a reference driven at constant speed v_ref along a
curve whose curvature is  kappa(s) = amp * sin(2 pi s / 40 + phase),
amp ~ U[0, 0.2], phase ~ U[0, 2 pi), sampled on the dt grid.  The lateral
offset from the reference (the signed distance along the reference's left
normal) is bounded by +-2 m as a soft (L1-penalised) constraint; a and
delta are hard-boxed.

These constants are not given by the paper (its racing vehicle, tyre and
track data are not published); the recipe here is a synthetic stand-in of
the same shape (nx=4, nu=2, horizons 100 .. 8192, ragged batches).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

WHEELBASE = 2.5
V_REF = 8.0
DT = 0.05
CURV_PERIOD = 40.0
A_BOUND = 3.0
STEER_BOUND = 0.4
LAT_BOUND = 2.0
GAMMA_L1 = 100.0
Q_DIAG = (1.0, 1.0, 0.5, 0.1)
R_DIAG = (0.1, 1.0)


@dataclass
class BicycleBatch:
    horizons: np.ndarray  # [B] int64, N_i
    stage_off: np.ndarray  # [B+1] int64, first stage of instance i (N_i + 1 stages each)
    ref: np.ndarray  # [S, 4] reference state per stage
    normal: np.ndarray  # [S, 2] left unit normal of the reference per stage
    x0: np.ndarray  # [B, 4]
    dt: float = DT
    wheelbase: float = WHEELBASE
    a_bound: float = A_BOUND
    steer_bound: float = STEER_BOUND
    lat_bound: float = LAT_BOUND
    gamma_l1: float = GAMMA_L1
    Qd: np.ndarray = field(default_factory=lambda: np.array(Q_DIAG))
    Rd: np.ndarray = field(default_factory=lambda: np.array(R_DIAG))
    Qfd: np.ndarray = field(default_factory=lambda: np.array(Q_DIAG))
    meta: dict = field(default_factory=dict)
    integrator: int = 0  # 0: implicit midpoint, 1: trapezoidal rule
    # racing features (Sec. "Hardware Deployment: Autonomous Racing"): the
    # control-rate weight diagonal W (1/2 (u_t - u_{t+1})'W(u_t - u_{t+1}))
    # and the fixed first control u_0 = u_init [B, 2] (None: free)
    Wd: np.ndarray = field(default_factory=lambda: np.zeros(2))
    u_init: Optional[np.ndarray] = None

    nx: int = 4
    nu: int = 2
    ng: int = 3

    @property
    def batch(self) -> int:
        return len(self.horizons)

    @property
    def n(self) -> int:
        return self.nx + self.nu

    def stages(self, i: int) -> slice:
        return slice(int(self.stage_off[i]), int(self.stage_off[i + 1]))

    def subset(self, idx) -> "BicycleBatch":
        idx = np.atleast_1d(np.asarray(idx))
        refs, normals = [], []
        for i in idx:
            refs.append(self.ref[self.stages(i)])
            normals.append(self.normal[self.stages(i)])
        hor = self.horizons[idx].copy()
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(hor + 1)
        return BicycleBatch(
            horizons=hor, stage_off=off, ref=np.concatenate(refs), normal=np.concatenate(normals),
            x0=self.x0[idx].copy(), dt=self.dt, wheelbase=self.wheelbase, a_bound=self.a_bound,
            steer_bound=self.steer_bound, lat_bound=self.lat_bound, gamma_l1=self.gamma_l1,
            Qd=self.Qd.copy(), Rd=self.Rd.copy(), Qfd=self.Qfd.copy(), meta=dict(self.meta),
            integrator=self.integrator, Wd=np.array(self.Wd, dtype=float).copy(),
            u_init=None if self.u_init is None else np.asarray(self.u_init)[idx].copy(),
        )


def _reference(N: int, amp: float, phase: float, dt: float):
    """Reference (px, py, yaw, v) at s_t = V_REF * dt * t, t = 0..N.

    yaw(s) is the exact integral of the curvature; positions are integrated
    with composite Simpson's rule (8 panels per dt step).
    """
    w = 2.0 * np.pi / CURV_PERIOD

    def yaw(s):
        return amp / w * (np.cos(phase) - np.cos(w * s + phase))

    ds = V_REF * dt
    sub = 8
    h = ds / sub
    s_fine = np.arange(N * sub + 1) * h
    c = np.cos(yaw(s_fine))
    sn = np.sin(yaw(s_fine))
    # Simpson on pairs of panels -> cumulative at every dt boundary
    px = np.zeros(N + 1)
    py = np.zeros(N + 1)
    wts = np.ones(sub + 1)
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    wts *= h / 3.0
    for t in range(N):
        seg = slice(t * sub, t * sub + sub + 1)
        px[t + 1] = px[t] + np.dot(wts, c[seg])
        py[t + 1] = py[t] + np.dot(wts, sn[seg])
    s = np.arange(N + 1) * ds
    psi = yaw(s)
    ref = np.stack([px, py, psi, np.full(N + 1, V_REF)], axis=1)
    normal = np.stack([-np.sin(psi), np.cos(psi)], axis=1)
    return ref, normal


def _instance(rng: np.random.Generator, N: int, dt: float):
    amp = rng.uniform(0.0, 0.2)
    phase = rng.uniform(0.0, 2.0 * np.pi)
    dy = rng.uniform(-0.5, 0.5)
    dpsi = rng.uniform(-0.1, 0.1)
    vfac = rng.uniform(0.8, 1.2)
    ref, normal = _reference(N, amp, phase, dt)
    x0 = ref[0].copy()
    x0[1] += dy
    x0[2] += dpsi
    x0[3] = V_REF * vfac
    return ref, normal, x0


def _assemble(horizons, refs, normals, x0s, dt, meta) -> BicycleBatch:
    hor = np.asarray(horizons, dtype=np.int64)
    off = np.zeros(len(hor) + 1, dtype=np.int64)
    off[1:] = np.cumsum(hor + 1)
    return BicycleBatch(horizons=hor, stage_off=off, ref=np.concatenate(refs),
                        normal=np.concatenate(normals), x0=np.stack(x0s), dt=dt, meta=meta)


def bicycle_batch(batch: int = 4096, N: int = 100, seed: int = 3, first: int = 0,
                  dt: float = DT) -> BicycleBatch:
    """`batch` instances of horizon N; instance i from default_rng([seed, first + i])."""
    refs, normals, x0s = [], [], []
    for i in range(batch):
        r, nrm, x0 = _instance(np.random.default_rng([seed, first + i]), N, dt)
        refs.append(r)
        normals.append(nrm)
        x0s.append(x0)
    return _assemble([N] * batch, refs, normals, x0s, dt, {"seed": seed, "first": first})


def bicycle_long_and_ragged(seed: int = 5, long_N: int = 8192, ragged: int = 256,
                            n_lo: int = 32, n_hi: int = 2048, first: int = 0,
                            dt: float = DT):
    """One instance of horizon `long_N` (default_rng([seed, 0])) and a ragged
    batch of `ragged` instances, instance i drawn from default_rng([seed, 1, first + i])
    whose first draw is its horizon N_i ~ U{n_lo .. n_hi}."""
    r, nrm, x0 = _instance(np.random.default_rng([seed, 0]), long_N, dt)
    long_b = _assemble([long_N], [r], [nrm], [x0], dt, {"seed": seed, "kind": "long"})
    hors, refs, normals, x0s = [], [], [], []
    for i in range(ragged):
        rng = np.random.default_rng([seed, 1, first + i])
        Ni = int(rng.integers(n_lo, n_hi + 1))
        r, nrm, x0 = _instance(rng, Ni, dt)
        hors.append(Ni)
        refs.append(r)
        normals.append(nrm)
        x0s.append(x0)
    rag_b = _assemble(hors, refs, normals, x0s, dt, {"seed": seed, "kind": "ragged", "first": first})
    return long_b, rag_b
