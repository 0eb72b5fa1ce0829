"""Problem rescaling (Remark 4, "Rescaling": states and controls normalised
inside the solver, transparently to the caller).

Written from the statement that the solver normalises states and controls
before it runs Algorithm 3 and hands back the solution of the original
problem.  A diagonal change of variables x_t = d * xh_t (the same d in R^n at
every stage), a cost factor c > 0 and row factors chosen so that the block
structure survives:

  scaled cost     c (1/2 x'Px + q'x):  Dh_t = c diag(d) D_t diag(d),
                  Eh_t = c diag(d) E_t diag(d),  qh_t = c d * q_t
  equality rows   rows of the initial state and of the dynamics multiplied by
                  1/d_x (component-wise), so A_init = [I 0] and A+ = [-I 0]
                  keep their form:  Amh_t = diag(1/d_x) Am_t diag(d),
                  Aph_t = diag(1/d_x) Ap_t diag(d),  bh_t = b_t / d_x,
                  xh_init = x_init / d_x
  inequality rows row r multiplied by e_g[r] (a selection row of variable j
                  with e_g = 1/d_j stays a selection row):
                  Gh_t = diag(e_g) G_t diag(d),  loh = e_g * lo,  hih = e_g * hi

The optimisers correspond one to one: x = d * xh, z_g = zh / e_g,
xi = xih / e_g, y_f = e_f * yh_f / c with e_f = 1/d_x, y_g = e_g * yh_g / c
(multiply the original KKT conditions by c diag(d) and the rows by e).  Soft
rows are supported with e_g = 1 on those rows; their slack weights are then
multiplied by c.

Parity: the scaled data are pinned by evaluating cost and constraints of both
problems at corresponding points; the solution map by the polished optimum of
the original problem and its KKT stationarity (tests/test_oracle_scaling.py).
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .qp import HARD, StageQP


@dataclass
class Scaling:
    d: np.ndarray    # [n] variable factors (x = d * xh)
    e_g: np.ndarray  # [ng] inequality-row factors
    c: float = 1.0   # cost factor


def identity_scaling(qp: StageQP) -> Scaling:
    return Scaling(np.ones(qp.n), np.ones(qp.ng), 1.0)


def _pow2(v):
    """The power of two nearest to v > 0 in the logarithm (2^rint(log2 v)):
    factors that scale exactly in floating point."""
    return float(np.exp2(np.rint(np.log2(v))))


def box_scaling(qp: StageQP, p: float = 0.6) -> Scaling:
    """Normalisation by the box widths, in powers of two: d_j = 2^rint(p
    log2 h_j) with h_j the half width of the bound on variable j for
    variables boxed by a selection row of G (read at stage 0), 1 for the
    others; e_g = 1/d_j on selection rows, 2^-rint(log2 max_j |G_rj d_j|) on
    other hard rows, 1 on soft rows; c = 2^-rint(log2 m) with m the largest
    diagonal entry of diag(d) D_t diag(d) over the stages."""
    n, ng = qp.n, qp.ng
    d = np.ones(n)
    G0 = qp.G[0]
    sel = np.full(ng, -1)
    for r in range(ng):
        nz = np.flatnonzero(G0[r] != 0.0)
        if nz.size == 1 and G0[r, nz[0]] == 1.0 and qp.soft[r] == HARD:
            sel[r] = nz[0]
            half = 0.5 * (qp.hi[0, r] - qp.lo[0, r])
            if np.isfinite(half) and half > 0:
                d[nz[0]] = float(np.exp2(np.rint(p * np.log2(half))))
    e_g = np.ones(ng)
    for r in range(ng):
        if qp.soft[r] != HARD:
            continue
        if sel[r] >= 0:
            e_g[r] = 1.0 / d[sel[r]]
        else:
            m = float(np.max(np.abs(G0[r] * d)))
            e_g[r] = 1.0 / _pow2(m) if m > 0 else 1.0
    dd = max(float(np.max(np.diag(qp.D[t]) * d * d)) for t in range(qp.N + 1))
    c = 1.0 / _pow2(dd) if dd > 0 else 1.0
    return Scaling(d, e_g, c)


def scale_qp(qp: StageQP, sc: Scaling) -> StageQP:
    """The rescaled QP (same stage structure)."""
    d = np.asarray(sc.d, float)
    e = np.asarray(sc.e_g, float)
    c = float(sc.c)
    nx = qp.nx
    if np.any(e[qp.soft != HARD] != 1.0):
        raise ValueError("soft rows need e_g = 1")
    dx = d[:nx]
    return replace(
        qp,
        D=c * d[None, :, None] * qp.D * d[None, None, :],
        E=c * d[None, :, None] * qp.E * d[None, None, :],
        q=c * qp.q * d[None, :],
        Am=qp.Am * d[None, None, :] / dx[None, :, None],
        Ap=qp.Ap * d[None, None, :] / dx[None, :, None],
        b=qp.b / dx[None, :],
        x_init=qp.x_init / dx,
        G=e[None, :, None] * qp.G * d[None, None, :],
        lo=qp.lo * e[None, :],
        hi=qp.hi * e[None, :],
        gamma2=c * qp.gamma2,
        gamma1=c * qp.gamma1,
    )


def _stage_tiles(qp: StageQP, sc: Scaling):
    N1 = qp.N + 1
    dv = np.tile(np.asarray(sc.d, float), N1)
    ef = np.tile(1.0 / np.asarray(sc.d, float)[:qp.nx], N1)
    eg = np.tile(np.asarray(sc.e_g, float), N1)
    return dv, ef, eg


def to_unscaled(qp: StageQP, sc: Scaling, x, z_g, xi, y_f, y_g):
    """Map a point of the scaled problem to the original variables."""
    dv, ef, eg = _stage_tiles(qp, sc)
    return dv * x, z_g / eg, xi / eg, ef * y_f / sc.c, eg * y_g / sc.c


def to_scaled(qp: StageQP, sc: Scaling, x, z_g, xi, y_f, y_g):
    """Inverse of to_unscaled."""
    dv, ef, eg = _stage_tiles(qp, sc)
    return x / dv, z_g * eg, xi * eg, sc.c * y_f / ef, sc.c * y_g / eg
