"""Pins for the slack-update projections (Sec. "Slack update"; Appendix
"ADMM with slack variables", Lemma-1 case analysis).

Each closed form is checked against a brute-force minimisation of the prox
objective over (z, xi) with z + xi in [lo, hi]: for a fixed w = z + xi the
problem in xi is one-dimensional and is minimised on a fine grid, then w is
scanned over [lo, hi].
"""
import numpy as np
import pytest

from oracle.admm import project
from oracle.qp import HARD, SOFT_L1, SOFT_L2


def _brute(v, lo, hi, rho, pen):
    """min over w in [lo,hi], xi of pen(xi) + rho/2 (w - xi - v)^2 (z = w - xi)."""
    ws = np.linspace(lo, hi, 2001)
    best = (np.inf, None, None)
    for w in ws:
        # xi grid around the unconstrained candidate region
        xis = np.linspace(-abs(w - v) - 1.0, abs(w - v) + 1.0, 4001)
        obj = pen(xis) + 0.5 * rho * (w - xis - v) ** 2
        j = np.argmin(obj)
        if obj[j] < best[0]:
            best = (obj[j], w - xis[j], xis[j])
    return best


@pytest.mark.parametrize("v", [-3.7, -1.2, -0.5, 0.3, 0.999, 1.4, 2.6, 7.0])
@pytest.mark.parametrize("rho", [0.1, 1.0, 4.0])
def test_l2_prox_matches_brute_force(v, rho):
    lo, hi, g2 = -1.0, 1.0, 2.5
    z, xi = project(np.array([v]), np.array([lo]), np.array([hi]), np.array([SOFT_L2]), rho, g2, 1.0)
    obj, zb, xib = _brute(v, lo, hi, rho, lambda x: 0.5 * g2 * x ** 2)
    ours = 0.5 * g2 * xi[0] ** 2 + 0.5 * rho * (z[0] - v) ** 2
    assert ours <= obj + 1e-6
    assert abs(z[0] - zb) < 5e-3 and abs(xi[0] - xib) < 5e-3


@pytest.mark.parametrize("v", [-9.0, -3.7, -1.2, -0.5, 0.3, 1.05, 1.4, 2.6, 30.0])
@pytest.mark.parametrize("rho", [0.1, 1.0, 4.0])
def test_l1_prox_matches_brute_force(v, rho):
    lo, hi, g1 = -1.0, 1.0, 2.0
    z, xi = project(np.array([v]), np.array([lo]), np.array([hi]), np.array([SOFT_L1]), rho, 1.0, g1)
    obj, zb, xib = _brute(v, lo, hi, rho, lambda x: g1 * np.abs(x))
    ours = g1 * abs(xi[0]) + 0.5 * rho * (z[0] - v) ** 2
    assert ours <= obj + 1e-6
    assert abs(ours - obj) < 1e-4


@pytest.mark.parametrize("v", [-3.0, -1.0, 0.2, 1.0, 5.0])
def test_hard_projection_is_clip(v):
    z, xi = project(np.array([v]), np.array([-1.0]), np.array([1.0]), np.array([HARD]), 0.3, 1.0, 1.0)
    assert z[0] == min(max(v, -1.0), 1.0) and xi[0] == 0.0


def test_projection_invariants(rng):
    """z + xi = Pi(v) on every row kind; gamma -> infinity recovers Pi."""
    v = rng.normal(scale=4.0, size=3000)
    lo = -rng.uniform(0.1, 2.0, size=3000)
    hi = rng.uniform(0.1, 2.0, size=3000)
    kind = rng.integers(0, 3, size=3000)
    z, xi = project(v, lo, hi, kind, 0.7, 3.0, 1.5)
    np.testing.assert_allclose(z + xi, np.clip(v, lo, hi), atol=1e-12)
    assert np.all(xi[kind == HARD] == 0.0)
    z2, xi2 = project(v, lo, hi, np.full(3000, SOFT_L2), 0.7, 1e12, 1.0)
    np.testing.assert_allclose(z2, np.clip(v, lo, hi), atol=1e-9)
    z1, xi1 = project(v, lo, hi, np.full(3000, SOFT_L1), 0.7, 1.0, 1e12)
    np.testing.assert_allclose(z1, np.clip(v, lo, hi), atol=1e-9)
    # L1 slack is exactly zero while the violation is within gamma1/rho
    z1, xi1 = project(v, lo, hi, np.full(3000, SOFT_L1), 0.7, 1.0, 1.5)
    small = np.abs(np.clip(v, lo, hi) - v) <= 1.5 / 0.7
    assert np.all(xi1[small] == 0.0)
