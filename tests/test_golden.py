"""Golden fixtures: constants and models the paper prints (tests/golden/*.json)."""
import json
import os

import numpy as np

from oracle.admm import ADMMSettings
from oracle.sqp import SQPSettings
from workloads import double_integrator

HERE = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def test_oracle_defaults_are_the_paper_constants():
    g = _load("paper_constants.json")
    s = ADMMSettings()
    assert s.sigma == g["sigma"]["value"]
    assert s.rho0 == g["rho_bar_0"]["value"]
    assert s.rho_f_scale == g["rho_f_over_rho_bar"]["value"]
    assert s.rho_min == g["rho_min"]["value"] and s.rho_max == g["rho_max"]["value"]
    assert s.k_rho == g["k_rho_iter"]["value"] and s.k_ratio == g["k_rho_ratio"]["value"]
    assert s.max_iter == g["max_admm_iterations"]["value"]
    assert SQPSettings().armijo_eta == g["armijo_eta"]["value"]


def test_double_integrator_workload_is_the_printed_euler_model():
    g = _load("point_mass_euler.json")
    b = double_integrator(3)
    for i in range(3):
        np.testing.assert_array_equal(b.A[i], np.array(g["A"]))
        np.testing.assert_array_equal(b.B[i], np.array(g["B"]))
    assert b.dt == g["dt"]
