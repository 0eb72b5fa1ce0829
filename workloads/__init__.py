"""Seeded synthetic workloads for the batched optimal-control QP/SQP solver.

This package only draws random numbers and lays out problem parameters
(dynamics matrices, weights, bounds, reference trajectories).  It holds none
of the solver's arithmetic: no QP assembly, no factorisation, no ADMM step.
Both the CPU oracle and the GPU path consume what it produces.

Instance ``i`` of workload ``k`` is always drawn from
``numpy.random.default_rng([k, i])`` so that any prefix of a batch is
reproducible on its own.
"""
from .lti import LTIBatch, double_integrator, random_lti, paper_point_mass_matrices
from .bicycle import BicycleBatch, bicycle_batch, bicycle_long_and_ragged

__all__ = [
    "LTIBatch",
    "double_integrator",
    "random_lti",
    "paper_point_mass_matrices",
    "BicycleBatch",
    "bicycle_batch",
    "bicycle_long_and_ragged",
]
