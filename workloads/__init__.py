"""Seeded synthetic spatio-temporal workloads shared by the oracle, the tests and the bench.

This package only draws inputs (grids, base matrices, observation locations, covariates,
data and hyperparameter points).  It holds none of the arithmetic of the INLA objective or
its gradient: building Q(theta), factorising it and differentiating it happen in the oracle
and in the HIP library, each with its own code.
"""
from .spde import (  # noqa: F401
    SpdeModel,
    make_model,
    named_config,
    NAMED_CONFIGS,
    neumann_second_difference,
)
