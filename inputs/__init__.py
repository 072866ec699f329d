"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds problem statements (domain, grid sizes, decomposition sizes,
feature counts, manufactured solutions and their forcing terms) and the seeded
random draws the method consumes (the fixed hidden-layer weights and biases of
the random features, and per-instance problem parameters).  It holds none of
the method's arithmetic: no windows, no feature evaluation, no operator rows,
no solver.  Both the CPU oracle and the GPU path take their random numbers from
here as plain arrays.
"""
from .problems import (  # noqa: F401
    ProblemSpec,
    feature_params,
    grid_axes,
    grid_points,
    mlp_init,
    n_phi,
)
from .families import (  # noqa: F401
    ode_cos_exact,
    ode_cos_forcing,
    sines_exact,
    sines_forcing,
)
from . import configs  # noqa: F401
