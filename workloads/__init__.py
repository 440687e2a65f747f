"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This package only draws random numbers and lays out grids and problem
parameters.  It holds none of the Leja method's arithmetic (no stencil, no
phi-function, no interpolation), so both the oracle and the HIP path can take
their inputs from it without sharing any computation.
"""
from .problems import (  # noqa: F401
    Problem,
    adr_neumann,
    advdiff_bump,
    allen_cahn_noise,
    brusselator_perturbed,
    burgers_sines,
    diag_problem,
    fourier_modes,
    gray_scott_spots,
    batch_instances,
    proposal_training_set,
    uniform_vector,
)
