"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds data only: the dynamic-circuit description (the triple
D = (Q, C, O) of Def. III.5), generators for the paper's fixed circuits and
for the seeded random brickwork workloads, and the random numbers the method
consumes (generic-init Gaussians, sampling uniforms, per-branch bond caps).
It contains none of the simulation arithmetic; each side (oracle, HIP path)
evaluates conditions, contracts tensors and samples outcomes on its own.
"""
from .circuits import (  # noqa: F401
    Gate, Measure, Cond, CGate, Circuit,
    X, Y, Z, H, I2, CNOT_01, CNOT_10,
    haar_unitary, teleportation, ghz_dynamic, brickwork, workload, WORKLOADS,
)
from .randomness import (  # noqa: F401
    bond_dims, bra_init_gaussians, shot_uniforms, branch_chi_draw,
)
