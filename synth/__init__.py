"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

Everything here draws random numbers and shapes them into the inputs of a
workload: permeability fields, grid shapes of a batch, accumulation values.
It holds none of the solver's arithmetic (no transmissibility, operator,
right-hand side or Krylov step), so that both sides of a parity test can take
their inputs from it without sharing any of the method.
"""
from .perm import (  # noqa: F401
    lognormal_iid,
    lognormal_correlated,
    channelised,
    batch_systems,
    Workload,
    WORKLOADS,
    workload_field,
    white_residuals,
)
from .mesh import cartesian_faces, random_face_mesh  # noqa: F401
