"""FP64 CPU oracle for the matrix-free TPFA conjugate-gradient solver.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import anything from this package; the
product path (the HIP library and its Python binding) never does, and shares
no code, table or helper with it.

The oracle is the plain definition written out: the operator is assembled
into a sparse CSR matrix from the face transmissibilities (Sec. II-A, Eq. 3,
4 and 6) and solved with textbook conjugate gradient (Alg. 1), in FP64 with
SciPy's CSR product as the only library step. Modules:

* ``tpfa``   -- transmissibilities, Dirichlet set, CSR assembly, right-hand side.
* ``krylov`` -- CG, Jacobi-PCG, flexible CG, mixed-precision iterative refinement.
* ``nn``     -- direct 3D convolution network (forward, backward, Adam) in FP64
               on BF16-rounded operands, for the learned preconditioner.
* ``timestep`` -- backward-Euler time steps with storage and wells, each solved
               directly (a step's residual is linear, one Newton step).
* ``faces``  -- the same operator on a face-list (unstructured) mesh.

Each function is pinned by CPU tests against closed forms, invariants, dense
solves and brute force (``tests/test_oracle_*.py``).
"""
from . import tpfa, krylov, timestep, faces  # noqa: F401
