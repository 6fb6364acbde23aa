"""Helpers of the GPU tests: build the same problem on the GPU (through the C
ABI) and in the oracle, from one seeded permeability field.

The two sides share only the input field and the problem description; the
GPU computes its transmissibilities, right-hand side and operator in the HIP
library, the oracle computes its own in FP64 (rounding T to FP32 once, as the
library's inputs are FP32).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from oracle import tpfa


def gpu_problem(mf, k, c=1e-3, kz_ratio=1.0, dmask=None, pd=None, accum=None, stream=None):
    import torch
    nx, ny, nz = k.shape
    n = k.size
    dev = torch.device("cuda")
    kd = torch.from_numpy(np.ascontiguousarray(k, dtype=np.float64).ravel()).to(dev)
    tx, ty, tz = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
    mf.perm_to_trans(nx, ny, nz, kd, kz_ratio, tx, ty, tz, stream=stream)
    g = mf.create_grid(nx, ny, nz, stream=stream)
    b = torch.empty(n, dtype=torch.float32, device=dev)
    dm = None if dmask is None else torch.from_numpy(dmask.astype(np.uint8).ravel()).to(dev)
    pdd = None if pd is None else torch.from_numpy(pd.astype(np.float32).ravel()).to(dev)
    acc = None if accum is None else torch.from_numpy(accum.astype(np.float32).ravel()).to(dev)
    mf.set_transmissibility(g, tx, ty, tz, accum=acc, accum_scalar=c, dmask=dm, pD=pdd, b_out=b)
    return g, (tx, ty, tz), b


class OracleProblem:
    def __init__(self, k, c=1e-3, kz_ratio=1.0, dmask=None, pd=None, accum=None):
        self.shape = k.shape
        self.T = tpfa.round_to_f32(*tpfa.transmissibility(k, kz_ratio))
        if dmask is None:
            self.dmask, self.pd = tpfa.x_plane_dirichlet(k.shape)
        else:
            self.dmask = dmask.astype(bool)
            self.pd = tpfa.round_to_f32(pd)
        self.c = tpfa.round_to_f32(accum if accum is not None else np.float32(c))
        self.A, self.b = tpfa.assemble(*self.T, self.c, self.dmask, self.pd)
        self.Auu, self.bu, self.u = tpfa.reduce_to_unknowns(self.A, self.b, self.dmask)
        self._direct = None

    def direct(self):
        if self._direct is None:
            # the reduced matrix is symmetric: a minimum-degree ordering of
            # A^T + A keeps the LU fill (and the time) a third of COLAMD's on 3D grids
            xu = spla.spsolve(self.Auu.tocsc(), self.bu, permc_spec="MMD_AT_PLUS_A")
            self._direct = tpfa.scatter_solution(xu, self.u, self.pd, self.dmask)
        return self._direct

    def diag(self):
        """c + sum of the six faces on unknown cells, 1 on Dirichlet cells."""
        return self.A.diagonal()

    def rel_residual(self, x):
        return tpfa.relative_residual(self.A, self.b, x, self.dmask)
