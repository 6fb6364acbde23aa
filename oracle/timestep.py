"""Backward-Euler time stepping of the pressure equation with wells (FP64).

Test infrastructure only (see the package docstring).

Paper passages followed:

* Sec. II-A: the pressure system comes from a low-order finite-volume scheme
  in space with an implicit (backward-Euler) step in time; the residual of
  Eq. 3 uses the TPFA flux of Eq. 4 at the new time level, and each time step
  is solved by Newton steps ``J dp = -r`` (Eq. 5).

Readings where the paper is silent:

* Storage. The paper's fluid is incompressible, so its equations carry no
  time derivative. A slightly compressible fluid adds the storage term
  ``c_K (p_K^{n+1} - p_K^n)`` with ``c_K = phi c_t V_K / dt``; with c = 0 it is
  the paper's model.
* Wells. The paper mentions injection and production but gives no well model.
  A perforated cell K carries the Peaceman-form term ``WI_K (p_K - pw_K)``
  (well index ``WI_K >= 0``, bottom-hole pressure ``pw_K``), treated
  implicitly; a source adds its rate ``q_K`` (positive = injection).
* Per unknown cell the step equation is
  ``c_K (p_K - p_K^n) + sum_L T_KL (p_K - p_L) + WI_K (p_K - pw_K) = q_K``
  and ``p_K = p_K^D`` on Dirichlet cells. It is linear in p: its Jacobian is the
  operator of ``tpfa.assemble`` with accumulation ``c + WI``, and one Newton
  step from any start solves it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import tpfa


def _field(v, shape):
    return np.broadcast_to(np.asarray(0.0 if v is None else v, dtype=np.float64), shape)


def step_rhs(b, c, p_old, dmask, wi=None, pw=None, q=None):
    """Right-hand side of one step: ``b + c p^n + WI pw + q`` on unknown cells,
    ``b`` (the Dirichlet value) on Dirichlet cells. ``b`` is the right-hand
    side of ``tpfa.assemble`` (the Dirichlet couplings)."""
    d = np.asarray(dmask, dtype=bool)
    shape = d.shape
    b = np.asarray(b, dtype=np.float64).reshape(shape)
    extra = (_field(c, shape) * np.asarray(p_old, dtype=np.float64).reshape(shape)
             + _field(wi, shape) * _field(pw, shape) + _field(q, shape))
    return np.where(d, b, b + extra)


def step(tx, ty, tz, c, dmask, pd, p_old, wi=None, pw=None, q=None):
    """One backward-Euler step: the new pressure field (shape of the grid),
    from a sparse direct solve of the unknown-cell block."""
    d = np.asarray(dmask, dtype=bool)
    shape = d.shape
    acc = _field(c, shape) + _field(wi, shape)
    A, b = tpfa.assemble(tx, ty, tz, acc, d, pd)
    rhs = step_rhs(b, c, p_old, d, wi, pw, q).ravel()
    Auu, _, u = tpfa.reduce_to_unknowns(A, b, d)
    xu = spla.spsolve(Auu.tocsc(), rhs[u])
    return tpfa.scatter_solution(xu, u, pd, d).reshape(shape)


def run(tx, ty, tz, c, dmask, pd, p0, nsteps, wi=None, pw=None, q=None):
    """``nsteps`` steps from p0; returns the list of fields after each step."""
    out, p = [], np.asarray(p0, dtype=np.float64)
    for _ in range(nsteps):
        p = step(tx, ty, tz, c, dmask, pd, p, wi, pw, q)
        out.append(p)
    return out


def step_residual_loops(p_new, p_old, tx, ty, tz, c, dmask, pd, wi=None, pw=None, q=None):
    """Residual of the step equation by explicit loops over cells and their six
    neighbours (pure Python, tiny grids only): on unknown cells
    ``c (p - p^n) + sum_L T (p_K - p_L) + WI (p - pw) - q``, and ``p - p^D`` on
    Dirichlet cells. Zero at the step's solution."""
    nx, ny, nz = np.shape(p_new)
    shape = (nx, ny, nz)
    cv, wv, pwv, qv = (_field(v, shape) for v in (c, wi, pw, q))
    r = np.zeros(shape)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                pk = p_new[i, j, k]
                if dmask[i, j, k]:
                    r[i, j, k] = pk - pd[i, j, k]
                    continue
                s = cv[i, j, k] * (pk - p_old[i, j, k]) + wv[i, j, k] * (pk - pwv[i, j, k]) - qv[i, j, k]
                for (ii, jj, kk) in ((i - 1, j, k), (i + 1, j, k), (i, j - 1, k),
                                     (i, j + 1, k), (i, j, k - 1), (i, j, k + 1)):
                    if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                        continue
                    if ii != i:
                        t = tx[min(i, ii), j, k]
                    elif jj != j:
                        t = ty[i, min(j, jj), k]
                    else:
                        t = tz[i, j, min(k, kk)]
                    s += t * (pk - p_new[ii, jj, kk])
                r[i, j, k] = s
    return r
