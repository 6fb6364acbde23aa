"""TPFA operator of the single-phase pressure system, assembled into CSR (FP64).

Test infrastructure only (see the package docstring).

Paper passages followed:

* Sec. II-A, Eq. 3: the constrained residual; rows of Dirichlet cells are
  ``p_K - p_K^D``, the others are the sum of the interface fluxes.
* Eq. 4: the TPFA flux ``f_KL = Upsilon_KL * lambda_KL * (p_L - p_K)``.
* Eq. 6 / Alg. 2: the Jacobian-vector product, sum of ``T_KL (x_L - x_K)`` over
  the six face neighbours on non-Dirichlet cells, ``x_K`` on Dirichlet cells.

Readings where the paper is silent or at odds with itself:

* Mobility is constant (lambda = 1), and ``T = Upsilon*lambda`` is the
  harmonic two-point transmissibility of unit cells, ``1/(1/(2k_K) + 1/(2k_L))``;
  the paper gives no formula for Upsilon.
* The interior rows of Eq. 6 are negative semi-definite while the text calls J
  SPD; the solved operator is ``A = -J`` on the unknown cells, plus an
  accumulation diagonal ``c`` (a backward-Euler storage term standing in for
  the time step; with c = 0 it is the paper's incompressible model).
* Dirichlet cells are eliminated symmetrically: their couplings move to the
  right-hand side ``b_K = sum_{L in D} T_KL p_L^D`` and their rows become the
  identity, so the full-grid operator is ``diag(A_UU, I_D)``, symmetric and
  positive definite.

Layout: arrays of shape (nx, ny, nz); face array ``Tx[i, j, k]`` is the face
between cells (i, j, k) and (i+1, j, k) and is zero on the last x plane
(likewise Ty on the last y row, Tz on the last z column).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def harmonic_face(k_a: np.ndarray, k_b: np.ndarray) -> np.ndarray:
    """Transmissibility of the face between two unit cells (series of two half cells).

    Each half cell has area 1 and length 1/2, so its conductance is 2k; the
    two half cells act in series.
    """
    return 1.0 / (1.0 / (2.0 * k_a) + 1.0 / (2.0 * k_b))


def transmissibility(k: np.ndarray, kz_ratio: float = 1.0):
    """Face transmissibilities (Tx, Ty, Tz), FP64, zero-padded beyond the domain.

    ``kz_ratio`` scales the permeability used for z faces (k_z = kz_ratio * k).
    """
    k = np.asarray(k, dtype=np.float64)
    tx = np.zeros_like(k)
    ty = np.zeros_like(k)
    tz = np.zeros_like(k)
    tx[:-1, :, :] = harmonic_face(k[:-1, :, :], k[1:, :, :])
    ty[:, :-1, :] = harmonic_face(k[:, :-1, :], k[:, 1:, :])
    kz = kz_ratio * k
    tz[:, :, :-1] = harmonic_face(kz[:, :, :-1], kz[:, :, 1:])
    return tx, ty, tz


def round_to_f32(*arrays):
    """Round FP64 arrays to FP32 once and return them as FP64 again."""
    out = tuple(np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrays)
    return out if len(out) > 1 else out[0]


def x_plane_dirichlet(shape, p_left: float = 1.0, p_right: float = 0.0):
    """Dirichlet set on the planes i = 0 and i = nx-1, with their pressures."""
    nx = shape[0]
    dmask = np.zeros(shape, dtype=bool)
    dmask[0] = True
    dmask[nx - 1] = True
    pd = np.zeros(shape, dtype=np.float64)
    pd[0] = p_left
    pd[nx - 1] = p_right
    return dmask, pd


def _face_pairs(shape):
    """Flat indices (K, L) of every interior face, grouped by axis x, y, z."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    return ((idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()),
            (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()),
            (idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()))


def assemble(tx, ty, tz, c, dmask, pd):
    """Full-grid operator and right-hand side.

    Returns ``(A, b)`` with ``A`` an n-by-n CSR matrix in FP64: on an unknown cell
    K its row is ``(c_K + sum_L T_KL) p_K - sum_{L unknown} T_KL p_L``; on a
    Dirichlet cell it is the identity. ``b_K = sum_{L in D} T_KL p_L^D`` on the
    unknown cells and ``p_K^D`` on Dirichlet cells. ``c`` is a scalar or an
    array of the grid's shape.
    """
    shape = np.shape(tx)
    n = int(np.prod(shape))
    d = np.asarray(dmask, dtype=bool).ravel()
    pdv = np.asarray(pd, dtype=np.float64).ravel()
    cv = np.broadcast_to(np.asarray(c, dtype=np.float64), shape).ravel()

    diag = np.where(d, 0.0, cv).astype(np.float64)
    rows, cols, vals = [], [], []
    b = np.zeros(n)
    for (K, L), t in zip(_face_pairs(shape), (tx[:-1, :, :], ty[:, :-1, :], tz[:, :, :-1])):
        t = np.asarray(t, dtype=np.float64).ravel()
        uK, uL = ~d[K], ~d[L]
        # diagonal: every face of an unknown cell adds its T
        np.add.at(diag, K[uK], t[uK])
        np.add.at(diag, L[uL], t[uL])
        # off-diagonals between two unknown cells
        both = uK & uL
        rows += [K[both], L[both]]
        cols += [L[both], K[both]]
        vals += [-t[both], -t[both]]
        # couplings to Dirichlet cells move to the right-hand side
        kd = uK & ~uL
        np.add.at(b, K[kd], t[kd] * pdv[L[kd]])
        ld = uL & ~uK
        np.add.at(b, L[ld], t[ld] * pdv[K[ld]])
    diag[d] = 1.0
    b[d] = pdv[d]
    all_idx = np.arange(n)
    rows.append(all_idx)
    cols.append(all_idx)
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A, b


def reduce_to_unknowns(A, b, dmask):
    """The unknown-cell block ``A_UU`` and ``b_U``, with the index map of U."""
    u = np.flatnonzero(~np.asarray(dmask, dtype=bool).ravel())
    return A[u][:, u].tocsr(), b[u], u


def scatter_solution(x_u, u, pd, dmask):
    """Full-grid pressure: ``x_u`` on the unknown cells, ``p^D`` on Dirichlet cells."""
    p = np.asarray(pd, dtype=np.float64).ravel().copy()
    p[u] = x_u
    return p


def relative_residual(A, b, x, dmask):
    """``||b - A x|| / ||b||`` over the unknown cells only, in FP64."""
    u = ~np.asarray(dmask, dtype=bool).ravel()
    r = (b - A @ np.asarray(x, dtype=np.float64).ravel())[u]
    nb = np.linalg.norm(b[u])
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))


def constrained_residual_loops(p, tx, ty, tz, c, dmask, pd):
    """Residual of Eq. 3 by explicit loops over cells and their neighbours.

    Interior rows: ``sum_L T_KL (p_L - p_K) - c_K p_K`` (the flux sum of Eq. 3/4,
    with the accumulation as a sink); Dirichlet rows: ``p_K - p_K^D``. Pure
    Python, for tiny grids only; its Jacobian is ``-A`` on unknown rows.
    """
    nx, ny, nz = np.shape(p)
    cv = np.broadcast_to(np.asarray(c, dtype=np.float64), (nx, ny, nz))
    r = np.zeros((nx, ny, nz))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                if dmask[i, j, k]:
                    r[i, j, k] = p[i, j, k] - pd[i, j, k]
                    continue
                s = -cv[i, j, k] * p[i, j, k]
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
                    s += t * (p[ii, jj, kk] - p[i, j, k])
                r[i, j, k] = s
    return r


def apply_stencil(tx, ty, tz, c, dmask, x):
    """Full-grid operator applied by array slicing, FP64 (no matrix).

    Same operator as :func:`assemble` (pinned against it on small grids), for
    grids too large to assemble: on unknown cells
    ``c_K x_K + sum_L T_KL (x_K - x_L)`` with ``x_L`` taken as 0 on Dirichlet
    cells, and ``x_K`` itself on Dirichlet cells.
    """
    d = np.asarray(dmask, dtype=bool)
    x = np.asarray(x, dtype=np.float64).reshape(d.shape)
    xu = np.where(d, 0.0, x)                  # Dirichlet values leave the unknowns' rows
    y = np.broadcast_to(np.asarray(c, dtype=np.float64), d.shape) * x
    y = np.array(y, dtype=np.float64)
    for axis, t in ((0, tx), (1, ty), (2, tz)):
        t = np.asarray(t, dtype=np.float64)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        tf = t[lo]
        y[lo] += tf * (x[lo] - xu[hi])        # face seen from the lower cell
        y[hi] += tf * (x[hi] - xu[lo])        # the same face seen from the upper cell
    return np.where(d, x, y)
