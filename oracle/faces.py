"""TPFA operator on a face-list (unstructured) mesh, assembled into CSR (FP64).

Test infrastructure only (see the package docstring).

Paper passages followed:

* Sec. II-A, Eq. 3 and 4: the residual of an unknown cell sums the TPFA
  fluxes ``T_KL (p_L - p_K)`` over the cell's faces; Dirichlet rows are
  ``p_K - p_K^D``.
* Sec. VI names arbitrary mesh topologies as the next step; nothing in Eq. 3-4
  depends on the faces forming a Cartesian grid.

Readings: a face ``f`` joins two different cells ``k_f``, ``l_f`` with
``T_f = Upsilon_f lambda_f``; faces repeated between the same two cells add up.
The elimination of Dirichlet cells, the accumulation and the right-hand side
are those of ``tpfa.assemble``: on an unknown cell K the row is
``(c_K + sum_f T_f) p_K - sum_{f: L unknown} T_f p_L``, and
``b_K = sum_{f: L Dirichlet} T_f p_L^D``; Dirichlet rows are the identity.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble_faces(n, face_k, face_l, T, c, dmask, pd):
    """Full operator (n x n CSR, FP64) and right-hand side of a face-list mesh.
    ``c`` is a scalar or an array of n; ``dmask``/``pd`` arrays of n."""
    K = np.asarray(face_k, dtype=np.int64)
    L = np.asarray(face_l, dtype=np.int64)
    t = np.asarray(T, dtype=np.float64)
    d = np.asarray(dmask, dtype=bool).ravel()
    pdv = np.asarray(pd, dtype=np.float64).ravel()
    cv = np.broadcast_to(np.asarray(c, dtype=np.float64), (n,))
    uK, uL = ~d[K], ~d[L]
    diag = np.where(d, 0.0, cv).astype(np.float64)
    np.add.at(diag, K[uK], t[uK])
    np.add.at(diag, L[uL], t[uL])
    both = uK & uL
    rows = np.concatenate([K[both], L[both], np.arange(n)])
    cols = np.concatenate([L[both], K[both], np.arange(n)])
    b = np.zeros(n)
    kd = uK & ~uL
    np.add.at(b, K[kd], t[kd] * pdv[L[kd]])
    ld = uL & ~uK
    np.add.at(b, L[ld], t[ld] * pdv[K[ld]])
    diag[d] = 1.0
    b[d] = pdv[d]
    vals = np.concatenate([-t[both], -t[both], diag])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A, b


def residual_loops(p, n, face_k, face_l, T, c, dmask, pd):
    """Residual of Eq. 3 by a loop over faces (pure Python, small meshes):
    unknown rows ``sum_f T_f (p_L - p_K) - c_K p_K``, Dirichlet rows
    ``p_K - p_K^D``. Its Jacobian is ``-A`` on unknown rows."""
    cv = np.broadcast_to(np.asarray(c, dtype=np.float64), (n,))
    r = -cv * np.asarray(p, dtype=np.float64)
    for k, l, t in zip(face_k, face_l, T):
        r[k] += t * (p[l] - p[k])
        r[l] += t * (p[k] - p[l])
    d = np.asarray(dmask, dtype=bool)
    r[d] = p[d] - np.asarray(pd, dtype=np.float64)[d]
    return r
