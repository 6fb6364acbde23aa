"""Seeded face-list meshes (topology and per-face coefficients only).

A face-list mesh is n cells and faces (k, l) joining two of them. These
generators shape random numbers into such meshes; they hold none of the
solver's arithmetic.
"""
from __future__ import annotations

import numpy as np


def cartesian_faces(shape):
    """The faces of a Cartesian grid, in x, y, z order, as flat cell indices
    (z fastest): returns (face_k, face_l, axis) with face_k the lower cell."""
    idx = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape)
    ks, ls, ax = [], [], []
    for a, (lo, hi) in enumerate(((idx[:-1, :, :], idx[1:, :, :]),
                                  (idx[:, :-1, :], idx[:, 1:, :]),
                                  (idx[:, :, :-1], idx[:, :, 1:]))):
        ks.append(lo.ravel())
        ls.append(hi.ravel())
        ax.append(np.full(lo.size, a, dtype=np.int8))
    return np.concatenate(ks), np.concatenate(ls), np.concatenate(ax)


def random_face_mesh(shape, seed: int, drop: float = 0.1, extra: float = 0.05, sigma: float = 1.0):
    """An irregular mesh: the faces of a Cartesian grid with a fraction
    ``drop`` removed, ``extra`` x (number of cells) faces added between random
    cell pairs (repeated pairs allowed), cells renumbered by a random
    permutation, and a log-normal transmissibility per face.
    Returns (n, face_k, face_l, T) with int32 indices and FP64 T."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    fk, fl, _ = cartesian_faces(shape)
    keep = rng.random(fk.size) >= drop
    fk, fl = fk[keep], fl[keep]
    ne = int(extra * n)
    ek = rng.integers(0, n, ne)
    el = rng.integers(0, n - 1, ne)
    el = np.where(el >= ek, el + 1, el)          # never a self-face
    fk = np.concatenate([fk, ek])
    fl = np.concatenate([fl, el])
    perm = rng.permutation(n)
    fk, fl = perm[fk], perm[fl]
    T = np.exp(sigma * rng.standard_normal(fk.size))
    return n, fk.astype(np.int32), fl.astype(np.int32), T
