"""Pins of the oracle's face-list operator: a Cartesian grid written as a face
list gives the Cartesian oracle's operator exactly (also renumbered), the
residual of Eq. 3 by a loop over faces has it as its Jacobian, and on an
irregular mesh it is symmetric, an M-matrix and positive definite with the
row sums the accumulation and the Dirichlet faces fix."""
import numpy as np

from oracle import faces, tpfa
from synth import cartesian_faces, lognormal_iid, random_face_mesh


def cartesian_as_faces(k):
    tx, ty, tz = tpfa.transmissibility(k, 0.3)
    fk, fl, ax = cartesian_faces(k.shape)
    flat = [t.ravel() for t in (tx, ty, tz)]
    T = np.where(ax == 0, flat[0][fk], np.where(ax == 1, flat[1][fk], flat[2][fk]))
    return (tx, ty, tz), fk, fl, T


def test_cartesian_face_list_gives_the_cartesian_operator():
    shape = (6, 5, 4)
    k = lognormal_iid(shape, 1.0, 11)
    (tx, ty, tz), fk, fl, T = cartesian_as_faces(k)
    dmask, pd = tpfa.x_plane_dirichlet(shape, 1.5, -0.5)
    c = np.random.default_rng(1).uniform(0.0, 0.3, shape)
    A1, b1 = tpfa.assemble(tx, ty, tz, c, dmask, pd)
    n = k.size
    A2, b2 = faces.assemble_faces(n, fk, fl, T, c.ravel(), dmask.ravel(), pd.ravel())
    # the same terms, summed in another order on the diagonal
    tol = 1e-14 * abs(A1).max()
    assert abs(A1 - A2).max() <= tol and np.allclose(b1, b2, rtol=1e-15, atol=0)
    # renumbered cells: P A P^T and P b
    perm = np.random.default_rng(2).permutation(n)
    A3, b3 = faces.assemble_faces(n, perm[fk], perm[fl], T, c.ravel()[np.argsort(perm)],
                                  dmask.ravel()[np.argsort(perm)], pd.ravel()[np.argsort(perm)])
    assert abs(A3[perm][:, perm] - A1).max() <= tol and np.allclose(b3[perm], b1, rtol=1e-15, atol=0)


def test_face_loop_residual_has_minus_A_as_jacobian():
    n, fk, fl, T = random_face_mesh((4, 3, 3), 5, drop=0.2, extra=0.3)
    rng = np.random.default_rng(3)
    c = rng.uniform(0.0, 0.5, n)
    dmask = np.zeros(n, dtype=bool)
    dmask[rng.choice(n, 4, replace=False)] = True
    pd = np.where(dmask, rng.uniform(-1, 1, n), 0.0)
    A, b = faces.assemble_faces(n, fk, fl, T, c, dmask, pd)
    p = np.where(dmask, pd, rng.standard_normal(n))
    r = faces.residual_loops(p, n, fk, fl, T, c, dmask, pd)
    u = ~dmask
    # on unknown rows the residual is b - A p (Dirichlet couplings on the right)
    assert np.allclose(r[u], (b - A @ p)[u], rtol=1e-13, atol=1e-13)
    # brute-force Jacobian of the loop residual over the unknown cells
    J = np.zeros((n, n))
    for j in np.flatnonzero(u):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = faces.residual_loops(p + e, n, fk, fl, T, c, dmask, pd) - r
    Ad = A.toarray()
    assert np.allclose(J[np.ix_(u, u)], -Ad[np.ix_(u, u)], atol=1e-12)


def test_irregular_mesh_operator_properties():
    n, fk, fl, T = random_face_mesh((7, 6, 5), 9, drop=0.15, extra=0.1)
    rng = np.random.default_rng(4)
    c = rng.uniform(0.0, 0.1, n)
    dmask = np.zeros(n, dtype=bool)
    dmask[rng.choice(n, 12, replace=False)] = True
    pd = np.where(dmask, 1.0, 0.0)
    A, b = faces.assemble_faces(n, fk, fl, T, c, dmask, pd)
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    off = Ad - np.diag(np.diag(Ad))
    assert np.all(off <= 0)
    u = ~dmask
    Auu = Ad[np.ix_(u, u)]
    assert np.linalg.eigvalsh(Auu).min() > 0
    # row sums of A_UU: accumulation plus the faces to Dirichlet cells
    to_d = np.zeros(n)
    for k, l, t in zip(fk, fl, T):
        if u[k] and dmask[l]:
            to_d[k] += t
        if u[l] and dmask[k]:
            to_d[l] += t
    assert np.allclose(Auu.sum(axis=1), (c + to_d)[u], rtol=1e-12, atol=1e-14)
    assert np.allclose(b[u], to_d[u] * 1.0, rtol=1e-12)      # p^D = 1 on every Dirichlet cell
    assert np.array_equal(b[dmask], pd[dmask])


def test_repeated_faces_add_up():
    n, fk, fl, T = random_face_mesh((3, 3, 2), 2)
    d = np.zeros(n, dtype=bool)
    d[0] = True
    pd = np.where(d, 2.0, 0.0)
    A1, b1 = faces.assemble_faces(n, fk, fl, T, 0.1, d, pd)
    A2, b2 = faces.assemble_faces(n, np.concatenate([fk, fk]), np.concatenate([fl, fl]),
                                  np.concatenate([T, T]) / 2.0, 0.1, d, pd)
    assert abs(A1 - A2).max() < 1e-14 and np.allclose(b1, b2, rtol=1e-14)
