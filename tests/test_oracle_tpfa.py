"""Pins of the oracle's TPFA operator against closed forms, invariants and brute force.

Each test checks the oracle against something other than itself: an analytic
pressure profile, a property the operator must have (symmetry, positive
definiteness, row sums, maximum principle, flux balance), a dense direct solve,
or the Jacobian of the constrained residual (Sec. II-A, Eq. 3 and 4) computed by
explicit loops over cells and neighbours.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import tpfa
from synth import lognormal_iid


def solve_direct(k, c, kz_ratio=1.0):
    tx, ty, tz = tpfa.transmissibility(k, kz_ratio)
    dmask, pd = tpfa.x_plane_dirichlet(k.shape)
    A, b = tpfa.assemble(tx, ty, tz, c, dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, b, dmask)
    xu = spla.spsolve(Auu.tocsc(), bu)
    return tpfa.scatter_solution(xu, u, pd, dmask).reshape(k.shape), (A, b, dmask, tx, ty, tz)


def test_face_transmissibility_special_cases():
    # equal permeabilities: two half cells of conductance 2k in series give k
    k = np.array([0.3, 1.0, 7.5, 1e3])
    assert np.allclose(tpfa.harmonic_face(k, k), k, rtol=1e-15)
    # a blocked half cell blocks the face; a huge contrast is limited by the smaller k
    assert tpfa.harmonic_face(np.array([1.0]), np.array([1e-300]))[0] < 1e-299
    assert np.isclose(tpfa.harmonic_face(np.array([1.0]), np.array([1e12]))[0], 2.0, rtol=1e-11)
    # padding and anisotropy: last plane zero, z faces scale with kz_ratio
    kk = lognormal_iid((3, 4, 5), 1.0, 7)
    tx, ty, tz = tpfa.transmissibility(kk, kz_ratio=0.1)
    assert np.all(tx[-1] == 0) and np.all(ty[:, -1] == 0) and np.all(tz[:, :, -1] == 0)
    _, _, tz1 = tpfa.transmissibility(kk, kz_ratio=1.0)
    assert np.allclose(tz, 0.1 * tz1, rtol=1e-14)


@pytest.mark.parametrize("kval", [1.0, 3.7])
def test_linear_profile_homogeneous(kval):
    # c = 0, homogeneous k: p_i = 1 - i/(nx-1), independent of (j, k)
    shape = (8, 3, 2)
    p, _ = solve_direct(np.full(shape, kval), 0.0)
    expect = 1.0 - np.arange(shape[0]) / (shape[0] - 1)
    assert np.max(np.abs(p - expect[:, None, None])) < 1e-14


@pytest.mark.parametrize("c", [1e-3, 0.05, 0.7])
def test_sinh_profile_with_accumulation(c):
    # k = 1 (T = 1), c > 0: p_{i+1} - (2+c) p_i + p_{i-1} = 0 with p_0 = 1, p_{nx-1} = 0
    # => p_i = sinh(theta (nx-1-i)) / sinh(theta (nx-1)), cosh(theta) = 1 + c/2
    shape = (11, 2, 3)
    p, _ = solve_direct(np.ones(shape), c)
    theta = np.arccosh(1.0 + c / 2.0)
    i = np.arange(shape[0])
    expect = np.sinh(theta * (shape[0] - 1 - i)) / np.sinh(theta * (shape[0] - 1))
    assert np.max(np.abs(p - expect[:, None, None])) < 1e-13


def test_x_layered_series_flux():
    # k depends on i only, c = 0: one flux q crosses every face; the face
    # resistance is the sum of the two half-cell resistances 1/(2k)
    rng = np.random.default_rng(3)
    nx = 9
    kx = np.exp(rng.normal(size=nx))
    k = np.broadcast_to(kx[:, None, None], (nx, 2, 3)).copy()
    p, _ = solve_direct(k, 0.0)
    R = 1.0 / (2 * kx[:-1]) + 1.0 / (2 * kx[1:])
    q = 1.0 / R.sum()
    expect = 1.0 - q * np.concatenate([[0.0], np.cumsum(R)])
    assert np.max(np.abs(p - expect[:, None, None])) < 1e-14


def test_yz_layered_linear_columns():
    # k depends on (j, k) only, c = 0: every (j, k) column is exactly linear in i
    rng = np.random.default_rng(4)
    nx, ny, nz = 7, 4, 5
    kyz = np.exp(2 * rng.normal(size=(ny, nz)))
    p, _ = solve_direct(np.broadcast_to(kyz, (nx, ny, nz)).copy(), 0.0)
    expect = 1.0 - np.arange(nx) / (nx - 1)
    assert np.max(np.abs(p - expect[:, None, None])) < 1e-13


def test_symmetry_and_spd():
    k = lognormal_iid((4, 4, 4), 2.0, 11)
    _, (A, b, dmask, *_) = solve_direct(k, 1e-3, kz_ratio=0.3)
    D = A.toarray()
    assert np.array_equal(D, D.T)
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=(2, D.shape[0]))
    lhs, rhs = x @ (A @ y), y @ (A @ x)
    assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + np.abs(x) @ (abs(A) @ np.abs(y)))
    assert np.linalg.eigvalsh(D).min() > 0
    # identity rows on Dirichlet cells, no coupling into them
    d = dmask.ravel()
    assert np.array_equal(D[d][:, d], np.eye(d.sum()))
    assert np.all(D[d][:, ~d] == 0) and np.all(D[~d][:, d] == 0)


def test_row_sums():
    shape = (5, 4, 3)
    k = lognormal_iid(shape, 1.5, 5)
    tx, ty, tz = tpfa.transmissibility(k)
    none = np.zeros(shape, dtype=bool)
    # no Dirichlet cells, c = 0: constants are in the kernel, A 1 = 0 exactly
    A0, _ = tpfa.assemble(tx, ty, tz, 0.0, none, np.zeros(shape))
    assert np.max(np.abs(A0 @ np.ones(A0.shape[0]))) < 1e-13
    # with accumulation: A 1 = c
    cfield = np.random.default_rng(1).uniform(1e-4, 1e-2, shape)
    Ac, _ = tpfa.assemble(tx, ty, tz, cfield, none, np.zeros(shape))
    assert np.allclose(Ac @ np.ones(Ac.shape[0]), cfield.ravel(), rtol=0, atol=1e-13)
    # with Dirichlet p^D = 1 on both planes and c = 0: p = 1 solves the system
    dmask, _ = tpfa.x_plane_dirichlet(shape)
    A1, b1 = tpfa.assemble(tx, ty, tz, 0.0, dmask, np.ones(shape))
    assert np.max(np.abs(A1 @ np.ones(A1.shape[0]) - b1)) < 1e-13


def test_jacobian_of_constrained_residual_brute_force():
    # The residual of Eq. 3 (flux sum with Eq. 4, accumulation as a sink) is affine
    # in p, so its Jacobian columns are exact finite differences. On unknown rows
    # it must equal -A_UU, and its value at p = (0 on U, p^D on D) must be b_U.
    shape = (4, 3, 2)
    rng = np.random.default_rng(9)
    k = np.exp(rng.normal(size=shape))
    c = rng.uniform(0, 0.1, shape)
    tx, ty, tz = tpfa.transmissibility(k, kz_ratio=0.5)
    dmask, pd = tpfa.x_plane_dirichlet(shape, 1.3, -0.4)
    A, b = tpfa.assemble(tx, ty, tz, c, dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, b, dmask)
    p0 = np.where(dmask, pd, 0.0)
    r0 = tpfa.constrained_residual_loops(p0, tx, ty, tz, c, dmask, pd).ravel()
    assert np.allclose(r0[u], bu, rtol=0, atol=1e-14)
    n = int(np.prod(shape))
    J = np.zeros((n, n))
    for j in range(n):
        pj = p0.ravel().copy()
        pj[j] += 1.0
        J[:, j] = tpfa.constrained_residual_loops(pj.reshape(shape), tx, ty, tz, c, dmask, pd).ravel() - r0
    assert np.allclose(-J[np.ix_(u, u)], Auu.toarray(), rtol=0, atol=1e-13)
    # Dirichlet rows of the residual are p_K - p_K^D: identity Jacobian
    d = np.flatnonzero(dmask.ravel())
    assert np.allclose(J[np.ix_(d, d)], np.eye(d.size))


def test_maximum_principle_and_flux_balance():
    shape = (10, 6, 5)
    k = lognormal_iid(shape, 2.0, 21)
    p, (A, b, dmask, tx, ty, tz) = solve_direct(k, 0.0)
    assert p.min() >= -1e-12 and p.max() <= 1 + 1e-12
    flux_in = np.sum(tx[0] * (p[0] - p[1]))
    flux_out = np.sum(tx[-2] * (p[-2] - p[-1]))
    assert flux_in > 0
    assert abs(flux_in - flux_out) < 1e-12 * flux_in
    p2, _ = solve_direct(k, 1e-2)
    assert p2.min() >= -1e-12 and p2.max() <= 1 + 1e-12
    # accumulation is a sink: it lowers the pressure everywhere inside
    assert np.all(p2[1:-1] <= p[1:-1] + 1e-12)


def test_dense_solve_4cube_and_relative_residual():
    k = lognormal_iid((4, 4, 4), 1.0, 0)
    tx, ty, tz = tpfa.transmissibility(k)
    dmask, pd = tpfa.x_plane_dirichlet(k.shape)
    A, b = tpfa.assemble(tx, ty, tz, 1e-3, dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, b, dmask)
    assert Auu.shape == (32, 32)
    xu = np.linalg.solve(Auu.toarray(), bu)
    p = tpfa.scatter_solution(xu, u, pd, dmask)
    assert tpfa.relative_residual(A, b, p, dmask) < 1e-15
    # the full-grid system has the same solution (identity rows carry p^D)
    assert np.allclose(np.linalg.solve(A.toarray(), b), p, rtol=0, atol=1e-14)


def test_slicing_apply_matches_assembled_operator():
    shape = (6, 5, 7)
    rng = np.random.default_rng(12)
    k = lognormal_iid(shape, 2.0, 13)
    tx, ty, tz = tpfa.transmissibility(k, kz_ratio=0.25)
    c = rng.uniform(0, 1e-2, shape)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    dmask[2, 1, 3] = True          # an interior Dirichlet cell as well
    A, _ = tpfa.assemble(tx, ty, tz, c, dmask, pd)
    for _ in range(3):
        x = rng.normal(size=shape)
        y = tpfa.apply_stencil(tx, ty, tz, c, dmask, x).ravel()
        assert np.allclose(y, A @ x.ravel(), rtol=1e-14, atol=1e-14)
