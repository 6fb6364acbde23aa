"""Pins of the oracle's backward-Euler time stepping with wells.

The step equation (storage, TPFA fluxes at the new time level, implicit
Peaceman-form wells and rate sources; Sec. II-A with Eq. 3-5) is checked
against: its residual written out by loops over cells and neighbours, the
closed-form decay of a discrete Laplacian eigenmode, the steady state as a
fixed point, and the discrete mass balance.
"""
import numpy as np

from oracle import timestep, tpfa
from synth import lognormal_iid


def problem(shape, seed):
    rng = np.random.default_rng(seed)
    k = lognormal_iid(shape, 1.0, seed)
    tx, ty, tz = tpfa.transmissibility(k, 0.5)
    dmask, pd = tpfa.x_plane_dirichlet(shape, 2.0, 0.5)
    c = rng.uniform(0.05, 0.5, shape)
    wi = np.zeros(shape)
    pw = np.zeros(shape)
    wi[1, 0, 0], pw[1, 0, 0] = 3.0, 5.0          # injector (pw above the field)
    wi[-2, -1, -1], pw[-2, -1, -1] = 2.0, -1.0   # producer
    q = np.zeros(shape)
    q[shape[0] // 2, 1, 1] = 0.75
    p0 = rng.uniform(0.0, 2.0, shape)
    p0[dmask] = pd[dmask]
    return tx, ty, tz, c, dmask, pd, wi, pw, q, p0


def test_step_satisfies_the_step_equation_by_loops():
    tx, ty, tz, c, dmask, pd, wi, pw, q, p0 = problem((6, 4, 3), 1)
    p1 = timestep.step(tx, ty, tz, c, dmask, pd, p0, wi, pw, q)
    r = timestep.step_residual_loops(p1, p0, tx, ty, tz, c, dmask, pd, wi, pw, q)
    assert np.max(np.abs(r)) < 1e-11 * (1 + np.max(np.abs(p1)))
    # the same field does not satisfy a step with the well or the source dropped
    r_nowell = timestep.step_residual_loops(p1, p0, tx, ty, tz, c, dmask, pd, None, None, q)
    r_noq = timestep.step_residual_loops(p1, p0, tx, ty, tz, c, dmask, pd, wi, pw, None)
    assert np.max(np.abs(r_nowell)) > 0.1 and np.max(np.abs(r_noq)) > 0.1


def test_eigenmode_decays_by_the_closed_form_factor():
    """Homogeneous unit cells (T = 1), p^D = 0 on both x planes, uniform c: the
    x profile sin(pi i / (nx - 1)) is an eigenvector of the 1D Dirichlet
    Laplacian on the nx - 2 unknown planes with eigenvalue
    2 (1 - cos(pi / (nx - 1))), so each step multiplies it by c / (c + lambda)."""
    shape = (9, 3, 2)
    k = np.ones(shape)
    tx, ty, tz = tpfa.transmissibility(k)
    dmask, pd = tpfa.x_plane_dirichlet(shape, 0.0, 0.0)
    c = 0.7
    i = np.arange(shape[0])
    p0 = np.broadcast_to(np.sin(np.pi * i / (shape[0] - 1))[:, None, None], shape).copy()
    lam = 2.0 * (1.0 - np.cos(np.pi / (shape[0] - 1)))
    steps = timestep.run(tx, ty, tz, c, dmask, pd, p0, 4)
    for s, p in enumerate(steps, start=1):
        assert np.allclose(p, p0 * (c / (c + lam)) ** s, rtol=1e-12, atol=1e-14), s


def test_steady_state_is_a_fixed_point():
    """The steady field solves (A_T + WI) p = b + WI pw + q; a step from it
    returns it, whatever the storage."""
    tx, ty, tz, c, dmask, pd, wi, pw, q, _ = problem((7, 5, 4), 2)
    import scipy.sparse.linalg as spla
    A, b = tpfa.assemble(tx, ty, tz, wi, dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, b, dmask)
    rhs = (b + (wi * pw + q).ravel())[u]
    ps = tpfa.scatter_solution(spla.spsolve(Auu.tocsc(), rhs), u, pd, dmask).reshape(dmask.shape)
    p1 = timestep.step(tx, ty, tz, c, dmask, pd, ps, wi, pw, q)
    assert np.allclose(p1, ps, rtol=1e-11, atol=1e-12)
    # and a run from elsewhere approaches it
    p0 = np.where(dmask, pd, 0.0)
    last = timestep.run(tx, ty, tz, 0.05, dmask, pd, p0, 60, wi, pw, q)[-1]
    assert np.max(np.abs(last - ps)) < 1e-6 * np.max(np.abs(ps))


def boundary_inflow(p, tx, ty, tz, dmask, pd):
    """Sum over faces between a Dirichlet and an unknown cell of T (p^D - p_U)."""
    tot = 0.0
    for t, sl_a, sl_b in ((tx, np.s_[:-1, :, :], np.s_[1:, :, :]),
                          (ty, np.s_[:, :-1, :], np.s_[:, 1:, :]),
                          (tz, np.s_[:, :, :-1], np.s_[:, :, 1:])):
        tf = t[sl_a]
        da, db = dmask[sl_a], dmask[sl_b]
        pa, pb = p[sl_a], p[sl_b]
        tot += np.sum(np.where(da & ~db, tf * (pd[sl_a] - pb), 0.0))
        tot += np.sum(np.where(db & ~da, tf * (pd[sl_b] - pa), 0.0))
    return tot


def test_discrete_mass_balance():
    """Storage change = sources + well inflow + inflow across the Dirichlet
    faces: the interior fluxes cancel pairwise."""
    tx, ty, tz, c, dmask, pd, wi, pw, q, p0 = problem((8, 5, 3), 3)
    p1 = timestep.step(tx, ty, tz, c, dmask, pd, p0, wi, pw, q)
    u = ~dmask
    storage = np.sum((c * (p1 - p0))[u])
    inflow = np.sum(q[u]) + np.sum((wi * (pw - p1))[u]) + boundary_inflow(p1, tx, ty, tz, dmask, pd)
    assert abs(storage - inflow) < 1e-10 * (1 + abs(storage))


def test_step_rhs_definition():
    tx, ty, tz, c, dmask, pd, wi, pw, q, p0 = problem((5, 3, 2), 4)
    _, b = tpfa.assemble(tx, ty, tz, c + wi, dmask, pd)
    rhs = timestep.step_rhs(b, c, p0, dmask, wi, pw, q)
    bb = b.reshape(dmask.shape)
    assert np.array_equal(rhs[dmask], pd[dmask])
    u = ~dmask
    assert np.allclose(rhs[u], (bb + c * p0 + wi * pw + q)[u], rtol=1e-15)
    # scalar storage and no wells
    r2 = timestep.step_rhs(b, 0.3, p0, dmask)
    assert np.allclose(r2[u], (bb + 0.3 * p0)[u], rtol=1e-15)
