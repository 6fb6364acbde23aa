"""Pins of the oracle's Krylov solvers: textbook CG invariants, library and
direct-solve cross-checks, special cases of PCG/FCG, and the refinement bound."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import tpfa, krylov
from synth import lognormal_iid

HERE = os.path.dirname(os.path.abspath(__file__))


def system(shape, sigma=1.0, seed=0, c=1e-3, kz_ratio=1.0):
    k = lognormal_iid(shape, sigma, seed)
    tx, ty, tz = tpfa.transmissibility(k, kz_ratio)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    A, b = tpfa.assemble(tx, ty, tz, c, dmask, pd)
    return tpfa.reduce_to_unknowns(A, b, dmask)


def test_cg_matches_dense_solve_4cube():
    Auu, bu, _ = system((4, 4, 4))
    res = krylov.cg(Auu, bu, tol=1e-13, max_iter=200)
    x = np.linalg.solve(Auu.toarray(), bu)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= 1e-12 * np.linalg.norm(x)
    # finite termination: at most n_U steps (plus a few for rounding)
    assert res.iters <= Auu.shape[0] + 3


def test_cg_orthogonality_and_monotone_energy_error():
    Auu, bu, _ = system((5, 4, 3), sigma=1.0, seed=2)
    xs = np.linalg.solve(Auu.toarray(), bu)
    rs, ps, errs = [bu.copy()], [], []

    def cb(k, x, r, p):
        rs.append(r.copy())
        ps.append(p.copy())
        e = xs - x
        errs.append(e @ (Auu @ e))

    krylov.cg(Auu, bu, tol=1e-10, max_iter=8, callback=cb)
    R = np.array(rs[:6])
    G = R @ R.T
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-10 * np.max(np.diag(G))
    P = np.array(ps[:5])
    H = P @ (Auu @ P.T)
    offh = H - np.diag(np.diag(H))
    assert np.max(np.abs(offh)) < 1e-10 * np.max(np.diag(H))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


def test_cg_matches_scipy_cg():
    Auu, bu, _ = system((12, 10, 8), sigma=1.0, seed=5)
    ours = krylov.cg(Auu, bu, tol=1e-8, max_iter=2000)
    count = [0]
    xs, info = spla.cg(Auu, bu, rtol=1e-8, atol=0.0, maxiter=2000,
                       callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0 and ours.converged
    assert abs(ours.iters - count[0]) <= 1
    assert np.linalg.norm(ours.x - xs) <= 1e-7 * np.linalg.norm(xs)
    # recursive and true residual agree in FP64
    true = np.linalg.norm(bu - Auu @ ours.x) / np.linalg.norm(bu)
    assert abs(true - ours.rel_res) < 1e-12


def test_pcg_special_cases():
    Auu, bu, _ = system((6, 5, 4), sigma=2.0, seed=8)
    plain = krylov.cg(Auu, bu, tol=1e-10, max_iter=1000)
    ident = krylov.pcg(Auu, bu, lambda r: r.copy(), tol=1e-10, max_iter=1000)
    assert plain.iters == ident.iters
    assert np.allclose(plain.history, ident.history, rtol=1e-12, atol=0)
    # Jacobi-PCG converges to the direct solution, in fewer steps on a rough field
    jac = krylov.pcg(Auu, bu, krylov.jacobi(Auu), tol=1e-10, max_iter=1000)
    xs = np.linalg.solve(Auu.toarray(), bu)
    assert np.linalg.norm(jac.x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert jac.iters < plain.iters
    # FCG with a fixed SPD preconditioner is PCG: the two beta formulas agree in
    # exact arithmetic; in FP64 the Krylov recurrences amplify rounding, so the
    # first iterates agree to rounding and the converged solutions agree
    for M, ref in ((lambda r: r.copy(), plain), (krylov.jacobi(Auu), jac)):
        f = krylov.fcg(Auu, bu, M, tol=1e-10, max_iter=1000)
        assert f.converged
        assert np.allclose(f.history[:12], ref.history[:12], rtol=1e-10, atol=0)
        assert np.linalg.norm(f.x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_fcg_tolerates_a_varying_preconditioner():
    # a preconditioner that changes every call (random SPD diagonal scalings)
    Auu, bu, _ = system((6, 6, 6), sigma=1.5, seed=4)
    rng = np.random.default_rng(0)
    d = Auu.diagonal()
    M = lambda r: r / d * rng.uniform(0.5, 1.5, r.size)  # noqa: E731
    res = krylov.fcg(Auu, bu, M, tol=1e-10, max_iter=2000)
    xs = np.linalg.solve(Auu.toarray(), bu)
    assert res.converged
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_breakdown_on_indefinite_operator():
    Auu, bu, _ = system((4, 3, 3))
    res = krylov.cg(-Auu, bu, tol=1e-10, max_iter=100)
    assert res.status == "breakdown" and not res.converged


def test_iterative_refinement_reaches_fp64_accuracy():
    Auu, bu, _ = system((16, 16, 16), sigma=2.0, seed=1)
    xs = spla.spsolve(Auu.tocsc(), bu)
    single = krylov.cg(Auu.astype(np.float32), bu.astype(np.float32), tol=1e-6,
                       max_iter=5000, dtype=np.float32)
    true32 = np.linalg.norm(bu - Auu @ single.x.astype(np.float64)) / np.linalg.norm(bu)
    ir = krylov.iterative_refinement(Auu, bu, tol=1e-10, inner_tol=1e-4)
    assert ir.converged and ir.outer >= 2
    true_ir = np.linalg.norm(bu - Auu @ ir.x) / np.linalg.norm(bu)
    assert true_ir <= 1e-10 < true32
    assert np.linalg.norm(ir.x - xs) <= 1e-8 * np.linalg.norm(xs)
    # each outer step reduces the FP64 residual by about the inner tolerance
    h = ir.history
    assert all(b2 < 1e-3 * b1 for b1, b2 in zip(h, h[1:]))


def test_cell_iteration_throughput_reproduces_the_paper_table():
    # cells * iterations / seconds reproduces the printed Gcell/s of the weak
    # scaling table (apply-only and full-CG columns) within 0.5 %: the printed
    # times carry three significant digits (0.0122 s is only known to 0.4 %)
    rows = np.loadtxt(os.path.join(HERE, "golden", "table3_weak_scaling.txt"))
    cells, steps = rows[:, 3], rows[:, 4]
    assert np.all(cells == rows[:, 0] * rows[:, 1] * rows[:, 2])
    for thr_col, t_col in ((5, 6), (8, 9)):
        rate = cells * steps / rows[:, t_col] / 1e9
        assert np.all(np.abs(rate / rows[:, thr_col] - 1) < 5e-3)
