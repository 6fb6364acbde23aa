"""Batched persistent CG against the oracle: per-system fields and residuals."""
import numpy as np
import pytest

from oracle import krylov, tpfa
from synth import batch_systems, lognormal_iid
from gpu_problem import gpu_problem, OracleProblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available()
    mffv.lib()
    return mffv


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def small_batch(seed, n=7):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        shape = tuple(int(v) for v in rng.integers(3, 23, 3))
        shape = (max(shape[0], 3),) + shape[1:]
        out.append((shape, lognormal_iid(shape, 1.5, 100 + s), float(10 ** rng.uniform(-4, -2))))
    return out


@pytest.mark.parametrize("precond", [0, 1])
def test_batched_matches_oracle(mf, precond):
    """MFFV_FP32: one FP32 pass per system to the recursive 1e-6, iteration
    counts like the oracle's FP32 CG, the FP64 true residual of the returned
    field reported."""
    systems = small_batch(3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, precond=precond))
    torch.cuda.synchronize()
    assert st == mf.OK
    for (shape, k, c), x, info in zip(systems, xs, infos):
        ref = OracleProblem(k, c=c)
        assert info["status"] == mf.OK and info["rel_res_recursive"] <= 1e-6 and info["ir_steps"] == 1
        M = krylov.jacobi(ref.Auu) if precond else None
        orc = krylov.pcg(ref.Auu.astype(np.float32), ref.bu.astype(np.float32), M, tol=1e-6,
                         max_iter=20000, dtype=np.float32)
        assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 10), (shape, info, orc.iters)
        p = ref.direct()
        xh = host(x)
        assert np.linalg.norm(xh - p) <= 5e-5 * np.linalg.norm(p), shape
        assert abs(info["rel_res_true"] - ref.rel_residual(xh)) <= 1e-2 * info["rel_res_true"] + 1e-10
        assert np.array_equal(xh.reshape(shape)[0], np.ones(shape[1:]))   # Dirichlet values


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("single_reduction", [0, 1])
def test_batched_refinement_meets_the_true_residual(mf, precond, single_reduction):
    """MFFV_FP32_IR: every system's FP64 true residual (of the returned FP32
    field, recomputed by the oracle) is <= 1e-6 and the field is within 1e-5
    of the direct solution; a nonzero initial guess is used as given."""
    systems = small_batch(13)
    systems[1] = ((30, 26, 28), lognormal_iid((30, 26, 28), 2.0, 9), 1e-4)   # harder: more drift
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]
        xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
        xs[2].fill_(0.5)
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(
            tol=1e-6, precision=mf.FP32_IR, precond=precond, single_reduction=single_reduction))
    torch.cuda.synchronize()
    assert st == mf.OK
    for (shape, k, c), x, info in zip(systems, xs, infos):
        ref = OracleProblem(k, c=c)
        xh = host(x)
        rel = ref.rel_residual(xh)
        assert info["status"] == mf.OK and info["rel_res_true"] <= 1e-6, (shape, info)
        assert rel <= 1e-6 and abs(info["rel_res_true"] - rel) <= 1e-2 * rel + 1e-10, (shape, rel, info)
        p = ref.direct()
        assert np.linalg.norm(xh - p) <= 1e-5 * np.linalg.norm(p), shape
        assert np.array_equal(xh.reshape(shape)[0], np.ones(shape[1:]))


def test_batched_graph_replay_is_deterministic(mf):
    systems = small_batch(5, n=5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]
        xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
        runs = []
        for _ in range(3):
            for x in xs:
                x.zero_()
            st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6))
            assert st == mf.OK
            runs.append(([host(x) for x in xs], [i["iters"] for i in infos]))
        # eager (no graph) gives the same bits
        for x in xs:
            x.zero_()
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, use_graph=0))
        runs.append(([host(x) for x in xs], [i["iters"] for i in infos]))
    torch.cuda.synchronize()
    for fields, iters in runs[1:]:
        assert iters == runs[0][1]
        for a, b in zip(fields, runs[0][0]):
            assert np.array_equal(a, b)


def test_batched_argument_errors(mf):
    shape = (5, 4, 4)
    g, _, b = gpu_problem(mf, lognormal_iid(shape, 1.0, 1))
    x = torch.zeros(80, dtype=torch.float32, device="cuda")
    with pytest.raises(mf.MffvError):
        mf.cg_solve_batched([g, g], [b, b], [x, x])
    with pytest.raises(mf.MffvError):
        mf.cg_solve_batched([g], [b], [x], mf.default_opts(precision=mf.FP64))
    with pytest.raises(mf.MffvError):
        mf.cg_solve_batched([g], [b], [b])


def test_batched_uneven_64_systems_workload(mf):
    # 64 systems, every dimension uniform in [32, 128], log-normal sigma 1.5,
    # c log-uniform in [1e-4, 1e-2]; residuals checked by the oracle's apply
    systems = batch_systems()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, sy.k, c=sy.c, stream=s) for sy in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]
        xs = [torch.zeros(sy.k.size, dtype=torch.float32, device="cuda") for sy in systems]
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, precision=mf.FP32_IR))
    torch.cuda.synchronize()
    assert st == mf.OK
    worst = 0.0
    for sy, x, b, info in zip(systems, xs, bs, infos):
        assert info["status"] == mf.OK and info["rel_res_true"] <= 1e-6
        T = [np.float32(t).astype(np.float64) for t in tpfa.transmissibility(sy.k)]
        dm, _ = tpfa.x_plane_dirichlet(sy.shape)
        xh = host(x).reshape(sy.shape)
        bh = host(b).reshape(sy.shape)
        r = np.where(dm, 0.0, bh - tpfa.apply_stencil(*T, np.float64(np.float32(sy.c)), dm, xh))
        rel = np.linalg.norm(r) / np.linalg.norm(np.where(dm, 0.0, bh))
        assert abs(rel - info["rel_res_true"]) <= 1e-2 * rel + 1e-10
        worst = max(worst, rel)
        assert xh.min() >= -1e-4 and xh.max() <= 1 + 1e-4
    # the refined FP32 fields meet the tolerance on the true residual
    assert worst <= 1e-6
    # and the fields of the two smallest systems (44k and 77k unknowns) match
    # the oracle's direct solution
    small = sorted(range(len(systems)), key=lambda i: systems[i].k.size)[:2]
    for i in small:
        ref = OracleProblem(systems[i].k, c=systems[i].c)
        p = ref.direct()
        assert np.linalg.norm(host(xs[i]) - p) <= 1e-5 * np.linalg.norm(p), systems[i].shape


def test_batched_single_reduction_matches_oracle_and_two_phase(mf):
    """The single-reduction batched iteration (one barrier per iteration) reaches
    the oracle's fields, takes about the two-phase form's iteration count, and
    is deterministic; with Jacobi the batch keeps the two-phase form."""
    systems = small_batch(7)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]

        def run(**kw):
            xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
            st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, **kw))
            torch.cuda.synchronize()
            return st, infos, [host(x) for x in xs]

        st2, inf2, x2 = run(single_reduction=0)
        st1, inf1, x1 = run(single_reduction=1)
        st1b, inf1b, x1b = run(single_reduction=1)
        stj, infj, _ = run(single_reduction=1, precond=mf.PRECOND_JACOBI)
    assert st1 == st2 == stj == mf.OK
    assert all(i["single_reduction"] == 1 for i in inf1)
    assert all(i["single_reduction"] == 0 for i in inf2 + infj)
    for a, b in zip(x1, x1b):
        assert np.array_equal(a, b)
    for (shape, k, c), xa, xb, ia, ib in zip(systems, x1, x2, inf1, inf2):
        ref = OracleProblem(k, c=c)
        p = ref.direct()
        assert ia["status"] == mf.OK and ia["rel_res_recursive"] <= 1e-6
        assert np.linalg.norm(xa - p) <= 5e-5 * np.linalg.norm(p), shape
        # FP32 recurrences drift from the true residual in both forms; the
        # single-reduction one must stay within a small factor of the two-phase one
        assert ia["rel_res_true"] <= max(1e-4, 10 * ib["rel_res_true"]), (shape, ia, ib)
        assert abs(ia["iters"] - ib["iters"]) <= max(3, ib["iters"] // 20), (shape, ia["iters"], ib["iters"])
        assert np.linalg.norm(xa - xb) <= 5e-5 * np.linalg.norm(p), shape
        assert np.array_equal(xa.reshape(shape)[0], np.ones(shape[1:]))   # Dirichlet values


def test_batched_watchdog_reports_and_recovers(mf):
    """With a watchdog limit of 0 every per-system wait that is not satisfied at
    once fails: the blocks record the error and leave (every kernel exits
    normally), and the solve reports it. The same batch then solves correctly
    with the default limit."""
    systems = small_batch(11, n=3)
    systems[0] = ((24, 20, 18), lognormal_iid((24, 20, 18), 1.5, 7), 1e-3)   # several blocks
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        grids = [p[0] for p in probs]
        bs = [p[2] for p in probs]
        xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
        try:
            mf.set_batched_watchdog(0.0)
            with pytest.raises(mf.MffvError) as err:
                mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6))
            assert "barrier" in str(err.value) or "wait" in str(err.value)
        finally:
            mf.set_batched_watchdog(2.0)
        for x in xs:
            x.zero_()
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6))
    torch.cuda.synchronize()
    assert st == mf.OK
    for (shape, k, c), x in zip(systems, xs):
        p = OracleProblem(k, c=c).direct()
        assert np.linalg.norm(host(x) - p) <= 5e-5 * np.linalg.norm(p), shape


def test_batched_solves_follow_new_coefficients(mf):
    """A plan (and its captured graph) made for a set of grids and vectors keeps
    working when the grids' coefficients are set again: a new scalar
    accumulation, then a Dirichlet mask of the caller's (which turns off the
    uniform-diagonal shortcut), each solved with the same pointers through the
    graph, eagerly and asynchronously, and compared with the oracle."""
    systems = small_batch(17, n=4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
        grids = [p[0] for p in probs]
        faces = [p[1] for p in probs]
        bs = [p[2] for p in probs]
        xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]

        def solve_all(tag, refs):
            for mode in ("graph", "eager", "async"):
                for x in xs:
                    x.zero_()
                o = mf.default_opts(tol=1e-6, precision=mf.FP32_IR, use_graph=1 if mode == "graph" else 0)
                o.async_ = 1 if mode == "async" else 0
                st, infos = mf.cg_solve_batched(grids, bs, xs, o)
                torch.cuda.synchronize()
                if mode == "async":
                    infos = mf.infos_from_device(infos)
                assert st == mf.OK and all(i["status"] == mf.OK for i in infos), (tag, mode, infos)
                for (shape, _, _), x, ref in zip(systems, xs, refs):
                    p = ref.direct()
                    xh = host(x)
                    assert np.linalg.norm(xh - p) <= 1e-5 * np.linalg.norm(p), (tag, mode, shape)
                    assert ref.rel_residual(xh) <= 1e-6, (tag, mode, shape)

        solve_all("initial", [OracleProblem(k, c=c) for _, k, c in systems])
        # a larger scalar accumulation: the uniform diagonal changes
        for g, (tx, ty, tz), b in zip(grids, faces, bs):
            mf.set_transmissibility(g, tx, ty, tz, accum_scalar=0.05, b_out=b)
        solve_all("accum 0.05", [OracleProblem(k, c=0.05) for _, k, _ in systems])
        # a caller's mask: the x = 0 plane and one interior cell, value 1 / 0.25
        refs = []
        for g, (tx, ty, tz), b, (shape, k, _) in zip(grids, faces, bs, systems):
            dm = np.zeros(shape, dtype=bool)
            dm[0] = True
            dm[shape[0] - 1, 0, 0] = True
            pd = np.where(dm, 1.0, 0.0)
            pd[shape[0] - 1, 0, 0] = 0.25
            mf.set_transmissibility(g, tx, ty, tz, accum_scalar=1e-3,
                                    dmask=torch.from_numpy(dm.astype(np.uint8).ravel()).cuda(),
                                    pD=torch.from_numpy(pd.astype(np.float32).ravel()).cuda(), b_out=b)
            refs.append(OracleProblem(k, c=1e-3, dmask=dm, pd=pd))
        solve_all("mask", refs)


def test_batched_shares_follow_iterations_and_keep_results(mf):
    """With block shares taken from the previous solve's iteration counts
    (mffv_set_batched_rebalance), the same batch solved again (graph captured
    anew) still meets the true residual in every system and returns the
    refined fields of the first solve to FP32 rounding of the dot products."""
    systems = small_batch(11, n=9)
    # uneven iteration counts: a larger, harder system among small ones with
    # much accumulation
    systems = [((30, 26, 28), lognormal_iid((30, 26, 28), 2.0, 9), 1e-4)] + \
        [(sh, k, 1e-2) for sh, k, _ in systems[1:]]
    s = torch.cuda.Stream()
    mf.set_batched_rebalance(True)
    grids = []
    try:
        with torch.cuda.stream(s):
            probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
            grids = [p[0] for p in probs]
            bs = [p[2] for p in probs]
            xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
            fields, iters = [], []
            for rep in range(3):
                for x in xs:
                    x.zero_()
                st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, precision=mf.FP32_IR))
                torch.cuda.synchronize()
                assert st == mf.OK, infos
                assert all(i["rel_res_true"] <= 1e-6 for i in infos), [i["rel_res_true"] for i in infos]
                fields.append([host(x) for x in xs])
                iters.append([i["iters"] for i in infos])
        print(f"\n[batched] iterations per solve: {iters}")
        for (shape, k, c), f0, f2 in zip(systems, fields[0], fields[2]):
            p = OracleProblem(k, c=c).direct()
            assert np.linalg.norm(f2 - p) <= 1e-5 * np.linalg.norm(p), shape
            assert np.linalg.norm(f2 - f0) <= 1e-5 * np.linalg.norm(f0), shape
    finally:
        mf.set_batched_rebalance(True)
        for g in grids:
            g.close()
