"""Asynchronous (capture-safe) solves: opts.async_ enqueues the persistent CG
and the FP64 residual without any host synchronisation, and writes the
per-system mffv_info into device memory. Checked against the synchronous call
(same kernels, so the same bits), inside a torch CUDA graph replayed several
times, and for one system against the oracle."""
import numpy as np
import pytest

from oracle import krylov
from synth import lognormal_iid
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


def batch(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        shape = tuple(int(v) for v in rng.integers(4, 21, 3))
        out.append((shape, lognormal_iid(shape, 1.5, 500 + s), float(10 ** rng.uniform(-4, -2))))
    out[0] = ((24, 20, 18), lognormal_iid((24, 20, 18), 1.5, 499), 1e-3)   # several blocks
    return out


def setup(mf, systems, s):
    probs = [gpu_problem(mf, k, c=c, stream=s) for _, k, c in systems]
    grids = [p[0] for p in probs]
    bs = [p[2] for p in probs]
    xs = [torch.zeros(k.size, dtype=torch.float32, device="cuda") for _, k, _ in systems]
    return grids, bs, xs


KEYS = ("status", "iters", "ir_steps", "single_reduction")


def same_info(a, b):
    for key in KEYS:
        assert a[key] == b[key], (key, a, b)
    for key in ("rel_res_recursive", "rel_res_true"):
        assert a[key] == pytest.approx(b[key], rel=1e-14, abs=0.0), (key, a, b)


@pytest.mark.parametrize("precond,single", [(0, 0), (1, 0), (0, 1)])
def test_async_batched_matches_sync(mf, precond, single):
    systems = batch(21, 5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        grids, bs, xs = setup(mf, systems, s)
        opts = dict(tol=1e-6, precond=precond, single_reduction=single)
        st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(**opts))
        assert st == mf.OK
        ref = [host(x) for x in xs]
        for x in xs:
            x.fill_(7.0)
            x.zero_()
        st, dinfo = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(async_=1, **opts))
        assert st == mf.OK
        got = [host(x) for x in xs]
        dinfos = mf.infos_from_device(dinfo)
    assert len(dinfos) == len(systems)
    for r, g, a, b in zip(ref, got, dinfos, infos):
        assert np.array_equal(r, g)
        same_info(a, b)
        assert a["status"] == mf.OK and a["single_reduction"] == single


def test_async_batched_in_cuda_graph(mf):
    """The plan is built by one call outside capture; the captured solve is then
    replayed with eager work and synchronisations in between, and every replay
    gives the eager result bit for bit, device infos included."""
    systems = batch(22, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        grids, bs, xs = setup(mf, systems, s)
        opts = mf.default_opts(tol=1e-6, async_=1)
        st, dinfo = mf.cg_solve_batched(grids, bs, xs, opts)   # builds the plan
        assert st == mf.OK
        ref = [host(x) for x in xs]
        ref_info = mf.infos_from_device(dinfo)
    assert all(i["status"] == mf.OK for i in ref_info)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for x in xs:
            x.zero_()
        st, ginfo = mf.cg_solve_batched(grids, bs, xs, opts)
    assert st == mf.OK
    for rep in range(4):
        with torch.cuda.stream(s):
            for x in xs:
                x.fill_(float(rep + 3))       # eager work the replay must overwrite
            junk = torch.randn(1 << 16, device="cuda").sum()
            g.replay()
        s.synchronize()
        assert torch.isfinite(junk)
        for r, x in zip(ref, xs):
            assert np.array_equal(r, host(x)), rep
        for a, b in zip(mf.infos_from_device(ginfo), ref_info):
            same_info(a, b)


def test_async_first_call_under_capture_is_refused(mf):
    systems = batch(23, 2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        grids, bs, xs = setup(mf, systems, s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        xs[0].zero_()
        with pytest.raises(mf.MffvError) as err:
            mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, async_=1))
    assert "capture" in str(err.value)
    # outside capture the same call builds its plan and solves
    with torch.cuda.stream(s):
        st, dinfo = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, async_=1))
        infos = mf.infos_from_device(dinfo)
    assert st == mf.OK and all(i["status"] == mf.OK for i in infos)


def test_async_watchdog_status_lands_in_device_info(mf):
    """A watchdog limit of 0 makes the persistent kernel's waits fail at once
    (its blocks leave normally); the async call reports it in the device info,
    and the next launch starts clean."""
    systems = batch(24, 2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        grids, bs, xs = setup(mf, systems, s)
        try:
            mf.set_batched_watchdog(0.0)
            st, dinfo = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, async_=1))
            assert st == mf.OK                       # only enqueued
            bad = mf.infos_from_device(dinfo)
        finally:
            mf.set_batched_watchdog(2.0)
        for x in xs:
            x.zero_()
        st, dinfo = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, async_=1))
        good = mf.infos_from_device(dinfo)
    assert bad[0]["status"] == mf.EHIP               # the multi-block system had to wait
    assert all(i["status"] == mf.OK for i in good)
    for (shape, k, c), x in zip(systems, xs):
        p = OracleProblem(k, c=c).direct()
        assert np.linalg.norm(host(x) - p) <= 5e-5 * np.linalg.norm(p), shape


@pytest.mark.parametrize("precond", [0, 1])
def test_async_cg_solve_matches_oracle(mf, precond):
    shape = (20, 17, 13)
    k = lognormal_iid(shape, 1.5, 77)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, c=1e-3, stream=s)
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st, dinfo = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, precond=precond, async_=1))
        assert st == mf.OK
        (info,) = mf.infos_from_device(dinfo)
    ref = OracleProblem(k, c=1e-3)
    assert info["status"] == mf.OK and info["rel_res_recursive"] <= 1e-6
    M = krylov.jacobi(ref.Auu) if precond else None
    orc = krylov.pcg(ref.Auu.astype(np.float32), ref.bu.astype(np.float32), M, tol=1e-6,
                     max_iter=20000, dtype=np.float32)
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 10), (info, orc.iters)
    p = ref.direct()
    xh = host(x)
    assert np.linalg.norm(xh - p) <= 5e-5 * np.linalg.norm(p)
    assert abs(info["rel_res_true"] - ref.rel_residual(xh)) <= 1e-2 * info["rel_res_true"] + 1e-8


def test_async_argument_errors(mf):
    shape = (6, 5, 4)
    k = lognormal_iid(shape, 1.0, 3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, stream=s)
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        with pytest.raises(mf.MffvError):
            mf.cg_solve(g, b, x, mf.default_opts(async_=1, precision=mf.FP64))
        with pytest.raises(mf.MffvError):
            mf.cg_solve(g, b, x, mf.default_opts(async_=2))
    s.synchronize()
