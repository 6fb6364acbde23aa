"""Backward-Euler time steps with wells through the C ABI, against the oracle
(each step solved directly in FP64) and against closed forms."""
import numpy as np
import pytest

from oracle import timestep
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).ravel()).cuda()


def wells_case(shape, seed):
    """Storage, two wells and a perforated column, two sources. Storage and
    well indices are dyadic, so c + WI is exact in FP32 on both sides."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    k = lognormal_iid(shape, 1.0, seed)
    c = rng.choice([0.125, 0.25, 0.375, 0.5], shape)
    wi = np.zeros(shape)
    pw = np.zeros(shape)
    wi[1, 1, 1], pw[1, 1, 1] = 3.0, 5.0
    wi[nx - 2, ny - 2, nz - 2], pw[nx - 2, ny - 2, nz - 2] = 2.0, -1.0
    wi[nx // 3, ny // 2, :], pw[nx // 3, ny // 2, :] = 1.5, 4.0
    q = np.zeros(shape)
    q[nx // 2, 1, nz // 2] = 0.75
    q[2 * nx // 3, ny - 1, 0] = -0.5
    p0 = np.float32(rng.uniform(0.0, 2.0, shape)).astype(np.float64)
    return k, c, wi, np.float32(pw).astype(np.float64), np.float32(q).astype(np.float64), p0


def setup(mf, k, c, wi, s):
    g, _, b = gpu_problem(mf, k, accum=c + wi, stream=s)
    return g, b


@pytest.mark.parametrize("shape", [(21, 17, 19), (20, 16, 12)])   # one cell per thread; four
def test_step_rhs_matches_oracle(mf, shape):
    k, c, wi, pw, q, p0 = wells_case(shape, 5)
    ref = OracleProblem(k, accum=c + wi)
    p0[ref.dmask] = ref.pd[ref.dmask]
    want = timestep.step_rhs(ref.b, c, p0, ref.dmask, wi, pw, q)
    scale = np.abs(ref.b.reshape(shape)) + np.abs(c * p0) + np.abs(wi * pw) + np.abs(q)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, b = setup(mf, k, c, wi, s)
        rhs = torch.empty_like(b)
        mf.step_rhs(g, b, dev(p0), rhs, c=dev(c), wi=dev(wi), pw=dev(pw), q=dev(q))
        got = host(rhs).reshape(shape)
        # scalar storage, no wells, no sources
        rhs2 = torch.empty_like(b)
        mf.step_rhs(g, b, dev(p0), rhs2, c_scalar=0.25)
        got2 = host(rhs2).reshape(shape)
    # FP32 evaluation (b itself is the library's FP32 right-hand side): a few ulps of the terms
    assert np.all(np.abs(got - want) <= 4 * 2.0 ** -24 * scale + 1e-30)
    assert np.array_equal(got[ref.dmask], ref.pd[ref.dmask])
    want2 = timestep.step_rhs(ref.b, 0.25, p0, ref.dmask)
    scale2 = np.abs(ref.b.reshape(shape)) + np.abs(0.25 * p0)
    assert np.all(np.abs(got2 - want2) <= 4 * 2.0 ** -24 * scale2 + 1e-30)


@pytest.mark.parametrize("shape,nsteps", [((20, 16, 12), 5), ((13, 9, 7), 3)])
def test_time_steps_match_oracle(mf, shape, nsteps):
    """Step by step against the oracle's direct solves; the float4 kernels
    (nz % 4 == 0) and the one-cell-per-thread kernels (ragged nz)."""
    k, c, wi, pw, q, p0 = wells_case(shape, 6)
    ref = OracleProblem(k, accum=c + wi)
    p0[ref.dmask] = ref.pd[ref.dmask]
    want = timestep.run(*ref.T, c, ref.dmask, ref.pd, p0, nsteps, wi, pw, q)
    s = torch.cuda.Stream()
    opts = mf.default_opts(precision=mf.FP32_IR, tol=1e-9)
    with torch.cuda.stream(s):
        g, b = setup(mf, k, c, wi, s)
        args = dict(c=dev(c), wi=dev(wi), pw=dev(pw), q=dev(q), opts=opts)
        p = dev(p0)
        got = []
        for _ in range(nsteps):
            st, infos = mf.time_steps(g, 1, b, p, **args)
            assert st == mf.OK and infos[0]["status"] == mf.OK and infos[0]["rel_res_true"] <= 1e-9
            got.append(host(p).reshape(shape))
        # all steps in one call: the same kernels in the same order, the same bits
        p_all = dev(p0)
        st, infos = mf.time_steps(g, nsteps, b, p_all, **args)
        assert st == mf.OK and len(infos) == nsteps
        assert all(i["status"] == mf.OK for i in infos)
        assert np.array_equal(host(p_all).reshape(shape), got[-1])
    for step, (gp, wp) in enumerate(zip(got, want)):
        assert np.max(np.abs(gp - wp)) <= 1e-5 * np.max(np.abs(wp)), step
        assert np.array_equal(gp[ref.dmask], ref.pd[ref.dmask])


def test_time_steps_eigenmode_closed_form(mf):
    """Homogeneous unit cells, p^D = 0 on both x planes, uniform storage: the x
    profile sin(pi i / (nx - 1)) decays by c / (c + lambda) per step with
    lambda = 2 (1 - cos(pi / (nx - 1)))."""
    shape = (33, 8, 8)
    nx = shape[0]
    k = np.ones(shape)
    dmask = np.zeros(shape, dtype=bool)
    dmask[0] = dmask[-1] = True
    pd = np.zeros(shape)
    c = 0.7
    i = np.arange(nx)
    p0 = np.broadcast_to(np.sin(np.pi * i / (nx - 1))[:, None, None], shape)
    lam = 2.0 * (1.0 - np.cos(np.pi / (nx - 1)))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, c=c, dmask=dmask, pd=pd, stream=s)
        p = dev(p0)
        st, infos = mf.time_steps(g, 4, b, p, c_scalar=c,
                                  opts=mf.default_opts(precision=mf.FP32_IR, tol=1e-9))
        got = host(p).reshape(shape)
    assert st == mf.OK
    want = p0 * (c / (c + lam)) ** 4
    assert np.max(np.abs(got - want)) <= 2e-6 * np.max(np.abs(want))


def test_time_steps_mass_balance(mf):
    """Storage change = sources + well inflow + inflow across the Dirichlet
    faces, from the GPU fields in FP64, to the solve's tolerance."""
    shape = (40, 24, 32)
    k, c, wi, pw, q, p0 = wells_case(shape, 7)
    ref = OracleProblem(k, accum=c + wi)
    p0[ref.dmask] = ref.pd[ref.dmask]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, b = setup(mf, k, c, wi, s)
        p = dev(p0)
        st, _ = mf.time_steps(g, 1, b, p, c=dev(c), wi=dev(wi), pw=dev(pw), q=dev(q),
                              opts=mf.default_opts(precision=mf.FP32_IR, tol=1e-9))
        p1 = host(p).reshape(shape)
    assert st == mf.OK
    u = ~ref.dmask
    tx, ty, tz = ref.T
    storage = np.sum((c * (p1 - p0))[u])
    inflow = np.sum(q[u]) + np.sum((wi * (pw - p1))[u])
    for t, a, bsl in ((tx, np.s_[:-1, :, :], np.s_[1:, :, :]),
                      (ty, np.s_[:, :-1, :], np.s_[:, 1:, :]),
                      (tz, np.s_[:, :, :-1], np.s_[:, :, 1:])):
        da, db = ref.dmask[a], ref.dmask[bsl]
        inflow += np.sum(np.where(da & ~db, t[a] * (ref.pd[a] - p1[bsl]), 0.0))
        inflow += np.sum(np.where(db & ~da, t[a] * (ref.pd[bsl] - p1[a]), 0.0))
    flux_scale = np.sum(np.abs(q)) + np.sum(wi * np.abs(pw - p1)) + np.sum(np.abs(c * (p1 - p0)))
    assert abs(storage - inflow) <= 1e-5 * flux_scale


def test_time_steps_argument_errors(mf):
    shape = (6, 5, 4)
    k = lognormal_iid(shape, 1.0, 3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, c=0.5, stream=s)
        p = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        one = torch.ones_like(p)
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, 1, b, p, c_scalar=0.5, wi=one)            # wi without pw
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, -1, b, p, c_scalar=0.5)
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, 1, b, p, c_scalar=-1.0)
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, 1, b, p, c_scalar=0.5, opts=mf.default_opts(async_=1))
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, 1, b, p, c_scalar=0.5, opts=mf.default_opts(precision=mf.FP64))
        with pytest.raises(mf.MffvError):
            mf.step_rhs(g, b, p, p, c_scalar=0.5)                       # rhs aliases p_old
        with pytest.raises(mf.MffvError):
            mf.time_steps(g, 1, b, b, c_scalar=0.5)                     # p aliases b
        p.fill_(3.0)
        st, infos = mf.time_steps(g, 0, b, p, c_scalar=0.5)             # no steps: p unchanged
        assert st == mf.OK and infos == []
        assert torch.all(p == 3.0)
    s.synchronize()
