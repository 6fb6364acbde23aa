"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances. An FP32 apply sums 13 rounded terms per cell, each bounded by
``d_K * max|x|`` with ``d_K = c_K + sum of the cell's faces``, so its error is
below ``13 * 2^-24 * 3 d_K max|x|``: the tests allow ``3e-6 d_K max|x|``. In
FP64 the same bound is ``1e-14 d_K max|x|``. Solutions are compared with the
oracle's direct solve of the same FP32-rounded operator; the field error of a
solve stopped at relative residual ``tol`` is bounded by ``kappa * tol``, so the
tests check the residual target itself and the field to a margin stated per case.
"""
import numpy as np
import pytest

from oracle import krylov, tpfa
from synth import lognormal_iid, workload_field, WORKLOADS
from gpu_problem import gpu_problem, OracleProblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mffv.lib()
    return mffv


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda", dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


SHAPES = [(32, 32, 32),        # float4 path, one chunk per plane
          (9, 40, 64),         # float4 path, several chunks and a ragged chunk
          (5, 9, 512),         # float4 path, long rows: 4-row x 256-cell chunks, ragged row group
          (7, 13, 37),         # one cell per thread (nz odd), ragged
          (3, 5, 8),           # a single unknown plane
          (6, 1, 1)]           # a 1D column


@pytest.mark.parametrize("shape", SHAPES)
def test_transmissibility_matches_oracle(mf, shape):
    k = lognormal_iid(shape, 2.0, 31)
    tx, ty, tz = (torch.empty(k.size, dtype=torch.float32, device="cuda") for _ in range(3))
    mf.perm_to_trans(*shape, dev(k, torch.float64), 0.1, tx, ty, tz)
    ref = [np.float32(t).ravel() for t in tpfa.transmissibility(k, 0.1)]
    for got, want in zip((tx, ty, tz), ref):
        g = got.cpu().numpy()
        ulp = np.abs(g.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
        assert ulp.max() <= 1
        assert np.count_nonzero(ulp) <= max(1, g.size // 100000)


@pytest.mark.parametrize("shape", SHAPES)
def test_rhs_matches_oracle(mf, shape):
    k = lognormal_iid(shape, 1.0, 5)
    _, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    assert np.allclose(host(b), ref.b, rtol=1e-7, atol=0)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kz", [1.0, 0.1])
def test_apply_matches_oracle(mf, shape, kz):
    k = lognormal_iid(shape, 2.0, 17)
    g, _, _ = gpu_problem(mf, k, c=1e-3, kz_ratio=kz)
    ref = OracleProblem(k, c=1e-3, kz_ratio=kz)
    rng = np.random.default_rng(1)
    for _ in range(2):
        x = rng.normal(size=shape).astype(np.float32)
        y = torch.empty(k.size, dtype=torch.float32, device="cuda")
        mf.apply(g, dev(x), y)
        want = ref.A @ x.astype(np.float64).ravel()
        err = np.abs(host(y) - want)
        assert np.all(err <= 3e-6 * ref.diag() * np.abs(x).max())
        # FP64 apply
        y64 = torch.empty(k.size, dtype=torch.float64, device="cuda")
        mf.apply_f64(g, dev(x, torch.float64), y64)
        err64 = np.abs(host(y64) - want)
        assert np.all(err64 <= 1e-14 * ref.diag() * np.abs(x).max())


def test_apply_unaligned_and_custom_dirichlet(mf):
    shape = (8, 12, 16)
    rng = np.random.default_rng(4)
    k = lognormal_iid(shape, 1.0, 8)
    dmask = np.zeros(shape, dtype=bool)
    dmask[0, :, :] = True
    dmask[4, 3:6, 2:9] = True                      # an interior Dirichlet block
    pd = np.where(dmask, rng.uniform(-1, 2, shape), 0.0)
    accum = rng.uniform(0, 1e-2, shape)
    g, _, b = gpu_problem(mf, k, dmask=dmask, pd=pd, accum=accum)
    ref = OracleProblem(k, dmask=dmask, pd=pd, accum=accum)
    assert np.allclose(host(b), ref.b, rtol=1e-6, atol=1e-7)
    x = rng.normal(size=k.size).astype(np.float32)
    # views that start one element in: not 16-byte aligned, takes the scalar path
    xs = torch.zeros(k.size + 1, dtype=torch.float32, device="cuda")
    ys = torch.zeros(k.size + 1, dtype=torch.float32, device="cuda")
    xs[1:] = dev(x)
    mf.apply(g, xs[1:], ys[1:])
    want = ref.A @ x.astype(np.float64)
    assert np.all(np.abs(host(ys[1:]) - want) <= 3e-6 * ref.diag() * np.abs(x).max())


def test_long_rows_refined_solve_matches_direct(mf):
    """nz > 256: the float4 kernels use 4-row x 256-cell chunks (z-segment halos
    between chunks of one row); the refined solve must match the direct solve."""
    shape = (6, 7, 768)
    k = lognormal_iid(shape, 1.0, 21)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.double(), x, mf.default_opts(tol=1e-10, precision=mf.FP32_IR))
    assert st == mf.OK and info["rel_res_true"] <= 1e-10
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 1e-8 * np.linalg.norm(p)


@pytest.mark.parametrize("shape", [(24, 20, 32), (6, 7, 768)])
def test_single_reduction_matches_two_phase(mf, shape):
    """The single-reduction iteration (one kernel per iteration, r.r from a
    one-step recurrence on the exact value) and the two-phase iteration solve
    the same FP32 system: both reach the recursive target, the true residuals
    of the FP32 results are of the same size (the FP32 attainable accuracy, set
    by the same vector recurrence), their iteration counts stay close, and both
    refined fields match the direct solve."""
    k = lognormal_iid(shape, 1.5, 31)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    p = ref.direct()
    res, true = {}, {}
    for sr in (1, 0):
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, single_reduction=sr))
        assert st == mf.OK and info["single_reduction"] == sr
        assert info["rel_res_recursive"] <= 1e-6 and info["rel_res_true"] <= 1e-4
        x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
        st, info64 = mf.cg_solve_f64(g, b.double(), x64, mf.default_opts(
            tol=1e-10, precision=mf.FP32_IR, single_reduction=sr))
        assert st == mf.OK and info64["single_reduction"] == sr
        assert np.linalg.norm(host(x64) - p) <= 1e-8 * np.linalg.norm(p)
        res[sr], true[sr] = info["iters"], info["rel_res_true"]
    assert abs(res[1] - res[0]) <= max(3, 0.05 * res[0])
    assert true[1] <= 4 * true[0] + 1e-6 and true[0] <= 4 * true[1] + 1e-6


def test_apply_symmetry_on_device(mf):
    shape = (16, 24, 20)
    k = lognormal_iid(shape, 2.0, 3)
    g, _, _ = gpu_problem(mf, k, c=1e-3, kz_ratio=0.5)
    rng = np.random.default_rng(0)
    x, y = (dev(rng.normal(size=k.size), torch.float64) for _ in range(2))
    ax, ay = (torch.empty(k.size, dtype=torch.float64, device="cuda") for _ in range(2))
    mf.apply_f64(g, x, ax)
    mf.apply_f64(g, y, ay)
    lhs, rhs = float(x @ ay), float(y @ ax)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0) * 100


@pytest.fixture(scope="module")
def c0(mf):
    w = WORKLOADS["lognormal_iid_32cube"]
    k = workload_field(w)
    ref = OracleProblem(k, c=w.c)
    return w, k, ref


def test_cg_fp64_matches_oracle_iterations(mf, c0):
    w, k, ref = c0
    g, _, b = gpu_problem(mf, k, c=w.c)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    b64 = b.to(torch.float64)
    st, info = mf.cg_solve_f64(g, b64, x, mf.default_opts(precision=mf.FP64, tol=1e-6))
    assert st == mf.OK
    orc = krylov.cg(ref.Auu, ref.bu, tol=1e-6, max_iter=10000)
    assert abs(info["iters"] - orc.iters) <= 1
    assert info["rel_res_true"] <= 1e-6 * 1.001
    assert ref.rel_residual(host(x)) <= 1e-6 * 1.001
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 1e-5 * np.linalg.norm(p)


def test_cg_fp64_tight_matches_direct(mf, c0):
    w, k, ref = c0
    g, _, b = gpu_problem(mf, k, c=w.c)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.to(torch.float64), x,
                               mf.default_opts(precision=mf.FP64, tol=1e-11))
    assert st == mf.OK
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 1e-8 * np.linalg.norm(p)


def test_cg_fp32_then_refinement(mf, c0):
    w, k, ref = c0
    g, _, b = gpu_problem(mf, k, c=w.c)
    p = ref.direct()
    # plain FP32 CG: converges on the recursive residual; the FP64 true
    # residual is reported (FP32 rounding of x alone limits it near 1e-6 here)
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6))
    assert st == mf.OK and info["rel_res_recursive"] <= 1e-6
    orc = krylov.cg(ref.Auu.astype(np.float32), ref.bu.astype(np.float32), tol=1e-6,
                    max_iter=10000, dtype=np.float32)
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 20)
    assert abs(info["rel_res_true"] - ref.rel_residual(host(x))) <= 1e-3 * info["rel_res_true"] + 1e-9
    assert np.linalg.norm(host(x) - p) <= 2e-5 * np.linalg.norm(p)
    # refinement to 1e-6 on the true residual, FP32 output
    x.zero_()
    st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, precision=mf.FP32_IR))
    assert st == mf.OK and info["rel_res_true"] <= 1e-6
    # refinement to 1e-10 with an FP64 output field
    x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.to(torch.float64), x64,
                               mf.default_opts(tol=1e-10, precision=mf.FP32_IR))
    assert st == mf.OK and info["ir_steps"] >= 2
    assert ref.rel_residual(host(x64)) <= 1e-10 * 1.01
    assert np.linalg.norm(host(x64) - p) <= 1e-8 * np.linalg.norm(p)


def test_jacobi_pcg_matches_oracle(mf, c0):
    w, k, ref = c0
    g, _, b = gpu_problem(mf, k, c=w.c)
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, precond=mf.PRECOND_JACOBI))
    assert st == mf.OK
    orc = krylov.pcg(ref.Auu, ref.bu, krylov.jacobi(ref.Auu), tol=1e-6, max_iter=10000)
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 20)
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 2e-5 * np.linalg.norm(p)
    # refined Jacobi-PCG reaches the FP64 target too
    x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.to(torch.float64), x64,
                               mf.default_opts(tol=1e-9, precision=mf.FP32_IR,
                                               precond=mf.PRECOND_JACOBI))
    assert st == mf.OK and ref.rel_residual(host(x64)) <= 1e-9 * 1.01


@pytest.mark.parametrize("shape", [(3, 4, 5), (6, 1, 1), (5, 2, 3), (17, 3, 33)])
def test_small_and_degenerate_shapes_closed_form(mf, shape):
    # homogeneous k, c = 0: p_i = 1 - i/(nx-1)
    k = np.full(shape, 2.5)
    g, _, b = gpu_problem(mf, k, c=0.0)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.to(torch.float64), x,
                               mf.default_opts(tol=1e-12, precision=mf.FP64))
    assert st == mf.OK
    expect = np.broadcast_to((1.0 - np.arange(shape[0]) / (shape[0] - 1))[:, None, None], shape)
    assert np.max(np.abs(host(x) - expect.ravel())) < 1e-10


def test_sinh_profile_with_accumulation_fp32_ir(mf):
    shape, c = (40, 8, 12), 0.05
    g, _, b = gpu_problem(mf, np.ones(shape), c=c)
    x = torch.zeros(int(np.prod(shape)), dtype=torch.float64, device="cuda")
    st, _ = mf.cg_solve_f64(g, b.to(torch.float64), x, mf.default_opts(tol=1e-10, precision=mf.FP32_IR))
    assert st == mf.OK
    theta = np.arccosh(1.0 + np.float64(np.float32(c)) / 2.0)
    i = np.arange(shape[0])
    expect = np.sinh(theta * (shape[0] - 1 - i)) / np.sinh(theta * (shape[0] - 1))
    assert np.max(np.abs(host(x).reshape(shape) - expect[:, None, None])) < 1e-8


def test_no_dirichlet_cells_with_accumulation(mf):
    shape = (6, 8, 8)
    rng = np.random.default_rng(2)
    k = lognormal_iid(shape, 1.0, 9)
    dmask = np.zeros(shape, dtype=bool)
    g, _, _ = gpu_problem(mf, k, c=0.01, dmask=dmask, pd=np.zeros(shape))
    ref = OracleProblem(k, c=0.01, dmask=dmask, pd=np.zeros(shape))
    bb = rng.normal(size=k.size)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, _ = mf.cg_solve_f64(g, dev(bb, torch.float64), x, mf.default_opts(tol=1e-11, precision=mf.FP64))
    assert st == mf.OK
    xs = np.linalg.solve(ref.A.toarray(), bb)
    assert np.linalg.norm(host(x) - xs) <= 1e-8 * np.linalg.norm(xs)


def test_zero_rhs_and_initial_guess(mf):
    shape = (8, 8, 8)
    k = lognormal_iid(shape, 1.0, 1)
    pd = np.zeros(shape)
    dmask, _ = tpfa.x_plane_dirichlet(shape)
    g, _, b = gpu_problem(mf, k, dmask=dmask, pd=pd)
    assert float(b.abs().max()) == 0.0
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x)
    assert st == mf.OK and info["iters"] == 0 and float(x.abs().max()) == 0.0
    # a good initial guess: restart from a converged solution takes ~0 iterations
    g2, _, b2 = gpu_problem(mf, k, c=1e-3)
    x2 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    mf.cg_solve_f64(g2, b2.to(torch.float64), x2, mf.default_opts(tol=1e-10, precision=mf.FP64))
    st, info = mf.cg_solve_f64(g2, b2.to(torch.float64), x2, mf.default_opts(tol=1e-8, precision=mf.FP64))
    assert st == mf.OK and info["iters"] == 0


def test_errors_forced_from_the_host(mf):
    shape = (5, 4, 4)
    n = 80
    k = lognormal_iid(shape, 1.0, 2)
    g, (tx, ty, tz), b = gpu_problem(mf, k)
    bad = tx.clone()
    bad[3] = -1.0
    with pytest.raises(mf.MffvError) as e:
        mf.set_transmissibility(g, bad, ty, tz, accum_scalar=1e-3)
    assert e.value.code == mf.EINVAL and "transmissibility" in str(e.value)
    bad[3] = float("nan")
    with pytest.raises(mf.MffvError):
        mf.set_transmissibility(g, bad, ty, tz, accum_scalar=1e-3)
    with pytest.raises(mf.MffvError):
        mf.set_transmissibility(g, tx, ty, tz, accum_scalar=float("nan"))
    nodir = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(mf.MffvError) as e:
        mf.set_transmissibility(g, tx, ty, tz, accum_scalar=0.0, dmask=nodir)
    assert "singular" in str(e.value)
    # a failed set leaves the grid without coefficients
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(mf.MffvError) as e:
        mf.cg_solve(g, b, x)
    assert e.value.code == mf.ESTATE
    mf.set_transmissibility(g, tx, ty, tz, accum_scalar=1e-3)
    # iteration cap: NOT_CONVERGED is a result, x holds the last iterate
    st, info = mf.cg_solve(g, b, x, mf.default_opts(max_iter=2, tol=1e-12))
    assert st == mf.NOT_CONVERGED and info["iters"] == 2
    with pytest.raises(mf.MffvError):
        mf.cg_solve(g, b, b)
    with pytest.raises(mf.MffvError):
        mf.cg_solve(g, b, x, mf.default_opts(tol=2.0))
    with pytest.raises(mf.MffvError):
        mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED))


def test_deterministic_and_graph_equals_eager(mf, c0):
    w, k, ref = c0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, c=w.c, stream=s)
        outs = []
        for use_graph in (1, 1, 0):
            x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
            st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, use_graph=use_graph,
                                                            check_every=8))
            assert st == mf.OK
            outs.append((host(x), info["iters"]))
    torch.cuda.synchronize()
    for o, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(o, outs[0][0])


def test_full_size_apply_256cube(mf):
    w = WORKLOADS["lognormal_corr8_256cube"]
    k = workload_field(w)
    g, (tx, ty, tz), _ = gpu_problem(mf, k, c=w.c)
    T = [np.float32(t) for t in tpfa.transmissibility(k)]
    dmask, _ = tpfa.x_plane_dirichlet(k.shape)
    rng = np.random.default_rng(7)
    x = rng.normal(size=k.shape).astype(np.float32)
    y = torch.empty(k.size, dtype=torch.float32, device="cuda")
    mf.apply(g, dev(x), y)
    want = tpfa.apply_stencil(*T, np.float32(w.c), dmask, x)
    d = np.float32(w.c) + sum(np.abs(t) for t in T)
    assert np.all(np.abs(host(y).reshape(k.shape) - want) <= 3e-6 * (2 * d + 1) * np.abs(x).max())


def test_full_size_refined_solve_256cube(mf):
    w = WORKLOADS["lognormal_corr8_256cube"]
    k = workload_field(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, _, b = gpu_problem(mf, k, c=w.c, stream=s)
        x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
        st, info = mf.cg_solve_f64(g, b.to(torch.float64), x,
                                   mf.default_opts(tol=1e-8, precision=mf.FP32_IR))
    torch.cuda.synchronize()
    assert st == mf.OK, info
    T = [np.float32(t).astype(np.float64) for t in tpfa.transmissibility(k)]
    dmask, pd = tpfa.x_plane_dirichlet(k.shape)
    xh = host(x).reshape(k.shape)
    r = np.where(dmask, 0.0, host(b).reshape(k.shape) - tpfa.apply_stencil(*T, np.float64(np.float32(w.c)), dmask, xh))
    bu = np.where(dmask, 0.0, host(b).reshape(k.shape))
    rel = np.linalg.norm(r) / np.linalg.norm(bu)
    assert rel <= 1.05e-8, (rel, info)
    assert abs(rel - info["rel_res_true"]) <= 1e-3 * rel
    # the discrete maximum principle holds for the refined field
    assert xh.min() >= -1e-6 and xh.max() <= 1 + 1e-6


def test_crop_of_the_256cube_field_matches_the_oracle_elementwise(mf):
    """The [0:64]^3 crop of the correlated 256^3 field (sigma 2, correlation
    length 8, c = 1e-3) as its own problem: FP32 CG refined in FP64 to a true
    relative residual of 1e-8, against the oracle's FP64 Jacobi-PCG to 1e-12.
    The field lies in [0, 1] (maximum principle), so every cell must agree to
    1e-5 absolute, and the L2 field error must be below 1e-5 relative."""
    w = WORKLOADS["lognormal_corr8_256cube"]
    k = np.ascontiguousarray(workload_field(w)[:64, :64, :64])
    g, _, b = gpu_problem(mf, k, c=w.c)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.double(), x, mf.default_opts(tol=1e-8, precision=mf.FP32_IR))
    assert st == mf.OK and info["rel_res_true"] <= 1e-8
    ref = OracleProblem(k, c=w.c)
    orc = krylov.pcg(ref.Auu, ref.bu, krylov.jacobi(ref.Auu), tol=1e-12, max_iter=20000)
    assert orc.converged
    p = tpfa.scatter_solution(orc.x, ref.u, ref.pd, ref.dmask)
    xh = x.cpu().numpy()
    err = np.abs(xh - p)
    assert err.max() <= 1e-5, (float(err.max()), np.unravel_index(int(err.argmax()), k.shape))
    assert np.linalg.norm(xh - p) <= 1e-5 * np.linalg.norm(p)
    assert ref.rel_residual(xh) <= 1.01e-8
    g.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32_ir", "batched", "async"])
def test_non_finite_rhs_reports_breakdown(mf, precision):
    """A NaN in the right-hand side makes every dot product non-finite: the
    solve stops with MFFV_EBREAKDOWN (no hang, no fault) and fills info."""
    shape = (10, 9, 12)
    k = lognormal_iid(shape, 1.0, 31)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    b[5 * 9 * 12 + 40] = float("nan")
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    if precision in ("fp32", "fp32_ir"):
        o = mf.default_opts(precision=mf.FP32 if precision == "fp32" else mf.FP32_IR)
        with pytest.raises(mf.MffvError) as e:
            mf.cg_solve(g, b, x, o)
        assert e.value.code == mf.EBREAKDOWN
        # the raw call returns the code with info filled
        import ctypes
        info = mf.Info()
        rc = mf.lib().mffv_cg_solve(g.handle, b.data_ptr(), x.data_ptr(), ctypes.byref(o), ctypes.addressof(info))
        assert rc == mf.EBREAKDOWN and info.status == mf.EBREAKDOWN
    elif precision == "batched":
        with pytest.raises(mf.MffvError) as e:
            mf.cg_solve_batched([g], [b], [x], mf.default_opts(precision=mf.FP32_IR))
        assert e.value.code == mf.EBREAKDOWN
    else:
        o = mf.default_opts(precision=mf.FP32_IR)
        o.async_ = 1
        st, dinfo = mf.cg_solve(g, b, x, o)
        infos = mf.infos_from_device(dinfo)
        assert st == mf.OK and infos[0]["status"] == mf.EBREAKDOWN
    g.close()
