"""Autotuner and launch shapes: every shape computes the same apply bits, the
tuner's choice is cached, and solves stay correct under the tuned shapes."""
import json
import os

import numpy as np
import pytest

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


@pytest.mark.parametrize("shape", [(40, 24, 64), (21, 17, 19), (9, 37, 256), (5, 11, 512)])
def test_launch_shapes_give_identical_apply(mf, shape):
    k = lognormal_iid(shape, 1.5, 2)
    g, _, _ = gpu_problem(mf, k, c=1e-3)
    x = torch.randn(k.size, dtype=torch.float32, device="cuda")
    nz = shape[2]
    # chunk shapes: default, flat, and every row-segment length the float4 path accepts
    segs = [0, -1] + ([s for s in (16, 32, 64, 128, 256, 512, 1024) if nz % s == 0] if nz % 4 == 0 else [])
    outs = []
    for seg in segs:
        for ci, remap in ((0, 1), (1, 0), (3, 1), (8, 0), (64, 1)):
            mf.set_launch(g, ci, remap, seg)
            y = torch.empty_like(x)
            mf.apply(g, x, y)
            outs.append(host(y))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    with pytest.raises(mf.MffvError):
        mf.set_launch(g, -1, 0)
    for bad in (-2, 8, 24, 2048):
        with pytest.raises(mf.MffvError):
            mf.set_launch(g, 0, 1, bad)
    if nz % 4:
        with pytest.raises(mf.MffvError):
            mf.set_launch(g, 0, 1, 16)


_SEG_SHAPE = (14, 18, 256)


@pytest.fixture(scope="module")
def seg_problem():
    k = lognormal_iid(_SEG_SHAPE, 1.0, 4)
    return k, OracleProblem(k, c=1e-3).direct()


@pytest.mark.parametrize("seg", [-1, 16, 64, 256])
@pytest.mark.parametrize("single_reduction", [0, 1])
def test_chunk_shapes_solve_to_the_direct_solution(mf, seg_problem, seg, single_reduction):
    k, p = seg_problem
    g, _, b = gpu_problem(mf, k, c=1e-3)
    mf.set_launch(g, 4, 1, seg)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.double(), x, mf.default_opts(
        tol=1e-10, precision=mf.FP32_IR, single_reduction=single_reduction))
    assert st == mf.OK and info["single_reduction"] == single_reduction
    assert np.linalg.norm(host(x) - p) <= 1e-8 * np.linalg.norm(p)


def test_autotune_caches_and_keeps_results(mf, tmp_path):
    shape = (48, 32, 64)
    k = lognormal_iid(shape, 1.0, 3)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    cache = str(tmp_path / "tune.json")
    r1 = mf.autotune(g, cache)
    assert r1["candidates"] >= 4 and r1["apply_us"] > 0
    data = json.load(open(cache))
    assert len(data) == 1 and list(data.values())[0]["ci"] == r1["ci"]
    g2, _, _ = gpu_problem(mf, k, c=1e-3)
    r2 = mf.autotune(g2, cache)
    keys = ("ci", "remap", "seg", "apply_ci", "apply_remap", "apply_seg", "apply_blocks")
    assert r2["candidates"] == 0 and all(r2[k] == r1[k] for k in keys)
    assert r1["seg"] in (-1, 32) and r1["apply_seg"] in (-1, 32)
    # the apply runs at its own tuned shape and still equals the default shape's bits
    xa = torch.randn(k.size, dtype=torch.float32, device="cuda")
    ya, yb = torch.empty_like(xa), torch.empty_like(xa)
    mf.apply(g2, xa, ya)
    mf.set_launch(g2, 0, 1, 0)
    mf.apply(g2, xa, yb)
    assert torch.equal(ya, yb)
    x = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.double(), x, mf.default_opts(tol=1e-10, precision=mf.FP32_IR))
    assert st == mf.OK
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 1e-8 * np.linalg.norm(p)


def test_autotune_batched_keeps_results(mf):
    rng = np.random.default_rng(9)
    shapes = [tuple(int(v) for v in rng.integers(8, 30, 3)) for _ in range(6)]
    ks = [lognormal_iid(s, 1.0, i) for i, s in enumerate(shapes)]
    probs = [gpu_problem(mf, k, c=1e-3) for k in ks]
    grids = [p[0] for p in probs]
    bs = [p[2] for p in probs]
    xs = [torch.zeros(g.n, dtype=torch.float32, device="cuda") for g in grids]
    best = mf.autotune_batched(grids, bs, xs, mf.default_opts(tol=1e-6, use_graph=0))
    assert best["ms"] > 0 and best["items_per_block"] in (1, 2, 4, 8, 16)
    for x in xs:
        x.zero_()
    st, infos = mf.cg_solve_batched(grids, bs, xs, mf.default_opts(tol=1e-6, use_graph=0))
    assert st == mf.OK
    for k, x in zip(ks, xs):
        ref = OracleProblem(k, c=1e-3)
        p = ref.direct()
        assert np.linalg.norm(host(x) - p) <= 5e-5 * np.linalg.norm(p)
    mf.set_batched_launch(0, 4)


def test_kernel_timing_keeps_results(mf):
    shape = (40, 24, 64)
    k = lognormal_iid(shape, 1.0, 5)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    xs = []
    for timing in (0, 1):
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, timing=timing))
        assert st == mf.OK
        xs.append(host(x))
        if timing:
            assert info["timed_iters"] == min(32, info["iters"])
            assert info["phase_a_us"] > 0 and info["phase_b_us"] >= 0 and info["precond_us"] >= 0
            assert info["phase_b_us"] > 0 or info["single_reduction"] == 1
            assert info["phase_a_us"] < info["ms"] * 1e3
        else:
            assert info["timed_iters"] == 0 and info["phase_a_us"] == 0
    assert np.array_equal(xs[0], xs[1])
