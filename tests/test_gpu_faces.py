"""Face-list (unstructured) grids through the C ABI against the oracle's
face-list operator: apply in FP32 and FP64, CG / Jacobi-PCG / refined
solves, a Cartesian grid written as a face list against the Cartesian path,
closed-form small cases and argument errors."""
import numpy as np
import pytest

from oracle import faces, krylov, tpfa
from synth import cartesian_faces, lognormal_iid, random_face_mesh
from gpu_problem import gpu_problem

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


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).ravel()).cuda()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def mesh_case(shape, seed, n_dirichlet=10):
    n, fk, fl, T = random_face_mesh(shape, seed, drop=0.1, extra=0.05)
    rng = np.random.default_rng(seed + 100)
    c = f32(rng.uniform(0.01, 0.05, n))
    dmask = np.zeros(n, dtype=bool)
    dmask[rng.choice(n, n_dirichlet, replace=False)] = True
    pd = f32(np.where(dmask, rng.uniform(-1.0, 2.0, n), 0.0))
    return n, fk, fl, f32(T), c, dmask, pd


def face_grid(mf, n, fk, fl, T, c, dmask, pd, s):
    g = mf.create_grid_faces(n, fk, fl, stream=s)
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    mf.set_face_transmissibility(g, dev(T), accum=dev(c), dmask=dev(dmask, np.uint8), pD=dev(pd), b_out=b)
    return g, b


def test_face_apply_matches_oracle(mf):
    n, fk, fl, T, c, dmask, pd = mesh_case((9, 8, 7), 1)
    A, b_ref = faces.assemble_faces(n, fk, fl, T, c, dmask, pd)
    x = f32(np.random.default_rng(2).standard_normal(n))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, b = face_grid(mf, n, fk, fl, T, c, dmask, pd, s)
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        mf.apply(g, dev(x), y)
        y64 = torch.empty(n, dtype=torch.float64, device="cuda")
        mf.apply_f64(g, dev(x, np.float64), y64)
        got, got64, gb = host(y), host(y64), host(b)
    want = A @ x
    scale = abs(A) @ np.abs(x)
    assert np.all(np.abs(got - want) <= 32 * 2.0 ** -24 * scale + 1e-30)
    assert np.all(np.abs(got64 - want) <= 1e-14 * scale + 1e-300)
    assert np.allclose(gb, b_ref, rtol=4 * 2.0 ** -24, atol=1e-30)
    assert np.array_equal(got[dmask], x[dmask])


@pytest.mark.parametrize("precond", [0, 1])
def test_face_cg_matches_oracle(mf, precond):
    n, fk, fl, T, c, dmask, pd = mesh_case((14, 12, 10), 3, n_dirichlet=20)
    A, b_ref = faces.assemble_faces(n, fk, fl, T, c, dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, b_ref, dmask)
    import scipy.sparse.linalg as spla
    p = tpfa.scatter_solution(spla.spsolve(Auu.tocsc(), bu), u, pd, dmask)
    M = krylov.jacobi(Auu) if precond else None
    orc = krylov.pcg(Auu.astype(np.float32), bu.astype(np.float32), M, tol=1e-6, max_iter=20000,
                     dtype=np.float32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, b = face_grid(mf, n, fk, fl, T, c, dmask, pd, s)
        x = torch.zeros(n, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(g, b, x, mf.default_opts(tol=1e-6, precond=precond))
        assert st == mf.OK and info["single_reduction"] == 0
        x2 = torch.zeros(n, dtype=torch.float32, device="cuda")
        st2, info2 = mf.cg_solve(g, b, x2, mf.default_opts(tol=1e-9, precond=precond,
                                                           precision=mf.FP32_IR))
        xr = host(x2)
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 10), (info["iters"], orc.iters)
    assert st2 == mf.OK and info2["rel_res_true"] <= 1e-9
    assert np.linalg.norm(xr - p) <= 1e-5 * np.linalg.norm(p)
    assert np.array_equal(xr[dmask], pd[dmask])


def test_cartesian_grid_as_faces_matches_cartesian_path(mf):
    """The same 12x10x8 problem through the Cartesian kernels and through the
    face-list kernels (faces taken from the Cartesian grid's own device
    transmissibilities): both refined solutions match the oracle and each other."""
    shape = (12, 10, 8)
    k = lognormal_iid(shape, 1.5, 21)
    n = k.size
    fk, fl, ax = cartesian_faces(shape)
    s = torch.cuda.Stream()
    opts = mf.default_opts(tol=1e-9, precision=mf.FP32_IR)
    with torch.cuda.stream(s):
        g, (tx, ty, tz), b = gpu_problem(mf, k, c=1e-3, stream=s)
        xc = torch.zeros(n, dtype=torch.float32, device="cuda")
        st, _ = mf.cg_solve(g, b, xc, opts)
        assert st == mf.OK
        fk_t = torch.from_numpy(fk).cuda()
        ax_t = torch.from_numpy(ax.astype(np.int64)).cuda()
        T = torch.where(ax_t == 0, tx[fk_t], torch.where(ax_t == 1, ty[fk_t], tz[fk_t])).contiguous()
        dmask, pd = tpfa.x_plane_dirichlet(shape)
        gf = mf.create_grid_faces(n, fk, fl, stream=s)
        bf = torch.empty(n, dtype=torch.float32, device="cuda")
        mf.set_face_transmissibility(gf, T, accum_scalar=1e-3, dmask=dev(dmask, np.uint8), pD=dev(pd), b_out=bf)
        xf = torch.zeros(n, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(gf, bf, xf, opts)
        assert st == mf.OK
        hc, hf, hb, hbf = host(xc), host(xf), host(b), host(bf)
    assert np.array_equal(hb, hbf)       # each right-hand side entry is one product T * p^D
    Tx, Ty, Tz = tpfa.round_to_f32(*tpfa.transmissibility(k))
    A, bo = tpfa.assemble(Tx, Ty, Tz, np.float64(np.float32(1e-3)), dmask, pd)
    Auu, bu, u = tpfa.reduce_to_unknowns(A, bo, dmask)
    import scipy.sparse.linalg as spla
    p = tpfa.scatter_solution(spla.spsolve(Auu.tocsc(), bu), u, pd, dmask)
    for x in (hc, hf):
        assert np.linalg.norm(x - p) <= 2e-6 * np.linalg.norm(p)
    assert np.linalg.norm(hc - hf) <= 2e-6 * np.linalg.norm(p)


def test_face_closed_forms(mf):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # one cell, no face: the operator is c
        g1 = mf.create_grid_faces(1, [], [], stream=s)
        mf.set_face_transmissibility(g1, None, accum_scalar=2.5)
        y = torch.empty(1, dtype=torch.float32, device="cuda")
        mf.apply(g1, dev([3.0]), y)
        assert host(y)[0] == 7.5
        # two cells, one face, cell 0 Dirichlet: p_1 = T p^D / (c + T)
        g2 = mf.create_grid_faces(2, [0], [1], stream=s)
        b = torch.empty(2, dtype=torch.float32, device="cuda")
        mf.set_face_transmissibility(g2, dev([4.0]), accum_scalar=1.0, dmask=dev([1, 0], np.uint8),
                                     pD=dev([2.5, 0.0]), b_out=b)
        x = torch.zeros(2, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(g2, b, x, mf.default_opts(tol=1e-7))
        hx = host(x)
    assert st == mf.OK and 1 <= info["iters"] <= 2
    assert hx[0] == 2.5 and abs(hx[1] - 4.0 * 2.5 / 5.0) <= 1e-6


def test_face_argument_errors(mf):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with pytest.raises(mf.MffvError):
            mf.create_grid_faces(4, [0, 1], [1, 1], stream=s)          # a face joins a cell to itself
        with pytest.raises(mf.MffvError):
            mf.create_grid_faces(4, [0, 1], [1, 4], stream=s)          # cell out of range
        with pytest.raises(mf.MffvError):
            mf.create_grid_faces(0, [], [], stream=s)
        g = mf.create_grid_faces(4, [0, 1, 2], [1, 2, 3], stream=s)
        T = dev([1.0, 2.0, 3.0])
        with pytest.raises(mf.MffvError):
            mf.set_face_transmissibility(g, dev([1.0, -2.0, 3.0]), accum_scalar=1.0)   # negative T
        with pytest.raises(mf.MffvError):
            mf.set_face_transmissibility(g, T, accum_scalar=0.0)       # singular: no D, no c
        with pytest.raises(mf.MffvError):
            mf.set_face_transmissibility(g, T, accum_scalar=1.0, dmask=dev([1, 1, 1, 1], np.uint8))
        mf.set_face_transmissibility(g, T, accum_scalar=1.0, dmask=dev([1, 0, 0, 0], np.uint8))
        t4 = torch.zeros(4, dtype=torch.float32, device="cuda")
        with pytest.raises(mf.MffvError):
            mf.set_transmissibility(g, t4, t4, t4, accum_scalar=1.0)  # the Cartesian set-up
        with pytest.raises(mf.MffvError):
            mf.set_launch(g, 2, 1)
        with pytest.raises(mf.MffvError):
            mf.autotune(g, None)
        with pytest.raises(mf.MffvError):
            mf.cg_solve_batched([g], [t4], [torch.zeros_like(t4)])
        # a Cartesian grid refuses the face-list set-up
        k = lognormal_iid((4, 3, 2), 1.0, 1)
        gc, _, _ = gpu_problem(mf, k, stream=s)
        with pytest.raises(mf.MffvError):
            mf.set_face_transmissibility(gc, T, accum_scalar=1.0)
    s.synchronize()


def test_face_time_steps_match_oracle(mf):
    """Backward-Euler steps with a well on a face-list mesh: each step against
    the oracle's face-list operator (accumulation c + WI) solved directly."""
    n, fk, fl, T, c, dmask, pd = mesh_case((10, 9, 8), 7, n_dirichlet=15)
    rng = np.random.default_rng(8)
    wi = np.zeros(n)
    pw = np.zeros(n)
    wells = rng.choice(np.flatnonzero(~dmask), 3, replace=False)
    wi[wells] = [0.5, 1.0, 1.5]
    pw[wells] = [3.0, -1.0, 2.0]
    q = np.zeros(n)
    q[rng.choice(np.flatnonzero(~dmask), 2, replace=False)] = [0.25, -0.125]
    p0 = f32(np.where(dmask, pd, rng.uniform(0.0, 1.0, n)))
    from oracle import timestep
    import scipy.sparse.linalg as spla
    A, b_ref = faces.assemble_faces(n, fk, fl, T, f32(c + wi), dmask, pd)   # the FP32 accumulation the GPU gets
    Auu, _, u = tpfa.reduce_to_unknowns(A, b_ref, dmask)
    want, p = [], p0
    for _ in range(3):
        rhs = timestep.step_rhs(b_ref, c, p, dmask, wi, pw, q)
        p = tpfa.scatter_solution(spla.spsolve(Auu.tocsc(), rhs[u]), u, pd, dmask)
        want.append(p)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g, b = face_grid(mf, n, fk, fl, T, c + wi, dmask, pd, s)
        pt = dev(p0)
        got = []
        for _ in range(3):
            st, infos = mf.time_steps(g, 1, b, pt, c=dev(c), wi=dev(wi), pw=dev(pw), q=dev(q),
                                      opts=mf.default_opts(precision=mf.FP32_IR, tol=1e-9))
            assert st == mf.OK
            got.append(host(pt))
    for k, (gp, wp) in enumerate(zip(got, want)):
        assert np.max(np.abs(gp - wp)) <= 1e-5 * np.max(np.abs(wp)), k
