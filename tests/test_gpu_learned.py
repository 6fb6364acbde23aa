"""Learned preconditioner on the GPU against the network oracle, and flexible
CG with it: forward and gradients match the oracle to BF16 tolerance, a zero
network is Jacobi-PCG, a harmful network is caught by the safeguard, and a
trained network reduces the iteration count of flexible CG."""
import numpy as np
import pytest

from oracle import krylov, nn, tpfa
from synth import channelised, lognormal_iid
from gpu_problem import gpu_problem, OracleProblem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available()
    mffv.lib()
    return mffv


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda", dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def random_params(seed):
    rng = np.random.default_rng(seed)
    p = nn.init_params(seed=seed, last_scale=0.7).astype(np.float64)
    layers = nn.unpack(p)
    layers = [(W, rng.normal(0, 0.1, size=b.shape)) for W, b in layers]
    return nn.pack(layers).astype(np.float32)


SHAPE = (6, 10, 70)   # two z tiles (one ragged), ragged y tiles


def test_forward_matches_oracle(mf):
    rng = np.random.default_rng(1)
    p = random_params(2)
    r = rng.normal(size=SHAPE).astype(np.float32)
    f = rng.normal(size=SHAPE).astype(np.float32)
    net = mf.net_create(p)
    out = torch.empty(r.size, dtype=torch.float32, device="cuda")
    mf.nn_forward(net, SHAPE, dev(r), dev(f), out)
    torch.cuda.synchronize()
    ref, _, _ = nn.forward(p, r.astype(np.float64), f.astype(np.float64), bf16=True)
    got = host(out).reshape(SHAPE)
    assert np.linalg.norm(got - ref) <= 1e-2 * np.linalg.norm(ref)
    assert np.max(np.abs(got - ref)) <= 5e-2 * np.max(np.abs(ref))
    pb, _ = mf.net_get_params(net)
    assert np.array_equal(pb, p)


def oracle_feature(ref):
    d = ref.diag()
    u = ~ref.dmask.ravel()
    ld = np.log(d)
    return np.where(u, ld - ld[u].mean(), 0.0).reshape(ref.shape)


@pytest.mark.parametrize("relu", [True, False])
def test_gradients_match_oracle(mf, relu):
    rng = np.random.default_rng(3)
    p = random_params(4)
    k = lognormal_iid(SHAPE, 1.0, 6)
    g, _, _ = gpu_problem(mf, k, c=1e-2)
    ref = OracleProblem(k, c=1e-2)
    dmask = ref.dmask
    r = np.where(dmask, 0, rng.normal(size=SHAPE)).astype(np.float32)
    tgt = np.where(dmask, 0, rng.normal(size=SHAPE) + 0.5 * r).astype(np.float32)
    net = mf.net_create(p)
    mf.net_set_activation(net, relu)
    loss = mf.nn_loss_grad(net, g, dev(r), dev(tgt))
    _, grad = mf.net_get_params(net)
    ref_loss, ref_g, _ = nn.loss_and_grads(p, r.astype(np.float64), oracle_feature(ref),
                                           tgt.astype(np.float64), dmask,
                                           nn.scaled_operator(ref.A, dmask), relu=relu)
    assert abs(loss - ref_loss) <= 1e-2 * abs(ref_loss)
    o = 0
    for ci, co, _ in nn.LAYERS:
        for size in (27 * ci * co, co):
            a_, b_ = grad[o:o + size].astype(np.float64), ref_g[o:o + size]
            assert np.linalg.norm(a_ - b_) <= 3e-2 * np.linalg.norm(b_) + 1e-6, (o, size)
            o += size
    assert o == nn.n_params()


def test_feature_and_harvest_match_oracle(mf):
    shape = (10, 12, 16)
    k = channelised(shape, 7)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    feat = torch.empty(k.size, dtype=torch.float32, device="cuda")
    mf.grid_feature(g, feat)
    assert np.allclose(host(feat), oracle_feature(ref).ravel(), atol=1e-5, rtol=0)
    # a pair from a truncated Jacobi-PCG iterate, in the Jacobi-scaled space
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    mf.cg_solve(g, b, x, mf.default_opts(max_iter=5, tol=1e-12, precond=mf.PRECOND_JACOBI))
    xstar = torch.from_numpy(ref.direct()).cuda()
    rh, tg = (torch.empty(k.size, dtype=torch.float32, device="cuda") for _ in range(2))
    s = mf.harvest_pair(g, b, x, xstar, rh, tg)
    xh = host(x)
    u = ~ref.dmask.ravel()
    d = ref.diag()
    r = np.where(u, ref.b - ref.A @ xh, 0.0)
    s_ref = np.sqrt(np.sum(r * r / d) / u.sum())
    assert abs(s - s_ref) <= 1e-5 * s_ref
    want_r = r / np.sqrt(d) / s_ref
    want_t = np.where(u, (ref.direct() - xh) * np.sqrt(d), 0.0) / s_ref
    assert np.allclose(host(rh), want_r, rtol=0, atol=1e-4 * np.abs(want_r).max())
    assert np.allclose(host(tg), want_t, rtol=0, atol=1e-4 * np.abs(want_t).max())
    # consistency of the pair: A~ target = r_hat
    As = nn.scaled_operator(ref.A, ref.dmask)
    assert np.allclose(As(host(tg).reshape(shape)).ravel()[u], host(rh)[u], rtol=0,
                       atol=1e-3 * np.abs(want_r).max())


def test_fcg_with_zero_network_is_jacobi_pcg(mf):
    """Without the Jacobi sweeps (nn_smooth = 0) the zero network is Jacobi-PCG."""
    shape = (24, 24, 24)
    k = channelised(shape, 11)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    net = mf.net_create(nn.init_params(seed=0, last_scale=0.0))
    xj = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, ij = mf.cg_solve(g, b, xj, mf.default_opts(precond=mf.PRECOND_JACOBI))
    xf = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st2, iff = mf.cg_solve(g, b, xf, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_smooth=0.0))
    assert st == st2 == mf.OK
    assert abs(ij["iters"] - iff["iters"]) <= 2 and iff["fallbacks"] == 0
    ref = OracleProblem(k, c=1e-3)
    p = ref.direct()
    assert np.linalg.norm(host(xf) - p) <= 5e-5 * np.linalg.norm(p)
    # and the oracle's flexible CG with the Jacobi preconditioner agrees on the count
    orc = krylov.fcg(ref.Auu, ref.bu, krylov.jacobi(ref.Auu), tol=1e-6, max_iter=5000)
    assert abs(iff["iters"] - orc.iters) <= max(3, orc.iters // 20)


def harmful_params(c):
    """A network whose output is -c * r_hat: z = (1 - c) r / d, so z.r < 0 for c > 1."""
    layers = [(np.zeros((27, ci, co)), np.zeros(co)) for ci, co, _ in nn.LAYERS]
    layers[0][0][13, 0, 0], layers[0][0][13, 0, 1] = 1.0, -1.0     # relu(r), relu(-r)
    for li in (1, 2):
        layers[li][0][13, 0, 0] = layers[li][0][13, 1, 1] = 1.0
    layers[3][0][13, 0, 0], layers[3][0][13, 1, 0] = -c, c
    return nn.pack(layers).astype(np.float32)


@pytest.mark.parametrize("every", [2, 3])
def test_network_every_kth_iteration(mf, every):
    """opts.nn_every: the network preconditions every k-th iteration and the
    Jacobi step the others. With a network whose output is a scaled Jacobi step
    (z = 0.5 r / d) every iteration's z is a multiple of r / d, so flexible CG
    takes the same directions as Jacobi-PCG (up to scale) and needs the same
    count; with the zero network it is Jacobi-PCG outright."""
    shape = (24, 24, 24)
    k = channelised(shape, 11)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    p = ref.direct()
    xj = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, ij = mf.cg_solve(g, b, xj, mf.default_opts(precond=mf.PRECOND_JACOBI))
    assert st == mf.OK
    for params in (nn.init_params(seed=0, last_scale=0.0), harmful_params(0.5)):
        net = mf.net_create(params)
        for use_graph in (1, 0):
            xf = torch.zeros(k.size, dtype=torch.float32, device="cuda")
            st, info = mf.cg_solve(g, b, xf, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net,
                                                             nn_every=every, use_graph=use_graph,
                                                             nn_smooth=0.0))
            assert st == mf.OK and info["fallbacks"] == 0
            assert abs(info["iters"] - ij["iters"]) <= max(2, ij["iters"] // 50)
            assert np.linalg.norm(host(xf) - p) <= 5e-5 * np.linalg.norm(p)
    with pytest.raises(mf.MffvError):
        mf.cg_solve(g, b, xj, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_every=0))


def test_safeguard_falls_back_to_jacobi(mf):
    shape = (16, 16, 16)
    k = lognormal_iid(shape, 1.0, 4)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    net = mf.net_create(harmful_params(8.0))
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_smooth=0.0))
    assert st == mf.OK
    # every iteration rejected the network's z (the final convergence check
    # does not consume a preconditioned residual)
    assert info["fallbacks"] == info["iters"]
    xj = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    _, ij = mf.cg_solve(g, b, xj, mf.default_opts(precond=mf.PRECOND_JACOBI))
    assert abs(info["iters"] - ij["iters"]) <= 2
    p = ref.direct()
    assert np.linalg.norm(host(x) - p) <= 5e-5 * np.linalg.norm(p)


def test_training_gains_over_the_zero_network(mf):
    # held-in 32^3 channelised systems: train with the library's recipe, then
    # compare flexible CG with the trained network against the same solver with
    # the zero network (Jacobi-PCG) and against plain CG on held-out fields
    import time
    from paper_2408_03452_amd import learned
    shape = (32, 32, 32)
    held_in = [gpu_problem(mf, channelised(shape, seed), c=1e-3) for seed in range(3000, 3008)]
    systems = [(g, b) for g, _, b in held_in]
    # validation pairs from Jacobi-PCG iterates (energy loss of the zero net)
    pairs = learned.harvest(*systems[0])
    zero = mf.net_create(learned.init_params(0))
    net = learned.train_preconditioner(systems, validation=systems[:2], n_white=256, epochs=16,
                                       dagger_rounds=1, log=print)
    l0, l1 = learned.evaluate_loss(zero, pairs), learned.evaluate_loss(net, pairs)
    res = {}
    for seed in (3500, 3501):
        g, _, b = gpu_problem(mf, channelised(shape, seed), c=1e-3)
        for name, opts in (("zero", mf.default_opts(precond=mf.PRECOND_LEARNED, net=zero)),
                           ("trained", mf.default_opts(precond=mf.PRECOND_LEARNED, net=net)),
                           ("plain", mf.default_opts())):
            x = torch.zeros(g.n, dtype=torch.float32, device="cuda")
            mf.cg_solve(g, b, x, opts)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, info = mf.cg_solve(g, b, x, opts)
            torch.cuda.synchronize()
            assert st == mf.OK and info["rel_res_recursive"] <= 1e-6
            res.setdefault(name, []).append((info["iters"], time.perf_counter() - t0))
    print(f"\n[learned] validation energy loss zero-net {l0:.4f} trained {l1:.4f}; "
          f"held-out (iters, s): {res}")
    assert l1 < l0
    for (iz, _), (it, tt), (ip, tp) in zip(res["zero"], res["trained"], res["plain"]):
        # the zero network between the Jacobi sweeps is a polynomial
        # preconditioner; the trained network cuts iterations below it
        assert it < 0.9 * iz
        assert tt < tp                # and beats plain CG in time to 1e-6


def test_finetuning_starts_from_the_given_network(mf):
    """train_preconditioner(init=...) continues from a given network, and that
    network is the first candidate of the epoch selection: the result never
    takes more flexible-CG iterations on the validation systems than it."""
    from paper_2408_03452_amd import learned
    shape = (16, 16, 16)
    systems = [gpu_problem(mf, channelised(shape, seed), c=1e-3) for seed in (3000, 3001, 3002)]
    systems = [(g, b) for g, _, b in systems]
    start = learned.train_preconditioner(systems, validation=systems[:2], n_white=12, epochs=2,
                                         dagger_rounds=0)
    p_start, _ = mf.net_get_params(start)
    it_start = learned.fcg_iterations(start, systems[:2])
    tuned = learned.train_preconditioner(systems, validation=systems[:2], n_white=12, epochs=1,
                                         lr=1e-3, dagger_rounds=0, init=p_start)
    assert learned.fcg_iterations(tuned, systems[:2]) <= it_start
    # with no epoch better than the start, the start comes back unchanged
    same = learned.train_preconditioner(systems, validation=systems[:2], n_white=4, epochs=1,
                                        lr=1e-12, lr_final=1e-12, dagger_rounds=0, init=p_start)
    assert np.array_equal(mf.net_get_params(same)[0], p_start)


def test_new_network_after_a_destroyed_one_is_used(mf):
    """A solve captures its iterations in a graph keyed by the network. After
    that network is destroyed, a new network (whose handle may land at the
    same address) must be the one applied: solving the same grid again gives
    exactly what a fresh grid gives with the new network."""
    shape = (20, 22, 24)
    k = channelised(shape, 12)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    p_old = nn.init_params(seed=5, last_scale=0.2)
    p_new = harmful_params(0.5)          # z = 0.5 r / d: the directions of Jacobi-PCG
    for _ in range(3):
        old = mf.net_create(p_old)
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st, _ = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=old))
        assert st == mf.OK
        old.close()
        new = mf.net_create(p_new)
        x.zero_()
        st, info = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=new))
        assert st == mf.OK
        g2, _, b2 = gpu_problem(mf, k, c=1e-3)
        x2 = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st2, info2 = mf.cg_solve(g2, b2, x2, mf.default_opts(precond=mf.PRECOND_LEARNED, net=new))
        assert st2 == mf.OK and info["iters"] == info2["iters"]
        assert torch.equal(x, x2)
        g2.close()
        new.close()
    g.close()


@pytest.mark.parametrize("omega", [0.5, 0.8])
def test_zero_network_between_the_sweeps_is_the_polynomial_pcg(mf, omega):
    """With the zero network the sandwich preconditioner is the fixed SPD
    polynomial of three damped Jacobi steps: flexible CG takes the oracle's
    PCG iteration count with that polynomial (oracle.nn.learned_preconditioner
    with zero parameters), and the refined field matches the direct solve."""
    shape = (24, 24, 24)
    k = channelised(shape, 13)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    zero = nn.init_params(seed=0, last_scale=0.0)
    net = mf.net_create(zero)
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_smooth=omega))
    assert st == mf.OK and info["fallbacks"] == 0
    M = nn.learned_preconditioner(zero, ref.A, ref.dmask, np.zeros(shape), omega=omega)
    orc = krylov.pcg(ref.Auu, ref.bu, M, tol=1e-6, max_iter=5000)
    jac = krylov.pcg(ref.Auu, ref.bu, krylov.jacobi(ref.Auu), tol=1e-6, max_iter=5000)
    print(f"\n[learned] polynomial PCG (w {omega}): GPU {info['iters']}, oracle {orc.iters}, Jacobi {jac.iters}")
    assert orc.converged and orc.iters < jac.iters
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 20)
    x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, _ = mf.cg_solve_f64(g, b.double(), x64, mf.default_opts(
        tol=1e-9, precision=mf.FP32_IR, precond=mf.PRECOND_LEARNED, net=net, nn_smooth=omega))
    assert st == mf.OK
    p = ref.direct()
    assert np.linalg.norm(x64.cpu().numpy() - p) <= 1e-6 * np.linalg.norm(p)
    with pytest.raises(mf.MffvError):
        mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_smooth=2.0))


def test_smooth_sample_matches_the_oracle(mf):
    """mffv_nn_smooth_sample: (I - omega A~) r_hat on the unknown cells and 0 on
    Dirichlet cells, A~ = D^-1/2 A D^-1/2, against the oracle's assembled
    operator in FP64 (FP32 tolerance)."""
    shape = (21, 17, 19)
    k = lognormal_iid(shape, 1.0, 5)
    g, _, _ = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    rng = np.random.default_rng(8)
    rh = rng.standard_normal(k.size).astype(np.float32)
    out = torch.empty(k.size, dtype=torch.float32, device="cuda")
    for omega in (0.5, 0.0, 1.5):
        mf.nn_smooth_sample(g, omega, dev(rh), out)
        torch.cuda.synchronize()
        d = ref.A.diagonal()
        u = ~ref.dmask.ravel()
        x = np.where(u, rh.astype(np.float64), 0.0)
        want = x - omega * (ref.A @ (x / np.sqrt(d))) / np.sqrt(d)
        want[~u] = 0.0
        got = host(out)
        assert np.all(got[~u] == 0.0)
        assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want)), omega
    with pytest.raises(mf.MffvError):   # the weight lies in [0, 2)
        mf.nn_smooth_sample(g, 2.0, dev(rh), out)
    g.close()


def test_power_of_two_scaled_right_hand_side_scales_the_solve_exactly(mf):
    """The network's input scale is a power of two (the power of two nearest
    the residual's D^-1-weighted RMS), the first sweep writes the unscaled BF16
    input and the first convolution multiplies its products by 1/s. Every step
    of flexible CG with this preconditioner is then exactly equivariant under
    b -> 2^k b, even with a network whose biases are nonzero (which is not
    homogeneous): the solve takes the same iterations and returns exactly
    2^k x, in FP32 and with the FP64 refinement."""
    shape = (24, 20, 28)
    k = channelised(shape, 17)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    net = mf.net_create(random_params(18))
    base = None
    for kk in (0, -7, 5):
        bs = b * (2.0 ** kk)
        x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
        st, info = mf.cg_solve(g, bs, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, tol=1e-6))
        x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
        st64, info64 = mf.cg_solve_f64(g, bs.double(), x64, mf.default_opts(
            tol=1e-8, precision=mf.FP32_IR, precond=mf.PRECOND_LEARNED, net=net))
        assert st == mf.OK and st64 == mf.OK
        got = (info["iters"], host(x) / 2.0 ** kk, info64["iters"], x64.cpu().numpy() / 2.0 ** kk)
        if base is None:
            base = got
            continue
        assert got[0] == base[0] and got[2] == base[2]
        assert np.array_equal(got[1], base[1]) and np.array_equal(got[3], base[3])
    net.close()
    g.close()


def test_learned_solve_does_not_depend_on_the_host_poll_chunk(mf):
    """Iterations enqueued past convergence (the host polls the loop state one
    chunk behind) find the loop's done flag set, and every kernel of the
    preconditioner then returns at once: the solve's result and iteration
    count are exactly those of a run polled after every iteration."""
    shape = (22, 26, 20)
    k = channelised(shape, 19)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    net = mf.net_create(random_params(20))
    runs = []
    for every in (1, 5, 16, 64):
        for max_iter in (7, 100000):
            x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
            st, info = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, tol=1e-6,
                                                            check_every=every, max_iter=max_iter))
            assert st == (mf.NOT_CONVERGED if max_iter == 7 else mf.OK)
            runs.append((every, max_iter, info["iters"], host(x)))
    for every, max_iter, iters, x in runs:
        ref = next(r for r in runs if r[0] == 1 and r[1] == max_iter)
        assert iters == ref[2], (every, max_iter)
        assert np.array_equal(x, ref[3]), (every, max_iter)
    net.close()
    g.close()
