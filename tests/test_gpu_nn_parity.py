"""Element-wise parity of the learned preconditioner's kernels with the
network oracle, through the C ABI.

* Integer-valued cases (tests/nn_cases.py) are exact in FP32, so the forward
  pass, the loss and every parameter gradient must equal the oracle bit for
  bit, for each march length of the convolutions (planes per block: one, a
  few with a ragged tail, the whole grid), so that the LDS ring of the march
  wraps and its prefetch lands in reused slots.
* Adam: K training steps, each compared with the oracle's Adam on the
  gradients the GPU computed.
* Every loss kind on a TPFA operator with neighbour coupling and an exact
  Jacobi scaling, bit for bit.
* Flexible CG with a fixed random network against the oracle's flexible CG
  with the oracle network as the preconditioner.
"""
import numpy as np
import pytest

import nn_cases
from gpu_problem import OracleProblem, gpu_problem
from oracle import krylov, nn
from synth import channelised

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available()
    mffv.lib()
    yield mffv
    mffv.set_nn_run(0)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda", dtype)


def identity_grid(mf, shape):
    """A grid whose operator is the identity on every cell (no faces,
    accumulation 1, x-plane Dirichlet cells): A~ = I on the unknown cells."""
    n = int(np.prod(shape))
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = mf.create_grid(*shape)
    mf.set_transmissibility(g, z, z, z, accum_scalar=1.0)
    return g


@pytest.fixture(scope="module")
def forward_ref():
    p, r, f = nn_cases.forward_case()
    out, _, _ = nn.forward(p, r, f)
    return p, r, f, out


@pytest.mark.parametrize("run", (0,) + nn_cases.RUNS)
def test_forward_is_bit_exact_at_every_march_length(mf, forward_ref, run):
    p, r, f, ref = forward_ref
    print(f"[nn-parity] forward {nn_cases.SHAPE} run {run}", flush=True)
    mf.set_nn_run(run)
    net = mf.net_create(p)
    out = torch.full((r.size,), np.nan, dtype=torch.float32, device="cuda")
    mf.nn_forward(net, nn_cases.SHAPE, dev(r), dev(f), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(nn_cases.SHAPE).astype(np.float64)
    bad = np.argwhere(got != ref)
    assert bad.size == 0, f"{len(bad)} cells differ, first {bad[:5].tolist()}"
    net.close()


@pytest.fixture(scope="module")
def gradient_refs():
    p, r, f, dmask = nn_cases.gradient_case()
    refs = {}
    for kind, with_t in ((0, False), (1, False), (0, True)):
        t = r if with_t else None
        loss, g, _ = nn.loss_and_grads(p, r, f, t, dmask, nn_cases.identity_operator, kind=kind)
        refs[(kind, with_t)] = (loss, g)
    return p, r, refs


@pytest.mark.parametrize("run", (0, 3, 37))
@pytest.mark.parametrize("kind,with_target", [(0, False), (1, False), (0, True)])
def test_loss_and_gradient_are_bit_exact(mf, gradient_refs, kind, with_target, run):
    p, r, refs = gradient_refs
    print(f"[nn-parity] loss kind {kind} target {with_target} run {run}", flush=True)
    mf.set_nn_run(run)
    g = identity_grid(mf, nn_cases.SHAPE)
    net = mf.net_create(p)
    mf.net_set_loss(net, kind)
    rd = dev(r)
    loss = mf.nn_loss_grad(net, g, rd, rd if with_target else None)
    _, grad = mf.net_get_params(net)
    ref_loss, ref_g = refs[(kind, with_target)]
    assert loss == ref_loss
    bad = np.flatnonzero(grad.astype(np.float64) != ref_g)
    assert bad.size == 0, f"{bad.size} gradient entries differ, first {bad[:8].tolist()}"
    net.close()
    g.close()


def test_adam_steps_match_the_oracle(mf, gradient_refs):
    """K steps of mffv_nn_train_step; after each, the oracle's Adam applied to
    the gradient the GPU computed (biases frozen) must give the same
    parameters, to FP32 rounding of the update."""
    p, r, _ = gradient_refs
    mf.set_nn_run(0)
    g = identity_grid(mf, nn_cases.SHAPE)
    net = mf.net_create(p)
    rd = dev(r)
    frozen = nn.bias_mask()
    po = p.astype(np.float64)
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    lr = 0.05
    moved = 0
    for step in range(1, 6):
        mf.nn_train_step(net, g, rd, None, lr)
        pg, gg = mf.net_get_params(net)
        po, m, v = nn.adam(po, gg.astype(np.float64), m, v, step, lr=lr, frozen=frozen)
        err = np.abs(pg.astype(np.float64) - po)
        tol = 4e-7 * np.abs(po) + step * 4e-6 * lr
        assert np.all(err <= tol), (step, int(np.argmax(err - tol)), float(np.max(err - tol)))
        assert np.array_equal(pg[frozen], p[frozen])
        moved = np.count_nonzero(pg != p)
    assert moved > 0.5 * (~frozen).sum()
    net.close()
    g.close()


@pytest.mark.parametrize("kind,with_target", [(0, False), (1, False), (0, True)])
def test_every_loss_kind_on_a_tpfa_operator_is_bit_exact(mf, kind, with_target):
    """The integer network and spikes on a TPFA operator with neighbour
    coupling whose Jacobi scaling is exact (tests/nn_cases.py): every loss
    kind's output gradient is dyadic, so the parameter gradient must equal the
    oracle's bit for bit; the loss itself (a sum over cells in FP32) to 1e-6."""
    p, r, f, dmask = nn_cases.gradient_case()
    tx, ty, tz, acc = nn_cases.dyadic_operator()
    print(f"[nn-parity] dyadic operator, loss kind {kind} target {with_target}", flush=True)
    mf.set_nn_run(3)
    g = mf.create_grid(*nn_cases.SHAPE)
    mf.set_transmissibility(g, dev(tx), dev(ty), dev(tz), accum=dev(acc))
    net = mf.net_create(p)
    mf.net_set_loss(net, kind)
    rd = dev(r)
    loss = mf.nn_loss_grad(net, g, rd, rd if with_target else None)
    _, grad = mf.net_get_params(net)
    As = nn_cases.dyadic_scaled(tx, ty, tz, acc, dmask)
    ref_loss, ref_g, _ = nn.loss_and_grads(p, r, f, r if with_target else None, dmask, As, kind=kind)
    assert abs(loss - ref_loss) <= 1e-6 * abs(ref_loss)
    bad = np.flatnonzero(grad.astype(np.float64) != ref_g)
    assert bad.size == 0, f"{bad.size} gradient entries differ, first {bad[:8].tolist()}"
    net.close()
    g.close()


@pytest.mark.parametrize("omega,shape", [(0.5, (16, 16, 20)), (0.0, (16, 16, 20)), (0.5, (15, 14, 19))])
def test_flexible_cg_with_a_random_network_matches_the_oracle(mf, omega, shape):
    """Flexible CG with a fixed, non-degenerate random network, with and without
    the Jacobi sweeps around it: the GPU's FP32 iteration count within 5 % (or
    3) of the oracle's FP64 flexible CG with the same preconditioner
    (oracle.nn.learned_preconditioner), no safeguard fallback on either side,
    and the FP64-refined field within 1e-5 of the direct solution. With nz a
    multiple of 4 the operator passes take their four-cells-per-thread form,
    otherwise the one-cell form (both write the network's input in the first
    sweep)."""
    k = channelised(shape, 3600)
    p = nn.init_params(seed=43, last_scale=0.2)
    mf.set_nn_run(3)
    g, _, b = gpu_problem(mf, k, c=1e-3)
    ref = OracleProblem(k, c=1e-3)
    feat = torch.empty(k.size, dtype=torch.float32, device="cuda")
    mf.grid_feature(g, feat)
    f = feat.cpu().numpy().astype(np.float64).reshape(shape)
    net = mf.net_create(p)
    x = torch.zeros(k.size, dtype=torch.float32, device="cuda")
    st, info = mf.cg_solve(g, b, x, mf.default_opts(precond=mf.PRECOND_LEARNED, net=net, nn_smooth=omega))
    assert st == mf.OK and info["fallbacks"] == 0
    M = nn.learned_preconditioner(p, ref.A, ref.dmask, f, omega=omega)
    zr_min = []

    def M_checked(r):
        z = M(r)
        zr_min.append(float(z @ r))
        return z
    orc = krylov.fcg(ref.Auu, ref.bu, M_checked, tol=1e-6, max_iter=2000)
    assert orc.converged and min(zr_min) > 0
    # the network is not the zero network: it changes the iteration count
    M0 = nn.learned_preconditioner(nn.init_params(seed=0, last_scale=0.0), ref.A, ref.dmask, f, omega=omega)
    base = krylov.fcg(ref.Auu, ref.bu, M0, tol=1e-6, max_iter=2000)
    print(f"\n[nn-parity] FCG iterations (w {omega}): GPU {info['iters']}, oracle {orc.iters}, "
          f"oracle zero network {base.iters}", flush=True)
    assert orc.iters != base.iters
    assert abs(info["iters"] - orc.iters) <= max(3, orc.iters // 20)
    x64 = torch.zeros(k.size, dtype=torch.float64, device="cuda")
    st, info = mf.cg_solve_f64(g, b.double(), x64, mf.default_opts(
        tol=1e-9, precision=mf.FP32_IR, precond=mf.PRECOND_LEARNED, net=net, nn_smooth=omega))
    assert st == mf.OK
    pref = ref.direct()
    err = np.linalg.norm(x64.cpu().numpy() - pref) / np.linalg.norm(pref)
    assert err <= 1e-5, err
    net.close()
    g.close()
