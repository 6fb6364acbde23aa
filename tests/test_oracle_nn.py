"""Pins of the network oracle: BF16 rounding against torch's conversion, the
convolution against SciPy's correlate and the identity kernel, gradients
against central finite differences, and Adam's first step in closed form."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn


def test_bf16_rounding_ties_to_even_and_matches_torch():
    one = 1.0
    assert nn.bf16_round(one) == 1.0
    assert nn.bf16_round(1 + 2 ** -8) == 1.0                 # tie -> even mantissa
    assert nn.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6     # tie -> even mantissa (up)
    assert nn.bf16_round(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(size=10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(-6, 6, 10000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16_round(x), ref)


def test_conv_identity_kernel_and_scipy_correlate():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 6, 7, 3))
    W = np.zeros((27, 3, 3))
    W[13] = np.eye(3)                           # centre tap (0, 0, 0)
    assert np.allclose(nn.conv3d(x, W, np.zeros(3)), x, atol=0, rtol=0)
    # one channel: cross-correlation with zero padding = scipy.ndimage.correlate
    w = rng.normal(size=(3, 3, 3))
    W1 = w.reshape(27, 1, 1)
    y = nn.conv3d(x[..., :1], W1, np.array([0.5]))[..., 0]
    ref = ndimage.correlate(x[..., 0], w, mode="constant", cval=0.0) + 0.5
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)
    assert [nn.offsets()[t] for t in (0, 13, 26)] == [(-1, -1, -1), (0, 0, 0), (1, 1, 1)]


@pytest.mark.parametrize("relu", [True, False])
def test_gradients_match_central_differences(relu):
    from oracle import tpfa
    from synth import lognormal_iid
    rng = np.random.default_rng(3)
    shape = (4, 3, 5)
    params = nn.init_params(seed=4, last_scale=0.5).astype(np.float64)
    params[-1] = 0.1
    k = lognormal_iid(shape, 1.0, 5)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dmask, pd)
    As = nn.scaled_operator(A, dmask)
    r = np.where(dmask, 0.0, rng.normal(size=shape))
    f = rng.normal(size=shape)
    tgt = np.where(dmask, 0.0, rng.normal(size=shape))
    tgt *= np.sign(np.sum(tgt * r)) or 1.0
    loss, g, _ = nn.loss_and_grads(params, r, f, tgt, dmask, As, bf16=False, relu=relu)
    idx = rng.choice(params.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        l1 = nn.loss_and_grads(p1, r, f, tgt, dmask, As, bf16=False, relu=relu)[0]
        l2 = nn.loss_and_grads(p2, r, f, tgt, dmask, As, bf16=False, relu=relu)[0]
        fd = (l1 - l2) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_energy_loss_special_cases():
    import scipy.sparse as sp
    from oracle import tpfa
    from synth import lognormal_iid
    # a diagonal operator: A~ = I, the scaled error equals the scaled residual,
    # so the zero network (Jacobi) is exact and the loss is 0
    shape = (3, 2, 2)
    A = sp.diags(np.full(12, 3.0)).tocsr()
    nod = np.zeros(shape, dtype=bool)
    r = np.random.default_rng(0).normal(size=shape)
    p0 = nn.init_params(seed=0, last_scale=0.0)
    loss, _, out = nn.loss_and_grads(p0, r, np.zeros(shape), r, nod, nn.scaled_operator(A, nod),
                                     bf16=False)
    assert loss == 0.0 and np.all(out == 0)
    # a TPFA operator: the zero network's loss is the energy of the Jacobi
    # error relative to the error's energy, from a dense solve
    shape = (4, 3, 3)
    k = lognormal_iid(shape, 1.0, 2)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dmask, pd)
    u = ~dmask.ravel()
    dis = 1.0 / np.sqrt(A.diagonal())
    At = (dis[:, None] * A.toarray() * dis[None, :])[np.ix_(u, u)]
    rt = np.random.default_rng(1).normal(size=u.sum())
    et = np.linalg.solve(At, rt)
    want = (rt - et) @ At @ (rt - et) / (et @ rt)
    rg = np.zeros(shape)
    rg.ravel()[u] = rt
    eg = np.zeros(shape)
    eg.ravel()[u] = et
    got, _, _ = nn.loss_and_grads(p0, rg, np.zeros(shape), eg, dmask,
                                  nn.scaled_operator(A, dmask), bf16=False)
    assert abs(got - want) <= 1e-12 * want


def test_input_gradient_of_a_single_convolution():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(3, 4, 3, 2))
    W = rng.normal(size=(27, 2, 3))
    dy = rng.normal(size=(3, 4, 3, 3))
    _, _, dx = nn.conv3d_grads(x, W, dy)
    h = 1e-6
    for _ in range(20):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (np.sum(nn.conv3d(xp, W, np.zeros(3)) * dy) - np.sum(nn.conv3d(xm, W, np.zeros(3)) * dy)) / (2 * h)
        assert abs(fd - dx[i]) < 1e-7 * max(1.0, abs(fd))


def test_zero_last_layer_gives_zero_output_and_adam_first_step():
    p = nn.init_params(seed=1, last_scale=0.0)
    out, _, _ = nn.forward(p, np.ones((3, 3, 3)), np.zeros((3, 3, 3)))
    assert np.all(out == 0)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    newp, m, v = nn.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), step=1, lr=0.01, eps=1e-8)
    # first step: m_hat = g, v_hat = g^2 -> update -lr * g / (|g| + eps)
    assert np.allclose(newp, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert nn.n_params() == 27 * 2 * 16 + 16 + 2 * (27 * 16 * 16 + 16) + 27 * 16 + 1
