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


# --- the three training losses: prediction_loss pinned by closed forms --------

def _dense_scaled(shape, seed, c=1e-2):
    """A TPFA operator with x-plane Dirichlet cells, its Jacobi-scaled form on
    the unknown cells as a dense matrix, and apply_scaled for the oracle."""
    from oracle import tpfa
    from synth import lognormal_iid
    k = lognormal_iid(shape, 1.0, seed)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), c, dmask, pd)
    u = ~dmask.ravel()
    dis = 1.0 / np.sqrt(A.diagonal())
    At = (dis[:, None] * A.toarray() * dis[None, :])[np.ix_(u, u)]
    return dmask, u, At, nn.scaled_operator(A, dmask)


def _grid(u, shape, v):
    g = np.zeros(int(np.prod(shape)))
    g[u] = v
    return g.reshape(shape)


def test_losses_at_the_closed_form_minimiser():
    """On a dense 4^3 system the error z* = A~^-1 r_hat minimises the energy
    functional with value -r_hat' A~^-1 r_hat / r_hat' r_hat and zero gradient,
    and zeroes the residual-space loss and its gradient; completing the square
    gives F(z) - F(z*) = (z - z*)' A~ (z - z*) / r_hat' r_hat for any z."""
    shape = (4, 4, 4)
    dmask, u, At, As = _dense_scaled(shape, 7)
    rng = np.random.default_rng(8)
    rt = rng.normal(size=u.sum())
    zs = np.linalg.solve(At, rt)
    rh, zg = _grid(u, shape, rt), _grid(u, shape, zs)
    F, dF = nn.prediction_loss(zg, rh, dmask, As, kind=0)
    assert abs(F - (-(rt @ zs) / (rt @ rt))) <= 1e-13 * abs(F)
    assert np.max(np.abs(dF)) <= 1e-12
    R, dR = nn.prediction_loss(zg, rh, dmask, As, kind=1)
    assert R <= 1e-24 and np.max(np.abs(dR)) <= 1e-12
    for _ in range(3):
        zt = rng.normal(size=u.sum())
        Fz, _ = nn.prediction_loss(_grid(u, shape, zt), rh, dmask, As, kind=0)
        gap = (zt - zs) @ At @ (zt - zs) / (rt @ rt)
        assert abs((Fz - F) - gap) <= 1e-12 * gap and gap > 0
        # residual space: ||A~ z - r||^2 / ||r||^2 = (z - z*)' A~^2 (z - z*) / ||r||^2
        Rz, _ = nn.prediction_loss(_grid(u, shape, zt), rh, dmask, As, kind=1)
        e = At @ (zt - zs)
        assert abs(Rz - e @ e / (rt @ rt)) <= 1e-12 * Rz


def test_losses_with_the_identity_operator():
    """A~ = I: the energy functional is ||z - r||^2/||r||^2 - 1 and the
    residual-space loss ||z - r||^2/||r||^2; a target t = r gives the energy
    norm ||z - r||^2 / ||r||^2."""
    shape = (3, 4, 5)
    nod = np.zeros(shape, dtype=bool)
    ident = lambda v: np.asarray(v, dtype=np.float64)
    rng = np.random.default_rng(9)
    r, z = rng.normal(size=shape), rng.normal(size=shape)
    d2 = np.sum((z - r) ** 2) / np.sum(r * r)
    F, dF = nn.prediction_loss(z, r, nod, ident, kind=0)
    R, dR = nn.prediction_loss(z, r, nod, ident, kind=1)
    T, dT = nn.prediction_loss(z, r, nod, ident, kind=0, target=r)
    assert abs(F - (d2 - 1.0)) <= 1e-14 and abs(R - d2) <= 1e-14 and abs(T - d2) <= 1e-14
    for g in (dF, dR, dT):
        assert np.allclose(g, 2.0 * (z - r) / np.sum(r * r), rtol=1e-14, atol=1e-15)


def test_energy_norm_and_functional_differ_by_a_constant():
    """With the consistent target t = A~^-1 r: (z - t)'A~(z - t) = z'A~z - 2 z'r + t'r,
    so E_t(z) t'r = F(z) r'r + t'r for every z."""
    shape = (4, 3, 4)
    dmask, u, At, As = _dense_scaled(shape, 10)
    rng = np.random.default_rng(11)
    rt = rng.normal(size=u.sum())
    tt = np.linalg.solve(At, rt)
    rh, tg = _grid(u, shape, rt), _grid(u, shape, tt)
    for _ in range(3):
        z = _grid(u, shape, rng.normal(size=u.sum()))
        E, _ = nn.prediction_loss(z, rh, dmask, As, kind=0, target=tg)
        F, _ = nn.prediction_loss(z, rh, dmask, As, kind=0)
        assert abs(E * (tt @ rt) - (F * (rt @ rt) + tt @ rt)) <= 1e-12 * abs(E * (tt @ rt))


def _pass_through(alpha):
    """Identity-activation network with N = alpha * (first input channel): the
    centre tap carries channel 0 through the three hidden layers."""
    layers = [(np.zeros((27, ci, co)), np.zeros(co)) for ci, co, _ in nn.LAYERS]
    for li in range(3):
        layers[li][0][13, 0, 0] = 1.0
    layers[3][0][13, 0, 0] = alpha
    return nn.pack(layers)


@pytest.mark.parametrize("kind", [0, 1])
def test_network_loss_in_closed_form_for_a_pass_through_network(kind):
    """N = alpha r_hat, so z = (1 + alpha) r_hat: the functional is
    ((1+a)^2 r'A~r - 2 (1+a) r'r) / r'r and the residual loss
    ||(1+a) A~r - r||^2 / r'r. The derivative with respect to the last layer's
    centre weight is dL/da, and with respect to the first layer's it is a dL/da
    (N = w4 w3 w2 w1 r_hat), from the dense matrix."""
    shape = (5, 3, 4)
    dmask, u, At, As = _dense_scaled(shape, 12)
    rng = np.random.default_rng(13)
    rt = rng.normal(size=u.sum()).astype(np.float32).astype(np.float64)   # FP32 network input
    rh = _grid(u, shape, rt)
    a = 0.37
    loss, g, out = nn.loss_and_grads(_pass_through(a), rh, rng.normal(size=shape), None, dmask, As,
                                     bf16=False, relu=False, kind=kind)
    assert np.allclose(out, a * rh, rtol=0, atol=1e-15)
    rr, rAr, Ar = rt @ rt, rt @ At @ rt, At @ rt
    if kind == 0:
        want = ((1 + a) ** 2 * rAr - 2 * (1 + a) * rr) / rr
        dlda = (2 * (1 + a) * rAr - 2 * rr) / rr
    else:
        e = (1 + a) * Ar - rt
        want = e @ e / rr
        dlda = 2 * e @ Ar / rr
    assert abs(loss - want) <= 1e-13 * abs(want)
    w4 = nn.n_params() - 1 - 27 * 16          # W4[13, 0, 0]
    w4 += 13 * 16
    w1 = 13 * 2 * 16                          # W1[13, 0, 0]
    assert abs(g[w4] - dlda) <= 1e-12 * abs(dlda)
    assert abs(g[w1] - a * dlda) <= 1e-12 * abs(a * dlda)


@pytest.mark.parametrize("kind,with_target", [(0, False), (1, False), (0, True)])
@pytest.mark.parametrize("relu", [True, False])
def test_every_loss_gradient_matches_central_differences(kind, with_target, relu):
    from oracle import tpfa
    from synth import lognormal_iid
    rng = np.random.default_rng(14)
    shape = (4, 3, 5)
    params = nn.init_params(seed=15, last_scale=0.5).astype(np.float64)
    k = lognormal_iid(shape, 1.0, 16)
    dmask, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dmask, pd)
    As = nn.scaled_operator(A, dmask)
    r = np.where(dmask, 0.0, rng.normal(size=shape))
    f = rng.normal(size=shape)
    tgt = None
    if with_target:
        tgt = np.where(dmask, 0.0, rng.normal(size=shape))
        tgt *= np.sign(np.sum(tgt * r)) or 1.0
    loss, g, _ = nn.loss_and_grads(params, r, f, tgt, dmask, As, bf16=False, relu=relu, kind=kind)
    h = 1e-6
    for i in rng.choice(params.size, 30, replace=False):
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        l1 = nn.loss_and_grads(p1, r, f, tgt, dmask, As, bf16=False, relu=relu, kind=kind)[0]
        l2 = nn.loss_and_grads(p2, r, f, tgt, dmask, As, bf16=False, relu=relu, kind=kind)[0]
        fd = (l1 - l2) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


# --- Adam: closed forms of the bias-corrected moments ------------------------

def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 3e-7])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        p, m, v = nn.adam(p, g, m, v, step=t, lr=0.01)
        assert np.allclose(p, -0.01 * t * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_single_impulse_then_zero_gradients():
    """A gradient g at step 1 and 0 afterwards: m_t = (1-b1) b1^(t-1) g and
    v_t = (1-b2) b2^(t-1) g^2, so step t moves by
    lr (1-b1) b1^(t-1)/(1-b1^t) g / (sqrt((1-b2) b2^(t-1)/(1-b2^t)) |g| + eps)."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    g = np.array([1.5, -0.25])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    want = np.zeros(2)
    for t in range(1, 6):
        p, m, v = nn.adam(p, g if t == 1 else np.zeros(2), m, v, step=t, lr=lr)
        mh = (1 - b1) * b1 ** (t - 1) / (1 - b1 ** t) * g
        vh = (1 - b2) * b2 ** (t - 1) / (1 - b2 ** t) * g * g
        want = want - lr * mh / (np.sqrt(vh) + eps)
        assert np.allclose(p, want, rtol=1e-12, atol=0)


def test_adam_frozen_entries_and_bias_mask():
    mask = nn.bias_mask()
    assert mask.sum() == 16 + 16 + 16 + 1
    layers = nn.unpack(np.arange(nn.n_params(), dtype=np.float64))
    flat_b = np.concatenate([b for _, b in layers])
    assert np.array_equal(np.flatnonzero(mask), flat_b.astype(int))
    p = np.ones(nn.n_params())
    g = np.full(nn.n_params(), 0.5)
    z = np.zeros(nn.n_params())
    p1, m1, v1 = nn.adam(p, g, z, z, step=1, lr=0.1, frozen=mask)
    assert np.all(p1[mask] == 1.0) and np.all(m1[mask] == 0) and np.all(v1[mask] == 0)
    assert np.allclose(p1[~mask], 1.0 - 0.1 * 0.5 / (0.5 + 1e-8), rtol=1e-14)


# --- the preconditioner around the network -----------------------------------

def test_sandwich_preconditioner_without_network_is_the_polynomial():
    """N = 0: the two damped Jacobi sweeps around the Jacobi step give the
    polynomial D^-1/2 p(A~) D^-1/2 with p(l) = (1 - w l)(1 + w - w l) + w,
    checked against the dense matrix polynomial on a 4^3 system; on a
    diagonal operator (A~ = I, p(1) = 1) it is Jacobi exactly."""
    import scipy.sparse as sp
    shape = (4, 4, 4)
    dmask, u, At, _ = _dense_scaled(shape, 21)
    from oracle import tpfa
    from synth import lognormal_iid
    k = lognormal_iid(shape, 1.0, 21)
    dm, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dm, pd)
    zero = nn.init_params(seed=0, last_scale=0.0)
    rng = np.random.default_rng(22)
    d = A.diagonal()[u]
    for w in (0.5, 0.8, 1.0, 1.9):   # the library accepts [0, 2): SPD on the whole range
        M = nn.learned_preconditioner(zero, A, dm, np.zeros(shape), omega=w)
        r = rng.normal(size=u.sum())
        I = np.eye(u.sum())
        P = (I - w * At) @ ((1 + w) * I - w * At) + w * I
        want = (P @ (r / np.sqrt(d))) / np.sqrt(d)
        assert np.allclose(M(r), want, rtol=1e-12, atol=1e-14)
        assert np.min(np.linalg.eigvalsh((P + P.T) / 2)) > 0          # SPD for A~'s spectrum
    # omega = 0 and N = 0: Jacobi
    M0 = nn.learned_preconditioner(zero, A, dm, np.zeros(shape), omega=0.0)
    r = rng.normal(size=u.sum())
    assert np.allclose(M0(r), r / d, rtol=1e-15, atol=0)
    # a diagonal operator: A~ = I, so the sandwich is Jacobi too
    n = int(np.prod(shape))
    Ad = sp.diags(np.full(n, 4.0)).tocsr()
    nod = np.zeros(shape, dtype=bool)
    Md = nn.learned_preconditioner(zero, Ad, nod, np.zeros(shape), omega=0.5)
    r = rng.normal(size=n)
    assert np.allclose(Md(r), r / 4.0, rtol=1e-15, atol=1e-16)


def test_sandwich_correction_is_the_network_through_the_post_sweep():
    """With a pass-through network N = a r_hat the sandwich gives
    z~ = p(A~) r~ + a (I - w A~)(I - w A~) r~ (the network sees the residual
    after the first sweep and its output passes the second), in closed form."""
    shape = (4, 4, 4)
    from oracle import tpfa
    from synth import lognormal_iid
    k = lognormal_iid(shape, 1.0, 23)
    dm, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dm, pd)
    u = np.flatnonzero(~dm.ravel())
    dis = 1.0 / np.sqrt(A.diagonal())
    At = (dis[:, None] * A.toarray() * dis[None, :])[np.ix_(u, u)]
    a, w = 0.3, 0.5
    M = nn.learned_preconditioner(_pass_through(a), A, dm, np.zeros(shape), omega=w, relu=False,
                                  bf16=False)
    r = np.random.default_rng(24).normal(size=u.size)
    rt = r * dis[u]
    I = np.eye(u.size)
    S = I - w * At
    poly = S @ ((1 + w) * I - w * At) + w * I
    # the network input is rounded to FP32: compare at FP32 resolution
    assert np.allclose(M(r) / dis[u], poly @ rt + a * S @ S @ rt, rtol=1e-6, atol=1e-7)
    # and the correction really passes through the second sweep (not (I - w A~) once)
    assert not np.allclose(M(r) / dis[u], poly @ rt + a * S @ rt, rtol=1e-3, atol=1e-4)


def test_network_scale_is_a_power_of_two_so_power_of_two_residual_scalings_commute():
    """The network's input scale s is the power of two nearest the
    D^-1-weighted RMS of the residual it is given: scaling r by 2^k scales s by
    2^k and leaves the network input r_hat unchanged, so C(2^k r) = 2^k C(r)
    exactly for any network (nonzero biases, BF16 input rounding and all),
    with and without the sweeps. A scaling that moves the RMS across
    2^(j + 1/2) changes s by a factor 2 instead of the RMS's factor; with
    nonzero biases the result then is not proportional."""
    from oracle import tpfa
    from synth import lognormal_iid
    shape = (6, 5, 7)
    k = lognormal_iid(shape, 1.0, 31)
    dm, pd = tpfa.x_plane_dirichlet(shape)
    A, _ = tpfa.assemble(*tpfa.transmissibility(k), 1e-2, dm, pd)
    u = ~dm.ravel()
    d = A.diagonal()[u]
    rng = np.random.default_rng(32)
    params = nn.init_params(seed=33, last_scale=0.5)
    params[nn.bias_mask()] = rng.normal(0.0, 0.3, int(nn.bias_mask().sum()))   # nonzero biases
    feat = rng.normal(size=shape)
    r = rng.normal(size=int(u.sum()))
    for w in (0.0, 0.5):
        M = nn.learned_preconditioner(params, A, dm, feat, omega=w)
        base = M(r)
        for kk in (-20, -3, 1, 7):
            assert np.array_equal(M(r * 2.0 ** kk), base * 2.0 ** kk)
    # s itself: a power of two within a factor sqrt 2 of the RMS (the nearest),
    # switching from 1 to 2 where the RMS crosses sqrt 2
    rms = np.sqrt(np.sum(r * r / d) / r.size)
    for target in (1e-9, 0.3, 0.7, 0.9999, 1.0, 1.3, 1.41, 1.42, 5.0, 3e7):
        sc = nn.network_scale(r * (target / rms), d)
        e = np.log2(sc)
        assert e == np.round(e) and abs(np.log2(target / sc)) <= 0.5 + 1e-12
    assert nn.network_scale(r * (0.999 * np.sqrt(2.0) / rms), d) == 1.0
    assert nn.network_scale(r * (1.001 * np.sqrt(2.0) / rms), d) == 2.0
    assert nn.network_scale(np.zeros_like(r), d) == 0.0
