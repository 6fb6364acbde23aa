"""Oracle of the learned preconditioner's network: direct 3D convolutions.

Test infrastructure only (see the package docstring).

The network maps two input channels per cell through four 3x3x3 convolutions
with 2 -> 16 -> 16 -> 16 -> 1 channels and a ReLU after each of the first
three. It works on the Jacobi-scaled system A~ = D^-1/2 A D^-1/2 (D = diag A):
the input channels are the scaled residual r~ = D^-1/2 r / s (s, a power of
two, brings its RMS over the unknown cells within a factor sqrt 2 of 1) and r~ times the log-diagonal feature
f = log d - mean_U log d, so the output vanishes with the residual; the
preconditioned residual is z = D^-1/2 (r~ + N) (times s), which is Jacobi
when N = 0. A convolution here is
the cross-correlation with zero padding ("same" size):

    y[K, o] = b[o] + sum_{tap} sum_{c} W[tap, c, o] * x[K + offset(tap), c],

with ``tap = 9*(di+1) + 3*(dj+1) + (dk+1)`` for offsets ``di, dj, dk`` in
{-1, 0, 1} along (x, y, z), and ``x = 0`` outside the grid.

Everything is computed in FP64. Where the GPU path stores a tensor in BF16
(weights, the network input, hidden activations, back-propagated activation
gradients) the oracle rounds the same tensor to BF16 with round-to-nearest-even,
so both sides see the same operands; sums are exact-ish FP64 here and FP32 on
the GPU.

Parameter vector layout (FP32 on the GPU): for each layer, W[27, cin, cout]
(C order) then b[cout].
"""
from __future__ import annotations

import numpy as np

LAYERS = ((2, 16, True), (16, 16, True), (16, 16, True), (16, 1, False))


def n_params() -> int:
    return sum(27 * ci * co + co for ci, co, _ in LAYERS)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def unpack(params):
    """List of (W[27, cin, cout], b[cout]) per layer from the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for ci, co, _ in LAYERS:
        W = p[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        b = p[o:o + co]
        o += co
        out.append((W, b))
    assert o == p.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed: int = 0, last_scale: float = 0.0) -> np.ndarray:
    """He-normal weights, zero biases; the last layer scaled by ``last_scale``
    (0 makes the network output 0, so flexible CG starts as Jacobi-PCG).
    Training keeps the biases at zero, so N(0) = 0."""
    rng = np.random.default_rng(seed)
    layers = []
    for li, (ci, co, _) in enumerate(LAYERS):
        W = rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=(27, ci, co))
        if li == len(LAYERS) - 1:
            W *= last_scale
        layers.append((W, np.zeros(co)))
    return pack(layers).astype(np.float32)


def offsets():
    return [(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)]


def shifted(x, off):
    """s[K] = x[K + off] with zeros outside the grid (x has a trailing channel axis)."""
    nx, ny, nz = x.shape[:3]
    out = np.zeros_like(x)
    src, dst = [], []
    for d, n in zip(off, (nx, ny, nz)):
        if d >= 0:
            src.append(slice(d, n))
            dst.append(slice(0, n - d))
        else:
            src.append(slice(0, n + d))
            dst.append(slice(-d, n))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv3d(x, W, b):
    """y[K, o] = b[o] + sum_tap x[K + off(tap), :] @ W[tap]."""
    y = np.broadcast_to(b, x.shape[:3] + (W.shape[2],)).astype(np.float64).copy()
    for t, off in enumerate(offsets()):
        y += shifted(x, off) @ W[t]
    return y


def conv3d_grads(x, W, dy):
    """Gradients of conv3d with respect to W, b and x, given dL/dy."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    ci, co = x.shape[-1], dy.shape[-1]
    dyf = dy.reshape(-1, co)
    for t, off in enumerate(offsets()):
        xs = shifted(x, off)
        dW[t] = xs.reshape(-1, ci).T @ dyf          # sum over cells of x[K + off] dy[K]
        # y[K] uses x[K + off]: the gradient flows back to x[K'] from dy[K' - off]
        dx += shifted(dy, tuple(-d for d in off)) @ W[t].T
    db = dy.sum(axis=(0, 1, 2))
    return dW, db, dx


def network_input(r_hat, feat):
    """The two input channels (r_hat, r_hat * feat); the product is taken in FP32."""
    r32 = np.asarray(r_hat, dtype=np.float32)
    return np.stack([r32.astype(np.float64),
                     (r32 * np.asarray(feat, dtype=np.float32)).astype(np.float64)], axis=-1)


def forward(params, r_hat, feat, bf16: bool = True, relu: bool = True):
    """Network output N (FP64, shape of the grid) and the cached activations.
    ``relu=False`` makes the hidden activations the identity."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = [(rnd(W), np.asarray(b, dtype=np.float64)) for W, b in unpack(params)]
    h = rnd(network_input(r_hat, feat))
    cache = [h]
    for li, ((W, b), (_, _, hidden)) in enumerate(zip(layers, LAYERS)):
        y = conv3d(h, W, b)
        if hidden:
            h = rnd(np.maximum(y, 0.0) if relu else y)
            cache.append(h)
        else:
            h = y
    return h[..., 0], cache, layers


def prediction_loss(z, r_hat, dmask, apply_scaled, kind=0, target=None):
    """Loss of a preconditioned residual ``z`` and its gradient with respect to z.

    All three are quadratic forms of the Jacobi-scaled operator A~ over the
    unknown cells (``apply_scaled(v)`` returns A~ v for a grid-shaped v that is
    0 on Dirichlet cells; z, r_hat and target are taken as 0 there):

    * ``kind=0`` with a target t (the scaled error, A~ t = r_hat): the energy
      norm of the prediction error relative to that of the error,
      ``(z - t)' A~ (z - t) / (t' r_hat)``; gradient ``2 A~ (z - t) / (t' r_hat)``.
    * ``kind=0`` without a target: the energy functional
      ``(z' A~ z - 2 z' r_hat) / (r_hat' r_hat)``, whose minimiser is the error
      A~^-1 r_hat (the quadratic CG minimises); gradient
      ``2 (A~ z - r_hat) / (r_hat' r_hat)``.
    * ``kind=1``: the residual-space loss ``||A~ z - r_hat||^2 / ||r_hat||^2``;
      gradient ``2 A~ (A~ z - r_hat) / ||r_hat||^2`` (A~ is symmetric).

    Returns (loss, dloss/dz as a grid-shaped array, 0 on Dirichlet cells).
    """
    u = ~np.asarray(dmask, dtype=bool)
    rh = np.where(u, np.asarray(r_hat, dtype=np.float64), 0.0)
    zz = np.where(u, np.asarray(z, dtype=np.float64), 0.0)
    Aop = lambda v: np.where(u, apply_scaled(v), 0.0)
    if kind == 1:
        E = float(np.sum(rh * rh))
        g = Aop(zz) - rh
        return float(np.sum(g * g) / E), 2.0 * Aop(g) / E
    if kind != 0:
        raise ValueError("loss kind must be 0 or 1")
    if target is None:
        E = float(np.sum(rh * rh))
        Az = Aop(zz)
        return float((np.sum(zz * Az) - 2.0 * np.sum(zz * rh)) / E), 2.0 * (Az - rh) / E
    t = np.where(u, np.asarray(target, dtype=np.float64), 0.0)
    E = float(np.sum(t * rh))
    delta = zz - t
    Ad = Aop(delta)
    return float(np.sum(delta * Ad) / E), 2.0 * Ad / E


def backprop(layers, cache, dy, bf16: bool = True, relu: bool = True):
    """Parameter gradient (flat vector) of the network for the output gradient
    ``dy`` (grid-shaped), from the activations ``cache`` and the BF16-rounded
    layers of :func:`forward`. Each back-propagated activation gradient is
    rounded to BF16 (with ``bf16``), as the GPU stores it."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    g = rnd(np.asarray(dy, dtype=np.float64))[..., None]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        dW, db, dx = conv3d_grads(cache[li], W, g)
        grads[li] = (dW, db)
        if li > 0:
            g = rnd(dx * (cache[li] > 0) if relu else dx)   # activation of the layer below
    return pack(grads)


def loss_and_grads(params, r_hat, feat, target, dmask, apply_scaled, bf16: bool = True,
                   relu: bool = True, kind: int = 0):
    """Training loss of one sample and its gradient with respect to the
    parameter vector: z = r_hat + N(r_hat, feat) scored by
    :func:`prediction_loss` (``kind`` 0: the energy norm of the prediction
    error with a target, the energy functional without one; 1: the residual
    space). r_hat is taken as 0 on Dirichlet cells, also as network input.
    Returns (loss, gradient, N).
    """
    u = ~np.asarray(dmask, dtype=bool)
    rh = np.where(u, np.asarray(r_hat, dtype=np.float64), 0.0)
    out, cache, layers = forward(params, rh, feat, bf16, relu)
    loss, dz = prediction_loss(rh + out, rh, dmask, apply_scaled, kind, target)
    return loss, backprop(layers, cache, dz, bf16, relu), out


def scaled_operator(A, dmask):
    """apply_scaled for loss_and_grads: v -> D^-1/2 A D^-1/2 v on the grid."""
    dis = 1.0 / np.sqrt(A.diagonal())
    shape = np.shape(dmask)
    return lambda v: (dis * (A @ (dis * np.asarray(v, dtype=np.float64).ravel()))).reshape(shape)


def adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, frozen=None):
    """One Adam step (Kingma and Ba, bias-corrected); returns new (params, m, v).
    Entries where ``frozen`` is true keep their parameter and moments."""
    m_new = beta1 * m + (1 - beta1) * grads
    v_new = beta2 * v + (1 - beta2) * grads * grads
    mh = m_new / (1 - beta1 ** step)
    vh = v_new / (1 - beta2 ** step)
    p_new = params - lr * mh / (np.sqrt(vh) + eps)
    if frozen is not None:
        keep = np.asarray(frozen, dtype=bool)
        p_new = np.where(keep, params, p_new)
        m_new = np.where(keep, m, m_new)
        v_new = np.where(keep, v, v_new)
    return p_new, m_new, v_new


def bias_mask() -> np.ndarray:
    """True at the bias entries of the parameter vector (held fixed in training)."""
    mask = np.zeros(n_params(), dtype=bool)
    o = 0
    for ci, co, _ in LAYERS:
        o += 27 * ci * co
        mask[o:o + co] = True
        o += co
    return mask


def network_scale(ru, du) -> float:
    """The scale s of the network's input for the residual ru on the unknown
    cells (du: their diagonal): the power of two nearest the D^-1-weighted RMS,
    2^round(log2 rms) with rms^2 = sum(ru^2 / du) / n_U; 0 for a zero residual."""
    rms = np.sqrt(np.sum(ru * ru / du) / ru.size)
    return 0.0 if rms == 0 else float(2.0 ** np.round(np.log2(rms)))


def learned_preconditioner(params, A, dmask, feat, omega: float = 0.5, relu: bool = True,
                           bf16: bool = True):
    """The preconditioner of flexible CG with the network, as a map on the
    unknown cells' residual vector (``A``: the assembled full-grid operator,
    ``feat``: the grid-shaped input feature).

    The network's correction of a residual r is C(r) = s D^-1/2 N(r_hat, f)
    with r_hat = D^-1/2 r / s (0 on Dirichlet cells), s the power of two
    nearest the D^-1-weighted RMS of r: s = 2^round(log2 rms),
    rms^2 = r' D^-1 r / n_U, so the input's RMS lies within a factor sqrt 2
    of one and dividing by s is exact in floating point.
    With omega = 0 the preconditioned residual is z = D^-1 r + C(r): Jacobi
    when N = 0. With omega > 0 the network sits between two damped Jacobi
    sweeps, each taken from the residual it is given:

        z1 = omega D^-1 r,  r1 = r - A z1,  z2 = z1 + D^-1 r1 + C(r1),
        z  = z2 + omega D^-1 (r - A z2),

    which with N = 0 is the polynomial preconditioner
    D^-1/2 [(I - w A~)((1 + w) I - w A~) + w I] D^-1/2 of A~ = D^-1/2 A D^-1/2.
    """
    d = A.diagonal()
    u = np.flatnonzero(~np.asarray(dmask, dtype=bool).ravel())
    n = d.size
    shape = np.shape(dmask)

    def C(ru):
        sc = network_scale(ru, d[u])
        if sc == 0:
            return np.zeros_like(ru)
        rh = np.zeros(n)
        rh[u] = ru / np.sqrt(d[u]) / sc
        N, _, _ = forward(params, rh.reshape(shape), feat, bf16=bf16, relu=relu)
        return sc * N.ravel()[u] / np.sqrt(d[u])

    def Au(vu):
        v = np.zeros(n)
        v[u] = vu
        return (A @ v)[u]

    def M(ru):
        ru = np.asarray(ru, dtype=np.float64)
        if omega == 0:
            return ru / d[u] + C(ru)
        z1 = omega * ru / d[u]
        r1 = ru - Au(z1)
        z2 = z1 + r1 / d[u] + C(r1)
        return z2 + omega * (ru - Au(z2)) / d[u]
    return M
