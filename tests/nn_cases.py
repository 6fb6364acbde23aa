"""Network test cases for the GPU parity tests of the learned preconditioner.

Integer-valued cases. With integer weights and biases, an integer-valued
input and the identity operator (A~ = I: no faces, accumulation 1), every
quantity of the network's forward and backward pass is an integer multiple
of a power of two, and every sum has a bound on the absolute values of its
terms below 2^24 of that unit. Each partial sum, in any order, is then
exactly representable in FP32, BF16 rounding acts on the same exact value on
both sides, and the GPU result must equal the FP64 oracle's bit for bit.
``exactness_margin`` checks those conditions on the oracle for a given case,
so a GPU test that expects equality states why it may. The same holds on a
TPFA operator whose Jacobi scaling is exact (``dyadic_operator``).
"""
from __future__ import annotations

import numpy as np

from oracle import nn

UNIT_LIMIT = 2.0 ** 24


def integer_params(seed: int, density: float, bias: bool = False) -> np.ndarray:
    """Weights in {-1, 0, 1} (nonzero with probability ``density``), biases 0
    or in {-1, 0, 1}; float32 parameter vector in the library's layout."""
    rng = np.random.default_rng(seed)
    layers = []
    for ci, co, _ in nn.LAYERS:
        W = rng.choice([-1.0, 1.0], size=(27, ci, co)) * (rng.random((27, ci, co)) < density)
        b = rng.integers(-1, 2, size=co).astype(np.float64) if bias else np.zeros(co)
        layers.append((W, b))
    return nn.pack(layers).astype(np.float32)


def spikes(dmask, positions, signs=None) -> np.ndarray:
    """A residual that is +-1 at the given unknown cells and 0 elsewhere."""
    r = np.zeros(np.shape(dmask))
    for t, pos in enumerate(positions):
        assert not dmask[pos], pos
        r[pos] = 1.0 if signs is None else signs[t]
    return r


def _unit(a) -> float:
    """Largest power of two dividing every entry of a (inf for all zeros)."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    a = a[a > 0]
    if a.size == 0:
        return np.inf
    m, e = np.frexp(a)
    # a = m 2^e with m in [0.5, 1): count the trailing zero bits of the 53-bit mantissa
    mant = np.ldexp(m, 53).astype(np.int64)
    tz = np.zeros(mant.shape, dtype=np.int64)
    x = mant.copy()
    while True:
        even = (x & 1) == 0
        if not even.any():
            break
        tz += even
        x = np.where(even, x >> 1, x)
    return float(np.min(np.ldexp(1.0, (e - 53 + tz))))


def exactness_margin(params, r_hat, feat, dy_out=None, relu: bool = True) -> float:
    """Largest (sum of absolute terms) / (unit of the terms) over every sum of
    the forward pass and, with dy_out, of the backward pass; the case is exact
    in FP32 when this is below 2^24 and every operand is a multiple of its
    unit. Returns inf if an operand is not such a multiple (not exact)."""
    out, cache, layers = nn.forward(params, r_hat, feat, bf16=True, relu=relu)
    worst = 0.0
    h, ha = cache[0], np.abs(cache[0])
    for li, ((W, b), (_, _, hidden)) in enumerate(zip(layers, nn.LAYERS)):
        unit = _unit(h) * _unit(W)
        if np.any(b):
            unit = min(unit, _unit(b))
        bound = nn.conv3d(ha, np.abs(W), np.abs(b))
        worst = max(worst, float(bound.max()) / unit)
        if hidden:
            h = cache[li + 1]
            ha = np.abs(h)
    if dy_out is not None:
        g = nn.bf16_round(dy_out)[..., None]
        ga = np.abs(g)
        for li in range(len(layers) - 1, -1, -1):
            W, _ = layers[li]
            x = cache[li]
            dWa, dba, dxa = nn.conv3d_grads(np.abs(x), np.abs(W), ga)
            worst = max(worst, float(dWa.max()) / (_unit(x) * _unit(g)), float(dba.max()) / _unit(g))
            if li > 0:
                _, _, dx = nn.conv3d_grads(x, W, g)
                worst = max(worst, float(dxa.max()) / (_unit(g) * _unit(W)))
                g = nn.bf16_round(dx * (cache[li] > 0) if relu else dx)
                ga = np.abs(g)
    return worst


# The cases the GPU tests use (37 x 18 x 70: ragged in x for runs of 3 and 5,
# ragged 4-row y tiles, a full and a ragged 64-cell z tile).
SHAPE = (37, 18, 70)
RUNS = (1, 2, 3, 5, 37)       # planes per block of the marching convolutions


def forward_case():
    """Dense integer input (r_hat in [-2, 2], feature in [-1, 1]) through a
    network with weights in {-1, 0, 1} (density 0.15) and integer biases."""
    rng = np.random.default_rng(20)
    r = rng.integers(-2, 3, size=SHAPE).astype(np.float64)
    f = rng.integers(-1, 2, size=SHAPE).astype(np.float64)
    return integer_params(21, 0.15, bias=True), r, f


def gradient_case():
    """Four +-1 spikes (so r_hat' r_hat = 4) near plane-run, y-tile and z-tile
    boundaries and the domain edges, through a network with weights in
    {-1, 0, 1} (density 0.12) and zero biases, on the identity operator."""
    from oracle import tpfa
    dmask, _ = tpfa.x_plane_dirichlet(SHAPE)
    r = spikes(dmask, [(5, 3, 63), (6, 17, 64), (1, 0, 69), (20, 9, 10)], [1, -1, 1, 1])
    return integer_params(23, 0.12), r, np.zeros(SHAPE), dmask


def identity_operator(v):
    return np.asarray(v, dtype=np.float64)


def dyadic_operator(seed: int = 30):
    """A TPFA operator whose Jacobi scaling is exact: faces T in {1, 2}
    (seeded), accumulation 16 minus the sum of each cell's faces, so that
    diag(A) = 16 on every cell and A~ = A / 16 has entries that are multiples
    of 1/16. With integer z, A~ z and everything the losses form from it are
    dyadic and exact in FP32 cell by cell. Returns (tx, ty, tz, accum) as FP64
    arrays in the library's face layout (0 beyond the domain)."""
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(seed)
    tx = rng.integers(1, 3, size=SHAPE).astype(np.float64)
    ty = rng.integers(1, 3, size=SHAPE).astype(np.float64)
    tz = rng.integers(1, 3, size=SHAPE).astype(np.float64)
    tx[nx - 1] = 0.0
    ty[:, ny - 1] = 0.0
    tz[:, :, nz - 1] = 0.0
    faces = tx + ty + tz
    faces[1:] += tx[:-1]
    faces[:, 1:] += ty[:, :-1]
    faces[:, :, 1:] += tz[:, :, :-1]
    return tx, ty, tz, 16.0 - faces


def dyadic_scaled(tx, ty, tz, accum, dmask):
    """apply_scaled of the oracle for the dyadic operator."""
    from oracle import tpfa
    A, _ = tpfa.assemble(tx, ty, tz, accum, dmask, np.zeros(SHAPE))
    assert np.all(A.diagonal()[~dmask.ravel()] == 16.0)
    return nn.scaled_operator(A, dmask)
