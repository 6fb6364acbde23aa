"""The integer-valued network cases of the GPU parity tests are exact in FP32:
every sum of their forward and backward passes has integer-multiple operands
whose absolute sum stays below 2^24 units, so the GPU must reproduce the
oracle bit for bit (tests/nn_cases.py)."""
import numpy as np
import pytest

import nn_cases
from oracle import nn


def test_unit_of_values():
    assert nn_cases._unit(np.array([3.0, 0.75, 12.0])) == 0.25
    assert nn_cases._unit(np.array([-8.0, 24.0])) == 8.0
    assert nn_cases._unit(np.zeros(3)) == np.inf


def test_forward_case_is_exact_in_fp32():
    p, r, f = nn_cases.forward_case()
    m = nn_cases.exactness_margin(p, r, f)
    assert m < nn_cases.UNIT_LIMIT / 64, m
    out, cache, _ = nn.forward(p, r, f)
    assert np.all(out == np.round(out)) and np.abs(out).max() > 100   # integers, not trivial
    # a few hidden activations are large enough that BF16 rounds them
    assert any(np.any(np.abs(h) > 256) for h in cache[1:])


@pytest.mark.parametrize("kind,with_target", [(0, False), (1, False), (0, True)])
def test_gradient_case_is_exact_in_fp32(kind, with_target):
    p, r, f, dmask = nn_cases.gradient_case()
    tgt = r if with_target else None
    loss, g, out = nn.loss_and_grads(p, r, f, tgt, dmask, nn_cases.identity_operator, kind=kind)
    _, dz = nn.prediction_loss(r + out, r, dmask, nn_cases.identity_operator, kind, tgt)
    m = nn_cases.exactness_margin(p, r, f, dz)
    assert m < nn_cases.UNIT_LIMIT / 64, m
    # most weights see a nonzero gradient, so most taps are exercised
    assert np.count_nonzero(g) > 0.5 * nn.n_params()
    assert loss == float(np.float32(loss))


@pytest.mark.parametrize("kind,with_target", [(0, False), (1, False), (0, True)])
def test_dyadic_operator_case_is_exact_in_fp32(kind, with_target):
    """The spikes through the integer network on the dyadic TPFA operator: the
    output gradient of every loss kind is dyadic (A~ = A / 16), and every
    backward sum stays exact."""
    p, r, f, dmask = nn_cases.gradient_case()
    tx, ty, tz, acc = nn_cases.dyadic_operator()
    assert acc.min() >= 4.0 and np.all(acc == np.round(acc))
    As = nn_cases.dyadic_scaled(tx, ty, tz, acc, dmask)
    tgt = r if with_target else None
    loss, g, out = nn.loss_and_grads(p, r, f, tgt, dmask, As, kind=kind)
    _, dz = nn.prediction_loss(r + out, r, dmask, As, kind, tgt)
    assert nn_cases._unit(dz) >= 2.0 ** -9
    m = nn_cases.exactness_margin(p, r, f, dz)
    assert m < nn_cases.UNIT_LIMIT, m
    assert np.count_nonzero(g) > 0.5 * nn.n_params()
