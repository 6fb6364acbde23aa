"""The measurement probes: the streaming probe writes the sum of its inputs to
every output (exact on small integers), and the copy probe copies."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available()
    mffv.lib()
    return mffv


def test_stream_probe_sums(mf):
    n = 4 * 100_003
    rng = np.random.default_rng(1)
    host = [rng.integers(-1000, 1000, n).astype(np.float32) for _ in range(7)]
    ins = [torch.from_numpy(h).cuda() for h in host]
    outs = [torch.full((n,), 5.0, device="cuda") for _ in range(3)]
    for ni, no in ((1, 1), (4, 1), (5, 2), (7, 3)):
        mf.stream_probe(ins[:ni], outs[:no])
        want = np.sum(host[:ni], axis=0)
        for o in outs[:no]:
            assert np.array_equal(o.cpu().numpy(), want), (ni, no)
    with pytest.raises(mf.MffvError):
        mf.stream_probe(ins[:2], [ins[1]])                       # an output aliases an input
    with pytest.raises(mf.MffvError):
        mf.stream_probe([torch.zeros(6, device="cuda")], [torch.zeros(6, device="cuda")])   # n % 4
    torch.cuda.synchronize()


def test_copy_probe_copies(mf):
    src = torch.arange(4096, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    mf.copy_probe(dst, src, 4096 * 4)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
