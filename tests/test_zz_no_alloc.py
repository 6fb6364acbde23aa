"""The no-allocation entry point mffv_true_residual_noalloc, called through the
raw C ABI, against mffv_true_residual on two calls in a row, the second on a
smaller grid: the residual vector and the relative norm agree bit for bit
(same kernels and launch shapes, partial sums in the static scratch array
instead of grid memory), and the required output is enforced."""
import ctypes

import numpy as np
import pytest

from gpu_problem import gpu_problem
from synth import lognormal_iid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_residual_matches_the_allocating_entry_point():
    from paper_2408_03452_amd import mffv
    assert torch.cuda.is_available()
    lib = mffv.lib()
    for shape, seed in (((40, 33, 52), 71), ((9, 7, 13), 72)):   # second call: smaller input
        print(f"[no-alloc] shape {shape}", flush=True)
        k = lognormal_iid(shape, 1.5, seed)
        g, _, b = gpu_problem(mffv, k, c=1e-3)
        n = k.size
        x = torch.from_numpy(np.random.default_rng(seed).uniform(0, 1, n)).cuda()
        r_ref = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        r_new = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        rel_ref = ctypes.c_double()
        rel_new = ctypes.c_double()
        assert lib.mffv_true_residual(g.handle, b.data_ptr(), x.data_ptr(), r_ref.data_ptr(),
                                      ctypes.byref(rel_ref)) == mffv.OK
        assert lib.mffv_true_residual_noalloc(g.handle, b.data_ptr(), x.data_ptr(), r_new.data_ptr(),
                                              ctypes.byref(rel_new)) == mffv.OK
        torch.cuda.synchronize()
        assert rel_new.value == rel_ref.value and rel_ref.value > 0
        assert torch.equal(r_new, r_ref)
        # the output vector is required
        assert lib.mffv_true_residual_noalloc(g.handle, b.data_ptr(), x.data_ptr(), None,
                                              ctypes.byref(rel_new)) == mffv.EINVAL
        g.close()
