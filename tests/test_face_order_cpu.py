"""The host-side reverse Cuthill-McKee numbering of face-list meshes (no GPU):
a permutation; a randomly numbered chain gets back a bandwidth-1 numbering; a
randomly numbered Cartesian grid gets its bandwidth back to about one plane,
as SciPy's reverse Cuthill-McKee does; components are numbered contiguously."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from synth import cartesian_faces


@pytest.fixture(scope="module")
def mf():
    from paper_2408_03452_amd import mffv
    mffv.lib()
    return mffv


def bandwidth(new, fk, fl):
    return int(np.max(np.abs(new[fk].astype(np.int64) - new[fl])))


def test_chain_gets_bandwidth_one(mf):
    n = 500
    perm = np.random.default_rng(1).permutation(n)
    fk, fl = perm[:-1], perm[1:]                      # a path through the cells in random order
    new = mf.face_order(n, fk, fl)
    assert np.array_equal(np.sort(new), np.arange(n))
    assert bandwidth(new, fk, fl) == 1


def test_cartesian_grid_bandwidth_restored(mf):
    shape = (12, 10, 9)
    n = int(np.prod(shape))
    fk, fl, _ = cartesian_faces(shape)
    perm = np.random.default_rng(2).permutation(n)
    rk, rl = perm[fk], perm[fl]
    new = mf.face_order(n, rk, rl)
    assert np.array_equal(np.sort(new), np.arange(n))
    assert bandwidth(np.arange(n), rk, rl) > n // 2           # the random numbering
    A = sp.coo_matrix((np.ones(rk.size), (rk, rl)), shape=(n, n)).tocsr()
    ref = reverse_cuthill_mckee(A + A.T, symmetric_mode=True)
    ref_new = np.empty(n, dtype=np.int64)
    ref_new[ref] = np.arange(n)
    assert bandwidth(new, rk, rl) <= 2 * bandwidth(ref_new, rk, rl)
    assert bandwidth(new, rk, rl) <= 3 * 10 * 9              # a few planes


def test_components_are_contiguous(mf):
    # two disjoint chains and an isolated cell
    fk = np.array([0, 1, 2, 4, 5])
    fl = np.array([1, 2, 3, 5, 6])
    new = mf.face_order(8, fk, fl)
    assert np.array_equal(np.sort(new), np.arange(8))
    for comp in ([0, 1, 2, 3], [4, 5, 6]):
        ids = np.sort(new[comp])
        assert ids[-1] - ids[0] == len(comp) - 1


def test_face_order_errors(mf):
    with pytest.raises(mf.MffvError):
        mf.face_order(3, [0, 1], [1, 1])
    with pytest.raises(mf.MffvError):
        mf.face_order(3, [0], [3])
    with pytest.raises(mf.MffvError):
        mf.face_order(0, [], [])
