"""GPU parity of the k closest pairs (include/clmap_kclosest.h, paper Code 8)
against ``oracle.kclosest``: indices and canonical squared distances must be
identical (bit for bit), in both precisions of the cell list, for cross and
single sets, with threshold refinement, large k (sorted outside LDS), fewer
pairs than k, and many exactly equal distances."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2202_06427_amd as clm
    return clm


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _check(got, ref):
    i, j, d2 = (t.cpu().numpy() for t in got)
    ri, rj, rd2 = ref
    assert len(i) == len(ri)
    assert np.array_equal(i.astype(np.int64), ri) and np.array_equal(j.astype(np.int64), rj)
    assert np.array_equal(d2, rd2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_code8_case(clm, precision):
    """Code 8: 100 and 1000 uniform points in a unit box, cutoff 0.1, k = 5."""
    x, y = W.rng(81).random((100, 3)), W.rng(82).random((1000, 3))
    H = np.eye(3)
    cl = clm.CellList(T(x), clm.Box(H, 0.1, 1), y=T(y), precision=precision)
    _check(cl.kclosest(5), oracle.kclosest(x, H, 0.1, 5, y=y))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("k", [1, 5, 100, 5000])
def test_cross_blob_with_refinement(clm, precision, k):
    """A Gaussian blob against a uniform solvent (the cross-set shape of the
    paper's section 4.1); beyond 8192 pairs the threshold is refined, and
    k = 5000 sorts in HBM."""
    H = np.diag([120.0] * 3)
    g = W.rng(83)
    x = np.mod(g.normal(60.0, 8.0, size=(1500, 3)), 120.0)
    y = W.uniform_in_box(150_000, H, 84)
    cl = clm.CellList(T(x), clm.Box(H, 5.0, 2), y=T(y), precision=precision)
    _check(cl.kclosest(k), oracle.kclosest(x, H, 5.0, k, y=y))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_set_triclinic_small_capacity(clm, precision):
    H = W.triclinic_h((32.0, 30.0, 31.0), (80.0, 95.0, 100.0))
    x = W.uniform_in_box(6000, H, 85)
    cl = clm.CellList(T(x), clm.Box(H, 4.0, 2), precision=precision)
    _check(cl.kclosest(50, capacity=64), oracle.kclosest(x, H, 4.0, 50))
    # 2D
    H2 = np.array([[55.0, -12.0], [0.0, 50.0]])
    x2 = W.uniform_in_box(4000, H2, 86)
    cl2 = clm.CellList(T(x2), clm.Box(H2, 3.2, 2), precision=precision)
    _check(cl2.kclosest(20, capacity=40), oracle.kclosest(x2, H2, 3.2, 20))


def test_fewer_pairs_than_k(clm):
    H = np.diag([50.0] * 3)
    x = W.uniform_in_box(300, H, 87)
    cl = clm.CellList(T(x), clm.Box(H, 2.0, 1), precision="fp32")
    ref = oracle.kclosest(x, H, 2.0, 10_000)
    assert 0 < len(ref[0]) < 10_000
    _check(cl.kclosest(10_000), ref)


def test_exactly_equal_distances(clm):
    """A simple-cubic lattice: every nearest-neighbour distance is exactly 0.5,
    so no histogram edge separates them; the capacity grows to all of them and
    the order goes by index."""
    m = 8
    grid = np.stack(np.meshgrid(*([np.arange(m)] * 3), indexing="ij"), -1).reshape(-1, 3)
    x = 0.25 + 0.5 * grid.astype(np.float64)
    H = np.diag([4.0] * 3)
    cl = clm.CellList(T(x), clm.Box(H, 0.6, 1), precision="fp64")
    with pytest.raises(clm.ClmError):
        cl.kclosest(3, capacity=16)
    _check(cl.kclosest(3), oracle.kclosest(x, H, 0.6, 3))
