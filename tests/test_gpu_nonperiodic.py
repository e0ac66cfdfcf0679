"""GPU parity of the non-periodic neighbour list (paper section 4.1) against
``oracle.neighbor_list_nonperiodic``: the library's extrema, bounding box and
cross/single-set lists give the same pairs bit for bit (FP64 distances
identical; FP32+guard distances within 2e-6 of the cutoff)."""
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


def _compare(pairs, dist, ref, precision, rc):
    p = pairs.cpu().numpy().astype(np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    p = p[order]
    assert len(p) == ref["count"]
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    d = dist.cpu().numpy()[order]
    if precision == "fp64":
        assert np.array_equal(d, ref["nl_d"])
    else:
        assert np.abs(d - ref["nl_d"]).max() <= 2e-6 * rc


def test_extrema_are_exact(clm):
    x = W.rng(92).normal(size=(300_001, 3)) * [3.0, 50.0, 0.01] + [-7.0, 1e4, 0.0]
    lo, hi = clm.extrema(T(x))
    assert np.array_equal(lo, x.min(0)) and np.array_equal(hi, x.max(0))
    lo2, hi2 = clm.extrema(T(x[:1, :2]))
    assert np.array_equal(lo2, x[0, :2]) and np.array_equal(hi2, x[0, :2])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_small", [10, 1000, 20000])
def test_e1_cross_sets(clm, precision, n_small):
    """Section 4.1's shape at a reduced large set (2*10^5 instead of 10^6)."""
    w = W.e1_sets(n_small, n_large=200_000, seed=93)
    ref = oracle.neighbor_list_nonperiodic(w["x"], w["cutoff"], y=w["y"])
    pairs, dist = clm.neighbor_list_nonperiodic(T(w["x"]), w["cutoff"], y=T(w["y"]), precision=precision)
    _compare(pairs, dist, ref, precision, w["cutoff"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,offset", [(3, -250.0), (3, 3.0e4), (2, 17.0)])
def test_single_set_far_from_the_origin(clm, precision, dim, offset):
    g = W.rng(94)
    x = offset + 6.0 * g.random((9000, dim))
    rc = 0.9 if dim == 3 else 0.3
    ref = oracle.neighbor_list_nonperiodic(x, rc)
    pairs, dist = clm.neighbor_list_nonperiodic(T(x), rc, precision=precision)
    _compare(pairs, dist, ref, precision, rc)
