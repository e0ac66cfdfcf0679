"""Repeated maps over the same cell list give bitwise-identical results: the
per-tile (or per tile and row group) partials are reduced in a fixed order,
forces are written by the wave that holds the particle, and neighbour lists
are written at offsets from a counting pass (same pairs in the same order).  Checked where
the rows of a tile are spread over several waves (few tiles: small sets,
cross sets) and where they are not (10^5 particles), in both precisions.
Per-bin FP64 sums of the speed histograms are merged with device atomics and
are not covered (their counts are).  A rebuild from the same positions gives
the same cell list, so maps over two builds match too."""
import numpy as np
import pytest
import torch

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


def _maps(cl, v):
    out = {}
    s, c = cl.sum_inv_d()
    out["sum_inv_d"], out["count"] = s.item(), int(c.item())
    out["sum_d"] = cl.sum_d()[0].item()
    e, _ = cl.lj_energy(3.4, 0.238)
    out["lj_e"] = e.item()
    r = cl.lj_forces(3.4, 0.238)
    out["lj_ef_e"] = r["energy"].item()
    out["forces"] = r["forces"].cpu().numpy().copy()
    out["grad_box"] = r["grad_box"].cpu().numpy().copy()
    h, _ = cl.histogram(10)
    out["hist10"] = h.cpu().numpy().copy()
    h, _ = cl.histogram(128)
    out["hist128"] = h.cpu().numpy().copy()
    hd = cl.dist_vel_histogram(v, 10)
    out["dv_counts"] = hd[0].cpu().numpy().copy()
    pairs, dist = cl.neighbor_list()  # two-pass list: the order is fixed too
    out["nl_pairs"] = pairs.cpu().numpy().copy()
    out["nl_dist"] = dist.cpu().numpy().copy()
    return out


def _same(a, b):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert a[k].tobytes() == b[k].tobytes(), k
        else:
            assert a[k] == b[k], k


@pytest.mark.parametrize("n", [3000, 100_000])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_repeated_maps_are_bitwise_identical(clm, n, precision):
    side = (n / 0.1) ** (1.0 / 3.0)
    H = W.triclinic_h((side, 0.97 * side, 1.03 * side), (85.0, 95.0, 100.0))
    x = W.uniform_in_box(n, H, 700 + n)
    v = T(W.rng(701).normal(size=(n, 3)))
    cl = clm.CellList(T(x), clm.Box(H, 8.0, 2), precision=precision)
    a = _maps(cl, v)
    b = _maps(cl, v)
    _same(a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_rebuilt_cell_list_gives_bitwise_identical_maps(clm, precision):
    """A rebuild from the same positions places every particle at the same
    sorted index (within a cell the order is by x, then by index, not by
    the order of the placing threads), so maps over two builds match bit
    for bit: the half-shell force sweep, the tile sweeps and the
    neighbour-list order."""
    n = 100_000
    side = (n / 0.1) ** (1.0 / 3.0)
    H = W.triclinic_h((side, 0.97 * side, 1.03 * side), (85.0, 95.0, 100.0))
    x = W.uniform_in_box(n, H, 704)
    v = T(W.rng(705).normal(size=(n, 3)))
    box = clm.Box(H, 8.0, 2)
    cl = clm.CellList(T(x), box, precision=precision)
    a = _maps(cl, v)
    cl.build(T(x))
    b = _maps(cl, v)
    _same(a, b)
    c = _maps(clm.CellList(T(x), box, precision=precision), v)
    _same(a, c)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_repeated_cross_maps_are_bitwise_identical(clm, precision):
    H = np.diag([120.0] * 3)
    x = np.mod(W.rng(702).normal(60.0, 6.0, size=(800, 3)), 120.0)
    y = W.uniform_in_box(150_000, H, 703)
    cl = clm.CellList(T(x), clm.Box(H, 5.0, 2), y=T(y), precision=precision)

    def run():
        s, c = cl.sum_inv_d()
        h, _ = cl.histogram(50)
        e, _ = cl.lj_energy(3.4, 0.238)
        return {"s": s.item(), "c": int(c.item()), "h": h.cpu().numpy().copy(), "e": e.item()}

    _same(run(), run())
