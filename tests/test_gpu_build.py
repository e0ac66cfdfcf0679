"""GPU parity of the cell-list build (LDS bucket counts, bucket records,
per-bucket placement) on inputs that reach its less common paths: a bucket
too large for the LDS assembly (written in place), every particle in one
cell, a sparse box whose buckets hold thousands of empty cells, and 2D.
Pair sets and FP64 distances are compared with the oracle bit for bit, and
every cell's particles must be exactly those the canonical wrap puts there."""
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


def _check_pairs(clm, x, H, rc, lcell=2, precision="fp64"):
    ref = oracle.compute(x, H, rc, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, lcell), precision=precision)
    pairs, d = cl.neighbor_list(sorted=True)
    p = pairs.cpu().numpy().astype(np.int64)
    assert len(p) == ref["count"]
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    if precision == "fp64":
        assert np.array_equal(d.cpu().numpy(), ref["nl_d"])
    return cl


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bucket_larger_than_the_lds_assembly(clm, precision):
    """5000 particles in a cube of side 1.5 (cells of side 1, rows of 60
    cells, buckets of 1024 consecutive cells: the cluster falls in two
    buckets of about 2500 particles, beyond the 2048 the placement
    assembles in LDS) among 20000 uniform ones."""
    H = np.diag([60.0, 60.0, 60.0])
    g = W.rng(41)
    x = np.concatenate([30.1 + 1.5 * g.random((5000, 3)), W.uniform_in_box(20000, H, 42)])
    x = x[g.permutation(len(x))]
    cl = _check_pairs(clm, x, H, 2.0, precision=precision)
    assert cl.info()["max_occupancy"] > 1000


def test_all_particles_in_one_cell(clm):
    H = np.diag([40.0, 40.0, 40.0])
    x = 9.3 + 0.9 * W.rng(43).random((3000, 3))  # inside cell 6 of 26 per axis: [9.23, 10.77)
    cl = _check_pairs(clm, x, H, 3.0)
    info = cl.info()
    assert info["nonempty_cells"] == 1 and info["max_occupancy"] == 3000


def test_sparse_box_with_mostly_empty_buckets(clm):
    """2000 particles in a box with 2.6e5 cells: buckets of hundreds of cells
    with a few particles or none."""
    H = np.diag([320.0, 320.0, 320.0])
    x = W.uniform_in_box(2000, H, 44)
    x = np.concatenate([x, x[:200] + 0.3])  # some close pairs
    cl = _check_pairs(clm, x, H, 5.0)
    assert cl.info()["ncells"] > 2 * 10 ** 5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_2d_clustered(clm, precision):
    H = np.diag([1.0, 1.0])
    g = W.rng(45)
    centres = g.random((20, 2))
    x = np.concatenate([np.mod(c + 0.003 * g.normal(size=(600, 2)), 1.0) for c in centres]
                       + [W.uniform_in_box(4000, H, 46)])
    x = x[g.permutation(len(x))]
    _check_pairs(clm, x, H, 0.01, precision=precision)


def test_cell_membership_is_the_canonical_wrap(clm):
    """Every particle sits in the cell its canonical wrapped position falls
    in, and every cell's particles are contiguous (checked through a
    neighbour list at the smallest cutoff: a pair set that equals the
    oracle's at cutoffs of 1/3 and 1 cell width on a triclinic box)."""
    H = W.triclinic_h((30.0, 31.0, 29.0), (75.0, 100.0, 95.0))
    x = W.uniform_in_box(8000, H, 47) + H @ np.array([5.0, -3.0, 2.0])
    for rc in (1.0, 3.0):
        _check_pairs(clm, x, H, rc, lcell=1)


def _stencil_pairs(x, H, grid, lx, l):
    """Candidate pairs of the cell method on a grid, by counting: the
    particles of each cell times those of each cell of its half-shell stencil
    (lx cells on along x; the rows with (dz, dy) > (0, 0) over the whole x
    reach), plus the pairs within a cell."""
    dim = H.shape[0]
    s = x @ np.linalg.inv(H).T
    s -= np.floor(s)
    n = np.array(grid)
    cell = np.minimum((s * n).astype(np.int64), n - 1)
    shape = tuple(n[::-1])
    cnt = np.zeros(shape, np.int64)
    np.add.at(cnt, tuple(cell[:, a] for a in reversed(range(dim))), 1)
    tot = int((cnt * (cnt - 1) // 2).sum())
    for dz in (range(0, l + 1) if dim == 3 else [0]):
        for dy in range(-l, l + 1):
            if dz == 0 and dy < 0:
                continue
            for dx in range(-lx, lx + 1):
                if dz == 0 and dy == 0 and dx <= 0:
                    continue
                sh = (-dz, -dy, -dx)[3 - dim:]
                tot += int((cnt * np.roll(cnt, shift=sh, axis=tuple(range(dim)))).sum())
    return tot


@pytest.mark.parametrize("case", ["tric3", "tric3_x6", "square2"])
def test_candidate_pairs_are_the_grids_half_shell(clm, case):
    """The candidate count reported with the cell list (the roofline unit)
    is the half-shell cell-pair count of the grid, whatever the tiles."""
    if case == "square2":
        H = np.diag([60.0, 60.0])
        x = W.uniform_in_box(20_000, H, 48)
        box = clm.Box(H, 2.0, 2)
    else:
        H = W.triclinic_h((50.0, 48.0, 52.0), (80.0, 95.0, 100.0))
        x = W.uniform_in_box(12_000, H, 49)
        box = clm.Box(H, 6.0, 2, 6 if case == "tric3_x6" else None)
    bi = box.info()
    cl = clm.CellList(T(x), box, precision="fp32")
    info = cl.info()
    assert info["candidate_pairs"] == _stencil_pairs(x, H, bi["grid"], bi["lcell_x"], bi["lcell"])
