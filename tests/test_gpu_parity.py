"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, on the
same seeded inputs.  Integers (pair sets, counts, histograms) must be
bit-exact in both precisions; floating-point results must meet the stated
tolerances (FP64 form: 1e-12 relative for sums and energies; FP32+guard
form: 1e-6 for energies and sums, 1e-5 per-particle force error relative to
the sum of the pair-force magnitudes on that particle)."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch.backends.cuda.matmul.allow_tf32 = False


@pytest.fixture(scope="module")
def clm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2202_06427_amd as clm
    return clm


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


CASES = {
    "cube3": (np.diag([30.0, 30.0, 30.0]), 4000, 5.0),
    "ortho3": (np.diag([28.0, 34.0, 31.0]), 5000, 4.5),
    "tric3": (W.triclinic_h((32.0, 30.0, 31.0), (80.0, 95.0, 100.0)), 6000, 4.0),
    "skew3": (W.triclinic_h((30.0, 29.0, 33.0), (70.0, 110.0, 75.0)), 5000, 4.0),
    "sq2": (np.diag([60.0, 60.0]), 5000, 3.0),
    "tric2": (np.array([[55.0, -12.0], [0.0, 50.0]]), 4000, 3.2),
}


def _sorted_pairs(pairs):
    p = pairs.cpu().numpy().astype(np.int64)
    order = np.lexsort((p[:, 1], p[:, 0]))
    return p[order], order


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lcell,lcell_x", [(1, None), (2, None), (3, None), (1, 2), (2, 3), (2, 4)])
def test_neighbor_list_and_sums_exact(clm, name, precision, lcell, lcell_x):
    H, n, rc = CASES[name]
    x = W.uniform_in_box(n, H, 1000 + n)
    ref = oracle.compute(x, H, rc, nl=True, sum_d=True, sum_inv_d=True)
    box = clm.Box(H, rc, lcell, lcell_x)
    cl = clm.CellList(T(x), box, precision=precision)
    pairs, dist = cl.neighbor_list()
    p, order = _sorted_pairs(pairs)
    assert len(p) == ref["count"]
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    d = dist.cpu().numpy()[order]
    if precision == "fp64":
        assert np.array_equal(d, ref["nl_d"]), "FP64 distances are the canonical sqrt"
    else:
        assert np.abs(d - ref["nl_d"]).max() <= 2e-6 * rc
    c = int(cl.count().item())
    assert c == ref["count"]
    sd, c1 = cl.sum_d()
    sid, c2 = cl.sum_inv_d()
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert int(c1.item()) == ref["count"] == int(c2.item())
    assert abs(sd.item() / ref["sum_d"] - 1) < tol
    assert abs(sid.item() / ref["sum_inv_d"] - 1) < tol


def _pair_force_abs_sums(x, H, rc, ref, sigma, eps):
    """Per particle: sum over its pairs of |f_ij| (scale of the force error)."""
    n = len(x)
    d = ref["nl_d"]
    xx = (sigma / d) ** 2
    x3 = xx ** 3
    fmag = np.abs(24.0 * eps * (2 * x3 * x3 - x3) / d)
    s = np.zeros(n)
    np.add.at(s, ref["nl_i"], fmag)
    np.add.at(s, ref["nl_j"], fmag)
    return s


@pytest.mark.parametrize("name", ["cube3", "tric3", "skew3", "tric2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lcell,lcell_x", [(1, None), (2, None), (2, 3)])
def test_lj_energy_forces_box_gradient(clm, name, precision, lcell, lcell_x):
    H, n, rc = CASES[name]
    dim = H.shape[0]
    sigma, eps = 1.1, 0.3
    # jittered lattice: no coincident pairs, physical LJ magnitudes
    m = int(round(n ** (1.0 / dim)))
    grid = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    s = (grid + 0.5 + 0.3 * (W.rng(7).random(grid.shape) - 0.5)) / m
    x = s @ H.T + (H @ np.array([3, -2, 5][:dim]))  # positions outside the primary cell
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True, nl=True)
    box = clm.Box(H, rc, lcell, lcell_x)
    cl = clm.CellList(T(x), box, precision=precision)
    e, c = cl.lj_energy(sigma, eps)
    assert int(c.item()) == ref["count"]
    tolE = 1e-12 if precision == "fp64" else 1e-6
    assert abs(e.item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    out = cl.lj_forces(sigma, eps, virial=True)
    assert int(out["count"].item()) == ref["count"]
    assert abs(out["energy"].item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    F = out["forces"].cpu().numpy()
    G = ref["lj_grad"]
    scale = _pair_force_abs_sums(x, H, rc, ref, sigma, eps)
    err = np.linalg.norm(F + G, axis=1) / np.maximum(scale, 1e-300)
    tolF = 1e-11 if precision == "fp64" else 1e-5
    assert err.max() <= tolF, err.max()
    Fsum = np.linalg.norm(F.sum(0))
    assert Fsum <= 1e-10 * np.linalg.norm(F, axis=1).sum() * (1 if precision == "fp64" else 1e4)
    tolB = 1e-11 if precision == "fp64" else 1e-5
    dEdH = out["grad_box"].cpu().numpy()
    assert np.abs(dEdH - ref["dEdH"]).max() <= tolB * np.abs(ref["dEdH"]).max()
    Wv = out["virial"].cpu().numpy()
    assert np.abs(Wv - ref["virial"]).max() <= tolB * np.abs(ref["virial"]).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lj_near_pairs_uniform_random(clm, precision):
    # uniform random points: a few pairs are far inside sigma and dominate E
    H, n, rc = CASES["tric3"]
    x = W.uniform_in_box(n, H, 77)
    sigma, eps = 3.4, 0.238
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    e, c = cl.lj_energy(sigma, eps)
    tolE = 1e-12 if precision == "fp64" else 1e-6
    assert abs(e.item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    out = cl.lj_forces(sigma, eps)
    G = ref["lj_grad"]
    F = out["forces"].cpu().numpy()
    rel = np.linalg.norm(F + G, axis=1).max() / np.linalg.norm(G, axis=1).max()
    assert rel <= (1e-11 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("name", ["cube3", "tric3", "sq2", "tric2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_distance_histogram_exact(clm, name, precision):
    H, n, rc = CASES[name]
    x = W.uniform_in_box(n, H, 2000 + n)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    for nb, hi in [(128, rc), (37, 0.73 * rc), (10, 2.0 * rc)]:
        ref = oracle.compute(x, H, rc, hist=(nb, hi))
        h, c = cl.histogram(nb, hi)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"]), (nb, hi)
        assert int(c.item()) == ref["count"]


@pytest.mark.parametrize("name", ["cube3", "tric3", "sq2", "tric2"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_relative_speed_histogram_exact(clm, name, precision):
    H, n, rc = CASES[name]
    dim = H.shape[0]
    x = W.uniform_in_box(n, H, 3000 + n)
    v = W.rng(5).normal(size=(n, dim))
    ref = oracle.compute(x, H, rc, rel_hist=(64, 6.0), vel_x=v)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    h, sums, c = cl.relspeed_histogram(T(v), 64, 6.0)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["rel_hist"])
    assert int(c.item()) == ref["count"]
    tol = 1e-12 if precision == "fp64" else 1e-6
    rs = ref["rel_sum"]
    assert np.all(np.abs(sums.cpu().numpy() - rs) <= tol * np.maximum(np.abs(rs), 1e-300) + 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cross_set_neighbor_list(clm, precision):
    H = np.diag([40.0, 40.0, 40.0])
    x = np.mod(W.rng(1).normal(20.0, 4.0, size=(700, 3)), 40.0)
    y = W.uniform_in_box(20000, H, 2)
    rc = 3.0
    ref = oracle.compute(x, H, rc, y, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, 1), y=T(y), precision=precision)
    pairs, _ = cl.neighbor_list()
    p, _ = _sorted_pairs(pairs)
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_box_minimum_image(clm, precision):
    H = W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0))
    x = W.uniform_in_box(300, H, 51)
    rc = 7.0
    ref = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, hist=(16, rc))
    box = clm.Box(H, rc, 1)
    assert box.info()["small_box"]
    cl = clm.CellList(T(x), box, precision=precision)
    pairs, d = cl.neighbor_list()
    p, order = _sorted_pairs(pairs)
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    assert np.array_equal(d.cpu().numpy()[order], ref["nl_d"])
    out = cl.lj_forces(1.0, 0.5, virial=True)
    assert int(out["count"].item()) == ref["count"]
    assert abs(out["energy"].item() / ref["lj_energy"] - 1) < 1e-12
    assert np.allclose(out["forces"].cpu().numpy(), -ref["lj_grad"], rtol=1e-10, atol=1e-12 * np.abs(ref["lj_grad"]).max())
    # box gradient and virial: the brute-force path sums per j-chunk partials
    assert np.abs(out["grad_box"].cpu().numpy() - ref["dEdH"]).max() <= 1e-11 * np.abs(ref["dEdH"]).max()
    assert np.abs(out["virial"].cpu().numpy() - ref["virial"]).max() <= 1e-11 * np.abs(ref["virial"]).max()
    h, _ = cl.histogram(16, rc)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_box_many_chunks_2d_and_cross(clm, precision):
    """Brute-force path with thousands of particles (many i blocks x j
    chunks), in 2D and for a cross set."""
    H2 = np.array([[9.0, 2.0], [0.0, 8.5]])
    x2 = W.uniform_in_box(3000, H2, 52)
    rc = 5.0
    ref = oracle.compute(x2, H2, rc, lj=(0.7, 0.2), lj_grad=True, sum_inv_d=True)
    box2 = clm.Box(H2, rc, 1)
    assert box2.info()["small_box"]
    cl = clm.CellList(T(x2), box2, precision=precision)
    out = cl.lj_forces(0.7, 0.2)
    assert int(out["count"].item()) == ref["count"]
    assert abs(out["energy"].item() / ref["lj_energy"] - 1) < 1e-12
    G = ref["lj_grad"]
    assert np.linalg.norm(out["forces"].cpu().numpy() + G, axis=1).max() <= 1e-10 * np.linalg.norm(G, axis=1).max()
    assert np.abs(out["grad_box"].cpu().numpy() - ref["dEdH"]).max() <= 1e-11 * np.abs(ref["dEdH"]).max()
    s, c = cl.sum_inv_d()
    assert int(c.item()) == ref["count"] and abs(s.item() / ref["sum_inv_d"] - 1) < 1e-12
    H3 = W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0))
    xa, ya = W.uniform_in_box(700, H3, 53), W.uniform_in_box(1900, H3, 54)
    refc = oracle.compute(xa, H3, 6.0, ya, nl=True)
    clc = clm.CellList(T(xa), clm.Box(H3, 6.0, 1), y=T(ya), precision=precision)
    pairs, _ = clc.neighbor_list()
    p, _ = _sorted_pairs(pairs)
    assert len(p) == refc["count"]
    assert np.array_equal(p[:, 0], refc["nl_i"]) and np.array_equal(p[:, 1], refc["nl_j"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_guard_band_adversarial_pairs(clm, precision):
    # pairs whose distance is the cutoff up to a few units in the last place:
    # membership must follow the canonical FP64 squared distance exactly
    H = np.diag([50.0, 50.0, 50.0])
    rc = 4.0
    g = W.rng(9)
    pts = []
    for k in range(400):
        c = g.random(3) * 50.0
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        t = rc * (1.0 + (k % 41 - 20) * 2.0 ** -52)
        if k % 3 == 0:
            t = rc * (1.0 + (k % 41 - 20) * 2.0 ** -25)  # FP32-scale offsets
        pts += [c, c + t * u]
    x = np.array(pts)
    ref = oracle.compute(x, H, rc, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    pairs, _ = cl.neighbor_list()
    p, _ = _sorted_pairs(pairs)
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    h, _ = cl.histogram(8, rc)
    assert int(h.sum().item()) == ref["count"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_degenerate_sizes(clm, precision):
    H = np.diag([30.0, 30.0, 30.0])
    for n in (0, 1, 2, 3, 65, 129):
        x = W.uniform_in_box(n, H, 60 + n)
        if n == 2:
            x = np.array([[1.0, 1.0, 1.0], [29.5, 1.0, 1.0]])  # across the boundary
        cl = clm.CellList(T(x.reshape(n, 3)), clm.Box(H, 5.0, 2), precision=precision)
        ref = oracle.compute(x.reshape(n, 3), H, 5.0, nl=True) if n else {"count": 0}
        assert int(cl.count().item()) == ref["count"]


def test_all_particles_in_one_cell_and_heavy_tiles(clm):
    H = np.diag([40.0, 40.0, 40.0])
    g = W.rng(3)
    x = np.concatenate([20.0 + 0.8 * g.random((900, 3)), W.uniform_in_box(3000, H, 4)])
    ref = oracle.compute(x, H, 3.0, nl=True, sum_inv_d=True)
    for precision in ("fp64", "fp32"):
        cl = clm.CellList(T(x), clm.Box(H, 3.0, 2), precision=precision)
        pairs, _ = cl.neighbor_list()
        p, _ = _sorted_pairs(pairs)
        assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
        s, _ = cl.sum_inv_d()
        assert abs(s.item() / ref["sum_inv_d"] - 1) < (1e-12 if precision == "fp64" else 1e-6)
    # LJ forces with the heavy cell: many tiles of one cell, and overlapping
    # pairs far inside sigma (re-evaluated in FP64)
    sigma, eps = 0.2, 0.01
    refl = oracle.compute(x, H, 3.0, lj=(sigma, eps), lj_grad=True)
    cl = clm.CellList(T(x), clm.Box(H, 3.0, 2), precision="fp32")
    out = cl.lj_forces(sigma, eps)
    assert int(out["count"].item()) == refl["count"]
    F = out["forces"].cpu().numpy()
    rel = np.linalg.norm(F + refl["lj_grad"], axis=1).max() / np.linalg.norm(refl["lj_grad"], axis=1).max()
    assert rel <= 1e-6


def test_autograd_lj_energy(clm):
    H = W.triclinic_h((30.0, 31.0, 29.0), (85.0, 95.0, 100.0))
    m = 14
    grid = np.stack(np.meshgrid(*([np.arange(m)] * 3), indexing="ij"), -1).reshape(-1, 3)
    x = ((grid + 0.5 + 0.3 * (W.rng(8).random(grid.shape) - 0.5)) / m) @ H.T
    sigma, eps, rc = 1.5, 0.4, 5.0
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True)
    for precision in ("fp64", "fp32"):
        xt = T(x).requires_grad_(True)
        Ht = torch.from_numpy(H.copy()).requires_grad_(True)
        E = clm.lj_energy(xt, Ht, sigma, eps, rc, 2, precision)
        (2.5 * E).backward()
        tol = 1e-11 if precision == "fp64" else 1e-5
        gx = xt.grad.cpu().numpy()
        assert np.abs(gx - 2.5 * ref["lj_grad"]).max() <= tol * np.abs(ref["lj_grad"]).max() * 2.5
        assert np.abs(Ht.grad.numpy() - 2.5 * ref["dEdH"]).max() <= tol * np.abs(ref["dEdH"]).max() * 2.5


@pytest.mark.parametrize("name", ["cube3", "tric3", "tric2", "small3"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_map_cutoff_below_the_box_cutoff(clm, name, precision):
    """A map with its own cutoff rm < rc over the cell list built for rc
    gives the pair set and sums of the definition at rm."""
    if name == "small3":
        H, n, rc = W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0)), 500, 7.0
    else:
        H, n, rc = CASES[name]
    dim = H.shape[0]
    x = W.uniform_in_box(n, H, 4000 + n)
    v = W.rng(6).normal(size=(n, dim))
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    assert cl.box.info()["small_box"] == (name == "small3")
    tol = 1e-12 if precision == "fp64" else 1e-6
    for rm in (0.61 * rc, rc):
        ref = oracle.compute(x, H, rm, nl=True, sum_d=True, hist=(24, rm), rel_hist=(16, 5.0),
                             vel_x=v)
        pairs, dist = cl.neighbor_list(cutoff=rm)
        p, order = _sorted_pairs(pairs)
        assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
        assert int(cl.count(cutoff=rm).item()) == ref["count"]
        sd, c = cl.sum_d(cutoff=rm)
        assert int(c.item()) == ref["count"] and abs(sd.item() / ref["sum_d"] - 1) < tol
        h, _ = cl.histogram(24, cutoff=rm)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])
        hr, _, c = cl.relspeed_histogram(T(v), 16, 5.0, cutoff=rm)
        assert np.array_equal(hr.cpu().numpy().astype(np.uint64), ref["rel_hist"])
        assert int(c.item()) == ref["count"]
    # forces on a jittered lattice (no coincident pairs)
    m = int(round(n ** (1.0 / dim)))
    grid = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    s = (grid + 0.5 + 0.3 * (W.rng(8).random(grid.shape) - 0.5)) / m
    xl = s @ H.T
    rm = 0.7 * rc
    ref = oracle.compute(xl, H, rm, lj=(1.1, 0.3), lj_grad=True, nl=True)
    cll = clm.CellList(T(xl), clm.Box(H, rc, 2), precision=precision)
    out = cll.lj_forces(1.1, 0.3, virial=True, cutoff=rm)
    assert int(out["count"].item()) == ref["count"]
    assert abs(out["energy"].item() - ref["lj_energy"]) <= tol * abs(ref["lj_energy"])
    scale = _pair_force_abs_sums(xl, H, rm, ref, 1.1, 0.3)
    err = np.linalg.norm(out["forces"].cpu().numpy() + ref["lj_grad"], axis=1) / np.maximum(scale, 1e-300)
    assert err.max() <= (1e-11 if precision == "fp64" else 1e-5)
    tolB = 1e-11 if precision == "fp64" else 1e-5
    assert np.abs(out["grad_box"].cpu().numpy() - ref["dEdH"]).max() <= tolB * np.abs(ref["dEdH"]).max()
    with pytest.raises(clm.ClmError):
        cl.count(cutoff=1.01 * rc)
