"""Adversarial placements against the oracle, through the C-ABI: pairs whose
squared distance (or squared relative speed) lies on a histogram bin edge or
within a few FP64 ulps or a few FP32 units of one, and particles whose
fractional coordinates sit on cell faces or at the top of the unit interval
(s = 1 - 2^-53, where the wrap may round up).

Bins are right-closed on (0, hi] with squared edges E_k = (k hi / nbins)^2
(paper Code 10's binning rule; the last edge is the cutoff when hi is the
cutoff), so every count must equal the oracle's bit for bit in both
precisions: the FP32 form re-tests every value within its error band of an
edge in canonical FP64."""
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


RC = 8.0
# relative offsets from an edge: exact, 1-3 FP64 ulps, 1-4 FP32 units
DELTAS = np.array([0.0] + [s * k * 2.0 ** -52 for k in (1, 2, 3) for s in (1, -1)]
                  + [s * k * 2.0 ** -24 for k in (1, 2, 4) for s in (1, -1)])


def _unit(g, n, dim):
    u = g.normal(size=(n, dim))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _ulp_steps(e, steps):
    out = np.array(e, dtype=np.float64)
    for i, k in enumerate(steps):
        for _ in range(abs(int(k))):
            out[i] = np.nextafter(out[i], np.inf if k > 0 else -np.inf)
    return out


def edge_config(dim, nbins, hi, vhi, seed):
    """Isolated pairs (sites 20 or 25 apart, so no two pairs come within the
    cutoff 8 of each other):

    * exact pairs: A on the plane x = 0 (or y = 0), B = A + t e_x (or e_y) in
      a box of power-of-two sides, so the wrapped difference is t itself and
      d^2 = fl(t^2) with t = k hi / nbins stepped 0-3 FP64 ulps either way:
      on an edge or a few ulps off it; their relative speeds likewise
      (v_A = 0, v_B = s e_x);
    * random pairs: random direction, t = (k hi / nbins)(1 + delta) with delta
      up to 4 FP32 units, random base velocities.
    """
    L = 256.0 if dim == 3 else 1024.0
    H = np.diag([L] * dim)
    g = W.rng(seed)
    h, hv = hi / nbins, vhi / nbins
    if dim == 3:
        a = 2.0 + 20.0 * np.arange(int((L - 10) // 20))
        yy, zz = np.meshgrid(a, a, indexing="ij")
        fx = np.stack([np.zeros(yy.size), yy.ravel(), zz.ravel()], 1)           # pairs along x
        fy = np.stack([yy.ravel(), np.zeros(yy.size), zz.ravel() + 10.0], 1)    # along y, z shifted
        r = 40.0 + 25.0 * np.arange(8)
        rs = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    else:
        fx = np.stack([np.zeros(51), 2.0 + 20.0 * np.arange(51)], 1)
        fy = np.stack([32.0 + 20.0 * np.arange(48), np.zeros(48)], 1)
        r = 40.0 + 25.0 * np.arange(38)
        rs = np.stack(np.meshgrid(r, r, indexing="ij"), -1).reshape(-1, 2)
    ne = len(fx) + len(fy)
    k = g.integers(1, nbins + 1, size=ne)
    t = _ulp_steps(k * h, g.integers(-3, 4, size=ne))
    kv = g.integers(1, nbins + 1, size=ne)
    sv = _ulp_steps(kv * hv, g.integers(-3, 4, size=ne))
    ax = np.concatenate([np.zeros(len(fx), int), np.ones(len(fy), int)])
    De = np.zeros((ne, dim))
    De[np.arange(ne), ax] = t
    Ve = np.zeros((ne, dim))
    Ve[:, 0] = sv
    nr = len(rs)
    k = g.integers(1, nbins + 1, size=nr)
    t = (k * h) * (1.0 + DELTAS[g.integers(0, len(DELTAS), size=nr)])
    beyond = g.random(nr) < 0.05             # some pairs between hi and the cutoff
    if hi < RC:
        t = np.where(beyond, hi + (RC - hi) * g.random(nr), t)
    Ar = rs + 0.5 * g.random((nr, dim))
    Dr = t[:, None] * _unit(g, nr, dim)
    kv = g.integers(1, nbins + 1, size=nr)
    s = (kv * hv) * (1.0 + DELTAS[g.integers(0, len(DELTAS), size=nr)])
    vA = np.where((g.random(nr) < 0.5)[:, None], 0.0, g.normal(size=(nr, dim)))
    A = np.concatenate([fx, fy, Ar])
    B = A + np.concatenate([De, Dr])
    x = np.empty((2 * len(A), dim))
    x[0::2], x[1::2] = A, B
    v = np.empty_like(x)
    v[0::2] = np.concatenate([np.zeros((ne, dim)), vA])
    v[1::2] = np.concatenate([Ve, vA + s[:, None] * _unit(g, nr, dim)])
    return H, x, v, ne


def _near_edges(vals, nbins, hi, rel=16 * 2.0 ** -24):
    e = (np.arange(1, nbins + 1) * (hi / nbins)) ** 2
    k = np.clip(np.searchsorted(e, vals), 0, nbins - 1)
    km = np.clip(k - 1, 0, nbins - 1)
    near = (np.abs(vals - e[k]) <= rel * e[k]) | (np.abs(vals - e[km]) <= rel * e[km])
    return int(np.count_nonzero(near))


def _check_isolated(ref, ne):
    i, j = ref["nl_i"], ref["nl_j"]
    assert np.all(i % 2 == 0) and np.array_equal(j, i + 1), "only the constructed pairs interact"
    # the exact pairs: d^2 = fl(t^2), t the stepped edge (a few may lie beyond the cutoff)
    assert np.count_nonzero(i < 2 * ne) >= 0.9 * ne


@pytest.mark.parametrize("dim", [3, 2])
@pytest.mark.parametrize("nbins", [10, 128, 256, 1000])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_histograms_at_bin_edges(clm, dim, nbins, precision):
    vhi = 3.0
    H, x, v, ne = edge_config(dim, nbins, RC, vhi, 40 + nbins + dim)
    ref = oracle.compute(x, H, RC, nl=True, hist=(nbins, RC), rel_hist=(nbins, vhi), vel_x=v,
                         dist_vel_hist=(nbins, RC))
    _check_isolated(ref, ne)
    # the placement is adversarial: most pairs sit within 16 FP32 units of an edge
    assert _near_edges(ref["nl_d2"], nbins, RC) >= 0.8 * ref["count"]
    # and the exact pairs within 3 FP64 ulps of theirs
    assert _near_edges(ref["nl_d2"][ref["nl_i"] < 2 * ne], nbins, RC, rel=8 * 2.0 ** -52) \
        >= 0.9 * ne
    cl = clm.CellList(T(x), clm.Box(H, RC, 2), precision=precision)
    print(f"case dim={dim} nbins={nbins} {precision}", flush=True)
    h, c = cl.histogram(nbins, RC)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])
    assert int(c.item()) == ref["count"]
    hr, sums, c = cl.relspeed_histogram(T(v), nbins, vhi)
    assert np.array_equal(hr.cpu().numpy().astype(np.uint64), ref["rel_hist"])
    tol = 1e-12 if precision == "fp64" else 1e-6
    rs = ref["rel_sum"]
    assert np.all(np.abs(sums.cpu().numpy() - rs) <= tol * np.abs(rs) + 1e-300)
    hd, dsum, c = cl.dist_vel_histogram(T(v), nbins, RC)
    assert np.array_equal(hd.cpu().numpy().astype(np.uint64), ref["dv_hist"])
    assert np.all(np.abs(dsum.cpu().numpy() - ref["dv_sum"]) <= tol * np.abs(ref["dv_sum"]) + 1e-300)


@pytest.mark.parametrize("nbins", [10, 128, 1000])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_distance_histogram_edges_below_the_cutoff(clm, nbins, precision):
    """hi < cutoff: the last edge is (hi)^2 itself and pairs beyond it go to
    the overflow slot."""
    hi = 0.75 * RC
    H, x, v, ne = edge_config(3, nbins, hi, 2.0, 90 + nbins)
    ref = oracle.compute(x, H, RC, nl=True, hist=(nbins, hi), dist_vel_hist=(nbins, hi), vel_x=v)
    _check_isolated(ref, ne)
    assert ref["hist"][nbins] > 0
    cl = clm.CellList(T(x), clm.Box(H, RC, 1), precision=precision)
    h, _ = cl.histogram(nbins, hi)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])
    hd, _, _ = cl.dist_vel_histogram(T(v), nbins, hi)
    assert np.array_equal(hd.cpu().numpy().astype(np.uint64), ref["dv_hist"])


def _face_coords(g, n, ncell):
    """Fractional coordinates on cell faces c / ncell, one FP64 ulp either
    side, and at the ends of [0, 1): 0, 2^-53, 1 - 2^-53, 1 - 2^-52."""
    special = [0.0, 2.0 ** -53, 1.0 - 2.0 ** -53, 1.0 - 2.0 ** -52]
    c = g.integers(0, ncell + 1, size=n) / ncell
    side = g.integers(-1, 2, size=n)
    f = np.where(side < 0, np.nextafter(c, -np.inf), np.where(side > 0, np.nextafter(c, np.inf), c))
    sp = np.array(special)[g.integers(0, len(special), size=n)]
    pick = g.random(n)
    return np.where(pick < 0.25, sp, np.where(pick < 0.8, f, g.random(n)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lcell", [1, 2])
@pytest.mark.parametrize("dim", [3, 2])
def test_particles_on_cell_faces_and_the_top_of_the_cell(clm, precision, lcell, dim):
    """Orthorhombic box of power-of-two side: x = L s is exact, so the
    wrapped fractional coordinate is s itself, on a cell face c / ncell (as
    rounded), one ulp either side of it, or at 1 - 2^-53 (the largest value
    below 1); a tenth of the particles are moved by whole box vectors.  The
    pair set, the FP64 distances and a histogram must equal the oracle's."""
    L = 64.0
    rc = 4.0
    H = np.diag([L] * dim)
    box = clm.Box(H, rc, lcell)
    grid = box.info()["grid"]
    g = W.rng(300 + lcell + 10 * dim)
    n = 3000 if dim == 3 else 2000
    s = np.stack([_face_coords(g, n, grid[a]) for a in range(dim)], 1)
    x = s * L
    x[: n // 10] += L * g.integers(-2, 3, size=(n // 10, dim))   # other periodic images
    ref = oracle.compute(x, H, rc, nl=True, hist=(64, rc))
    cl = clm.CellList(T(x), box, precision=precision)
    pairs, d = cl.neighbor_list(sorted=True)
    p = pairs.cpu().numpy().astype(np.int64)
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    if precision == "fp64":
        assert np.array_equal(d.cpu().numpy(), ref["nl_d"])
    h, _ = cl.histogram(64, rc)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coincident_particles_and_the_zero_bin(clm, precision):
    """d = 0 (coincident particles, also one box vector apart) goes to the
    first bin (v <= E_1 with v = 0); the pair is in the set."""
    H = W.triclinic_h((30.0, 29.0, 33.0), (70.0, 110.0, 75.0))
    base = W.uniform_in_box(400, H, 8)
    x = np.concatenate([base, base[:50], base[50:80] + H @ np.array([1.0, -1.0, 2.0])])
    ref = oracle.compute(x, H, 4.0, nl=True, hist=(16, 4.0))
    cl = clm.CellList(T(x), clm.Box(H, 4.0, 2), precision=precision)
    h, c = cl.histogram(16, 4.0)
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["hist"])
    assert int(h[0].item()) >= 80
    pairs, _ = cl.neighbor_list(sorted=True)
    p = pairs.cpu().numpy().astype(np.int64)
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
