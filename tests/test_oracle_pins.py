"""Pins for the CPU oracle, against things other than the oracle itself.

Each test ties an oracle function to a fact fixed by the paper or by the
mathematics: printed worked examples (tests/golden), closed forms, brute
force, scipy's periodic k-d tree, invariances and statistical expectations
for uniform points.  None of these tests needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

BOXES = {
    "cube3": np.diag([20.0, 20.0, 20.0]),
    "ortho3": np.diag([18.0, 23.0, 21.0]),
    "tric3": W.triclinic_h((20.0, 22.0, 21.0), (80.0, 95.0, 100.0)),
    "skew3": W.triclinic_h((20.0, 20.0, 22.0), (70.0, 110.0, 75.0)),
    "sq2": np.diag([25.0, 25.0]),
    "tric2": np.array([[24.0, -7.0], [0.0, 22.0]]),
}


def exhaustive_d2(xi, xj, H, kmax=3):
    """Minimum over every image K in [-kmax, kmax]^dim of |x_j - x_i + H K|^2 (numpy)."""
    dim = H.shape[0]
    rng = np.arange(-kmax, kmax + 1)
    Ks = np.stack(np.meshgrid(*([rng] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    D = (xj - xi)[None, :] + Ks @ H.T
    d2 = (D * D).sum(1)
    return d2.min()


# ---------------------------------------------------------------- box setup

@pytest.mark.parametrize("name", list(BOXES))
def test_inverse_is_inverse(name):
    H = BOXES[name]
    Hi = oracle.box_inverse(H)
    assert np.abs(H @ Hi - np.eye(H.shape[0])).max() < 1e-14
    assert np.abs(Hi @ H - np.eye(H.shape[0])).max() < 1e-14


@pytest.mark.parametrize("name", list(BOXES))
def test_widths_match_face_normals(name):
    # the perpendicular width along axis d is 1/|row d of H^-1| (independent formula)
    H = BOXES[name]
    w, V = oracle.box_widths(H)
    w_ref = 1.0 / np.linalg.norm(np.linalg.inv(H), axis=1)
    assert np.allclose(w, w_ref, rtol=1e-13)
    assert math.isclose(V, abs(np.linalg.det(H)), rel_tol=1e-13)


def test_lengths_angles_roundtrip():
    L = np.array([215.4, 215.4, 215.4])
    A = np.array([80.0, 95.0, 100.0])
    H = oracle.box_from_lengths_angles(L, A)
    a, b, c = H[:, 0], H[:, 1], H[:, 2]
    assert np.allclose([np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)], L, rtol=1e-14)
    ang = lambda u, v: math.degrees(math.acos(u @ v / np.linalg.norm(u) / np.linalg.norm(v)))
    assert np.allclose([ang(b, c), ang(a, c), ang(a, b)], A, atol=1e-10)
    assert np.allclose(H, W.triclinic_h(L, A), rtol=1e-14, atol=1e-12)


def test_code3_grid_and_column_convention(golden_dir):
    """Paper Code 3: lattice vectors are the columns of the input matrix."""
    g = json.load(open(os.path.join(golden_dir, "code3_box_grids.json")))
    for case in g["cases"]:
        H = np.array(case["input_rows"], dtype=float)
        printed = np.array(case["printed_unit_cell"]).reshape(3, 3)  # one lattice vector per row
        assert np.array_equal(printed, H.T), "printed unit cell = columns of H"
        n, sizes = oracle.paper_ghost_grid(H, case["cutoff"], 1)
        assert list(n) == case["cells_per_dim"]
        assert np.allclose(sizes, case["cell_sizes"], rtol=1e-12)
        assert int(np.prod(n)) == case["total_cells"]
        # rows-as-vectors would put the z extent (30) on y: the grid would differ
        n_rows, _ = oracle.paper_ghost_grid(H.T.copy(), case["cutoff"], 1)
        if not case["orthorhombic"]:
            assert list(n_rows) != case["cells_per_dim"]


# ---------------------------------------------------------------- wrapping

@pytest.mark.parametrize("name", list(BOXES))
def test_wrap_properties(name):
    H = BOXES[name]
    dim = H.shape[0]
    g = W.rng(11)
    x = (g.random((500, dim)) * 6.0 - 2.5) @ H.T  # spans several cells in every direction
    xw, fr, w = oracle.wrap(x, H)
    assert (fr >= 0).all() and (fr < 1).all()
    # wrapped = raw - H w, up to rounding
    assert np.abs(xw - (x - w @ H.T)).max() < 1e-11
    # shifting by a lattice vector changes only the wrap integers
    K = np.array([3, -2, 5][:dim])
    xw2, fr2, w2 = oracle.wrap(x + H @ K, H)
    assert (w2 - w == K).all()
    assert np.abs(xw2 - xw).max() < 1e-10


# ---------------------------------------------------------------- minimum image

@pytest.mark.parametrize("name", list(BOXES))
def test_min_image_vs_exhaustive(name):
    H = BOXES[name]
    dim = H.shape[0]
    g = W.rng(12)
    w, _ = oracle.box_widths(H)
    for _ in range(300):
        xi = g.random(dim) @ H.T + g.normal(0, 30, dim)
        xj = g.random(dim) @ H.T + g.normal(0, 30, dim)
        d2, K = oracle.pair_d2(xi, xj, H, reach=10 * w.max())
        ref = exhaustive_d2(xi, xj, H, kmax=8)
        assert math.isclose(d2, ref, rel_tol=1e-9, abs_tol=1e-9)
        D = xj - xi + H @ K
        assert math.isclose(D @ D, d2, rel_tol=1e-9, abs_tol=1e-9)


# ---------------------------------------------------------------- pair sets

@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("rc_frac", [0.12, 0.3])
def test_brute_force_equals_cell_list(name, rc_frac):
    H = BOXES[name]
    dim = H.shape[0]
    w, _ = oracle.box_widths(H)
    rc = rc_frac * w.min()
    n = 900 if dim == 3 else 700
    x = W.uniform_in_box(n, H, 21)
    v = W.rng(22).normal(size=(n, dim))
    kw = dict(sum_d=True, sum_inv_d=True, lj=(1.1, 0.3), lj_grad=True, hist=(24, rc),
              rel_hist=(16, 4.0), vel_x=v, nl=True)
    b = oracle.compute(x, H, rc, method=oracle.METHOD_BRUTE, **kw)
    c = oracle.compute(x, H, rc, method=oracle.METHOD_AUTO, **kw)
    if rc_frac <= 0.3:
        assert c["method"] == oracle.METHOD_CELLS
    assert b["count"] == c["count"] > 0
    assert np.array_equal(b["nl_i"], c["nl_i"]) and np.array_equal(b["nl_j"], c["nl_j"])
    assert np.array_equal(b["nl_d"], c["nl_d"])
    assert np.array_equal(b["hist"], c["hist"])
    assert np.array_equal(b["rel_hist"], c["rel_hist"])
    for k in ("sum_d", "sum_inv_d", "lj_energy"):
        assert math.isclose(b[k], c[k], rel_tol=1e-13), k
    assert np.allclose(b["virial"], c["virial"], rtol=1e-12, atol=1e-12 * abs(b["virial"]).max())
    assert np.allclose(b["lj_grad"], c["lj_grad"], rtol=1e-12, atol=1e-12 * abs(b["lj_grad"]).max())
    assert np.allclose(b["rel_sum"], c["rel_sum"], rtol=1e-13)


@pytest.mark.parametrize("name", ["cube3", "ortho3", "sq2"])
def test_pair_set_vs_scipy_periodic_kdtree(name):
    from scipy.spatial import cKDTree
    H = BOXES[name]
    L = np.diag(H)
    rc = 0.27 * L.min()
    x = W.uniform_in_box(1200, H, 31)
    r = oracle.compute(x, H, rc, nl=True)
    ours = set(zip(r["nl_i"].tolist(), r["nl_j"].tolist()))
    theirs = set(cKDTree(np.mod(x, L), boxsize=L).query_pairs(rc))
    diff = ours ^ theirs
    for i, j in diff:  # only pairs at the cutoff up to rounding may differ
        d2, _ = oracle.pair_d2(x[i], x[j], H, rc * 2)
        assert abs(d2 - rc * rc) < 1e-12 * rc * rc
    assert len(ours) > 1000


@pytest.mark.parametrize("name", ["cube3", "tric3", "sq2"])
def test_nl_distance_is_min_image_norm(name):
    H = BOXES[name]
    w, _ = oracle.box_widths(H)
    rc = 0.25 * w.min()
    x = W.uniform_in_box(400, H, 41)
    r = oracle.compute(x, H, rc, nl=True)
    for i, j, d in list(zip(r["nl_i"], r["nl_j"], r["nl_d"]))[::7]:
        ref = math.sqrt(exhaustive_d2(x[i], x[j], H))
        assert math.isclose(d, ref, rel_tol=1e-12)


def test_small_box_min_image_one_image_per_pair():
    # rc above half the box: each pair counted once, with its nearest image
    H = W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0))
    x = W.uniform_in_box(150, H, 51)
    rc = 7.0
    r = oracle.compute(x, H, rc, nl=True, sum_d=True)
    assert r["method"] == oracle.METHOD_BRUTE
    ref = []
    for i in range(len(x)):
        for j in range(i + 1, len(x)):
            d2 = exhaustive_d2(x[i], x[j], H, kmax=3)
            if d2 <= rc * rc:
                ref.append((i, j, math.sqrt(d2)))
    assert r["count"] == len(ref)
    assert list(zip(r["nl_i"].tolist(), r["nl_j"].tolist())) == [(i, j) for i, j, _ in ref]
    assert math.isclose(r["sum_d"], sum(d for _, _, d in ref), rel_tol=1e-12)


def test_cross_set_is_union_minus_parts():
    H = BOXES["tric3"]
    x = W.uniform_in_box(300, H, 61)
    y = W.uniform_in_box(700, H, 62)
    rc = 5.0
    cxy = oracle.compute(x, H, rc, y)["count"]
    both = oracle.compute(np.concatenate([x, y]), H, rc)["count"]
    cx = oracle.compute(x, H, rc)["count"]
    cy = oracle.compute(y, H, rc)["count"]
    assert cxy == both - cx - cy
    nl = oracle.compute(x, H, rc, y, nl=True)
    assert nl["nl_count"] == cxy and (nl["nl_i"] < 300).all() and (nl["nl_j"] < 700).all()


# ---------------------------------------------------------------- closed forms / statistics

def _ideal_gas(n, V, rc, dim):
    M = n * (n - 1) / 2
    p = (4.0 / 3.0) * math.pi * rc ** 3 / V if dim == 3 else math.pi * rc ** 2 / V
    return M * p, math.sqrt(M * p * (1 - p))


@pytest.mark.parametrize("seed", [101, 102, 103])
def test_ideal_gas_pair_count_3sigma(seed):
    H = BOXES["tric3"]
    _, V = oracle.box_widths(H)
    n, rc = 3000, 6.0
    x = W.uniform_in_box(n, H, seed)
    mu, sd = _ideal_gas(n, V, rc, 3)
    assert abs(oracle.compute(x, H, rc)["count"] - mu) < 3 * sd


def test_ideal_gas_config1_scale():
    c = W.config1()
    mu, sd = _ideal_gas(10_000, 46.42 ** 3, 8.0, 3)
    r = oracle.compute(c["x"], c["H"], c["cutoff"], sum_d=True, sum_inv_d=True)
    assert abs(r["count"] - mu) < 3 * sd
    M = 10_000 * 9_999 / 2
    V = 46.42 ** 3
    # E[sum 1/d] = M 2 pi rc^2 / V, E[sum d] = M pi rc^4 / V (uniform periodic points)
    assert abs(r["sum_inv_d"] / (M * 2 * math.pi * 8.0 ** 2 / V) - 1) < 0.01
    assert abs(r["sum_d"] / (M * math.pi * 8.0 ** 4 / V) - 1) < 0.01


def test_code9_sum_of_distances_statistical(golden_dir):
    """Paper Code 9 prints sum d = 10.446 for 1000 points, unit box, rc 0.05."""
    g = json.load(open(os.path.join(golden_dir, "code9_sum_d.json")))
    n, rc = g["n"], g["cutoff"]
    H = np.eye(3) * g["side"]
    vals = [oracle.compute(W.uniform_in_box(n, H, 1000 + s), H, rc, sum_d=True)["sum_d"]
            for s in range(120)]
    mean, sd = float(np.mean(vals)), float(np.std(vals))
    M = n * (n - 1) / 2
    expected = M * math.pi * rc ** 4  # closed form E[sum d]
    assert abs(mean - expected) < 4 * sd / math.sqrt(len(vals))
    assert abs(g["printed_value"] - mean) < 3 * sd


def test_distance_histogram_uniform_chi2():
    H = BOXES["cube3"]
    n, rc, nb = 4000, 6.0, 12
    x = W.uniform_in_box(n, H, 71)
    r = oracle.compute(x, H, rc, hist=(nb, rc))
    h = r["hist"]
    assert h[nb] == 0 and int(h.sum()) == r["count"]
    M = n * (n - 1) / 2
    e = np.arange(nb + 1) * rc / nb
    expct = M * (4.0 / 3.0) * math.pi * np.diff(e ** 3) / 8000.0
    chi2 = (((h[:nb] - expct) ** 2) / expct).sum()
    assert chi2 < 35.0  # 12 dof, p ~ 5e-4


def test_code10_binning_rule(golden_dir):
    """Right-closed bins of width binstep: paper Code 10 rounding-up rule."""
    g = json.load(open(os.path.join(golden_dir, "code10_binning.json")))
    step, nb = g["binstep"], g["nbins"]
    rc = step * nb
    H = np.eye(3) * 100.0
    for d, b1 in g["cases_d_and_bin_1based"] + [(d, None) for d in g["beyond_last_bin_d"]]:
        x = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]])
        r = oracle.compute(x, H, 6.0, hist=(nb, rc))
        got = int(np.nonzero(r["hist"])[0][0])
        assert got == (nb if b1 is None else b1 - 1), (d, got)


def test_two_particle_lj_closed_forms():
    s, e = 3.4, 0.238
    H = np.eye(3) * 50.0
    for d, u_ref, g_ref in [(s, 0.0, 24 * e / s), (2 ** (1 / 6) * s, -e, 0.0)]:
        x = np.array([[5.0, 5.0, 5.0], [5.0 + d, 5.0, 5.0]])
        r = oracle.compute(x, H, 12.0, lj=(s, e), lj_grad=True)
        assert abs(r["lj_energy"] - u_ref) < 1e-13
        # dE/dx_0: moving particle 0 towards 1 on the repulsive wall raises E
        assert abs(r["lj_grad"][0, 0] - g_ref) < 1e-12 and abs(r["lj_grad"][1, 0] + g_ref) < 1e-12
        assert math.isclose(r["virial"][0, 0], g_ref * d, rel_tol=1e-12, abs_tol=1e-12)


# ---------------------------------------------------------------- derivatives (no formula retyped)

def _lattice(H, m, seed, jitter=0.15):
    g = W.rng(seed)
    dim = H.shape[0]
    grid = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    s = (grid + 0.5 + jitter * (g.random(grid.shape) - 0.5)) / m
    return s @ H.T


def test_forces_sum_to_zero():
    H = BOXES["tric3"]
    x = W.uniform_in_box(2000, H, 81)
    r = oracle.compute(x, H, 6.0, lj=(3.4, 0.238), lj_grad=True)
    G = r["lj_grad"]
    assert np.linalg.norm(G.sum(0)) <= 1e-10 * np.linalg.norm(G, axis=1).sum()


@pytest.mark.parametrize("name", ["tric3", "tric2"])
def test_gradient_vs_finite_differences(name):
    H = BOXES[name]
    dim = H.shape[0]
    x = _lattice(H, 8 if dim == 3 else 20, 91)
    s, e, rc = 3.0, 0.238, 6.5
    r = oracle.compute(x, H, rc, lj=(s, e), lj_grad=True)
    h = 1e-6
    for i in (0, 17, 101):
        for a in range(dim):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd = (oracle.compute(xp, H, rc, lj=(s, e))["lj_energy"]
                  - oracle.compute(xm, H, rc, lj=(s, e))["lj_energy"]) / (2 * h)
            assert abs(fd - r["lj_grad"][i, a]) < 1e-6 * max(1.0, abs(r["lj_grad"][i]).max())


@pytest.mark.parametrize("name", ["tric3", "skew3", "tric2"])
def test_virial_trace_is_minus_scaling_derivative(name):
    # scaling positions, box and cutoff by lam keeps the pair set; dE/dlam = -tr W
    H = BOXES[name]
    dim = H.shape[0]
    x = _lattice(H, 7 if dim == 3 else 18, 92)
    s, e, rc = 3.0, 0.238, 6.0
    r = oracle.compute(x, H, rc, lj=(s, e))
    h = 1e-7
    Ep = oracle.compute(x * (1 + h), H * (1 + h), rc * (1 + h), lj=(s, e))["lj_energy"]
    Em = oracle.compute(x * (1 - h), H * (1 - h), rc * (1 - h), lj=(s, e))["lj_energy"]
    fd = (Ep - Em) / (2 * h)
    assert abs(fd + np.trace(r["virial"])) < 1e-6 * abs(np.trace(r["virial"]))


@pytest.mark.parametrize("name", ["tric3", "tric2"])
def test_box_gradient_vs_finite_differences(name):
    H = BOXES[name]
    dim = H.shape[0]
    x = _lattice(H, 7 if dim == 3 else 18, 93) + (H @ np.array([2, -1, 3][:dim]))
    s, e, rc = 3.0, 0.238, 6.0
    r = oracle.compute(x, H, rc, lj=(s, e))
    h = 1e-7
    for a in range(dim):
        for b in range(dim):
            Hp = H.copy(); Hp[a, b] += h
            Hm = H.copy(); Hm[a, b] -= h
            fd = (oracle.compute(x, Hp, rc, lj=(s, e))["lj_energy"]
                  - oracle.compute(x, Hm, rc, lj=(s, e))["lj_energy"]) / (2 * h)
            assert abs(fd - r["dEdH"][a, b]) < 2e-6 * max(1.0, abs(r["dEdH"]).max())


# ---------------------------------------------------------------- invariances

def test_translation_by_lattice_vectors():
    c = W.config2(n=20_000)
    H, rc = c["H"], c["cutoff"]
    x = c["x"]
    far = x + H @ np.array([1000.0, -700.0, 300.0])
    a = oracle.compute(x, H, rc, lj=(3.4, 0.238), lj_grad=True, nl=True)
    b = oracle.compute(far, H, rc, lj=(3.4, 0.238), lj_grad=True, nl=True)
    assert a["count"] == b["count"]
    assert np.array_equal(a["nl_i"], b["nl_i"]) and np.array_equal(a["nl_j"], b["nl_j"])
    assert math.isclose(a["lj_energy"], b["lj_energy"], rel_tol=1e-9)
    scale = np.abs(a["lj_grad"]).max()
    assert np.abs(a["lj_grad"] - b["lj_grad"]).max() < 1e-8 * scale


def test_permutation_invariance():
    H = BOXES["skew3"]
    x = W.uniform_in_box(800, H, 94)
    perm = W.rng(95).permutation(len(x))
    a = oracle.compute(x, H, 5.0, lj=(3.0, 0.2), lj_grad=True, nl=True)
    b = oracle.compute(x[perm], H, 5.0, lj=(3.0, 0.2), lj_grad=True, nl=True)
    assert a["count"] == b["count"]
    pa = set(zip(a["nl_i"].tolist(), a["nl_j"].tolist()))
    pb = {tuple(sorted((int(perm[i]), int(perm[j])))) for i, j in zip(b["nl_i"], b["nl_j"])}
    assert pa == pb
    assert math.isclose(a["lj_energy"], b["lj_energy"], rel_tol=1e-12)
    assert np.allclose(a["lj_grad"][perm], b["lj_grad"], rtol=1e-11, atol=1e-11 * abs(a["lj_grad"]).max())


def test_relative_speed_histogram_two_velocity_groups():
    # group A moves with u, group B rests: A-B pairs have |dv| = |u|, others 0
    H = BOXES["tric3"]
    n = 1000
    x = W.uniform_in_box(n, H, 96)
    A = W.rng(97).random(n) < 0.4
    u = np.array([1.3, -0.4, 0.9])
    v = np.where(A[:, None], u[None, :], 0.0)
    rc, nb, hi = 5.0, 20, 4.0
    r = oracle.compute(x, H, rc, rel_hist=(nb, hi), vel_x=v)
    n_ab = r["count"] - oracle.compute(x[A], H, rc)["count"] - oracle.compute(x[~A], H, rc)["count"]
    k = int(math.ceil(np.linalg.norm(u) / (hi / nb))) - 1
    exp = np.zeros(nb + 1, dtype=np.uint64)
    exp[0] = r["count"] - n_ab
    exp[k] += n_ab
    assert np.array_equal(r["rel_hist"], exp)
    assert math.isclose(r["rel_sum"][k], n_ab * np.linalg.norm(u), rel_tol=1e-12)
    assert r["rel_sum"][0] == 0.0


def test_thread_count_does_not_change_results():
    H = BOXES["tric3"]
    x = W.uniform_in_box(3000, H, 98)
    kw = dict(lj=(3.4, 0.238), lj_grad=True, sum_inv_d=True)
    a = oracle.compute(x, H, 6.0, nthreads=1, **kw)
    b = oracle.compute(x, H, 6.0, nthreads=7, **kw)
    assert a["lj_energy"] == b["lj_energy"] and a["sum_inv_d"] == b["sum_inv_d"]
    assert np.array_equal(a["lj_grad"], b["lj_grad"])


# ---------------------------------------------------------------- frames (positions kept in an earlier wrap)
def _framed_case(seed=61):
    H = BOXES["tric3"]
    x = W.uniform_in_box(700, H, seed)
    g = W.rng(seed + 1)
    k = g.integers(-1, 2, size=x.shape)
    frame = oracle.wrap(x, H)[2] + k            # some particles one image away
    return H, x, frame


def test_frame_equal_to_the_canonical_wrap_is_the_canonical_computation():
    H, x, _ = _framed_case()
    rc = 4.0
    a = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, sum_d=True)
    b = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, sum_d=True,
                       frame=oracle.wrap(x, H)[2])
    assert a["count"] == b["count"]
    for key in ("nl_i", "nl_j", "nl_d", "lj_grad", "virial", "dEdH"):
        assert np.array_equal(a[key], b[key]), key
    assert a["lj_energy"] == b["lj_energy"] and a["sum_d"] == b["sum_d"]


def test_shifted_frame_gives_the_same_pairs_and_values_to_rounding():
    """Moving the frame by lattice vectors changes no real distance: the pair
    set is the same and every value agrees to rounding."""
    H, x, frame = _framed_case()
    rc = 4.0
    a = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True)
    b = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, frame=frame)
    assert a["count"] == b["count"] > 1000
    assert np.array_equal(a["nl_i"], b["nl_i"]) and np.array_equal(a["nl_j"], b["nl_j"])
    assert np.abs(a["nl_d"] - b["nl_d"]).max() <= 1e-13 * rc
    assert abs(a["lj_energy"] / b["lj_energy"] - 1) < 1e-12
    G = np.abs(a["lj_grad"]).max()
    assert np.abs(a["lj_grad"] - b["lj_grad"]).max() <= 1e-11 * G
    # dE/dH is taken at fixed Cartesian positions: the frame does not enter
    assert np.abs(a["dEdH"] - b["dEdH"]).max() <= 1e-11 * np.abs(a["dEdH"]).max()


def test_framed_brute_force_and_cell_loops_agree_exactly():
    """The cell loop derives each pair's frame image from its cell image; the
    brute-force loop searches the images of the frame positions directly."""
    H, x, frame = _framed_case(63)
    rc = 4.0
    a = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, frame=frame,
                       method=oracle.METHOD_BRUTE)
    b = oracle.compute(x, H, rc, nl=True, lj=(1.0, 0.5), lj_grad=True, frame=frame,
                       method=oracle.METHOD_CELLS)
    assert a["method"] == oracle.METHOD_BRUTE and b["method"] == oracle.METHOD_CELLS
    assert a["count"] == b["count"]
    for key in ("nl_i", "nl_j", "nl_d"):
        assert np.array_equal(a[key], b[key]), key
    assert abs(a["lj_energy"] / b["lj_energy"] - 1) < 1e-13
    assert np.abs(a["lj_grad"] - b["lj_grad"]).max() <= 1e-12 * np.abs(a["lj_grad"]).max()


# ---------------------------------------------------------------- velocity Verlet
def _lj_gas(n=216, density=0.5, seed=64, T=1.0):
    """Reduced LJ units: a jittered simple-cubic start at the given density."""
    m = round(n ** (1 / 3))
    side = (n / density) ** (1 / 3)
    g = W.rng(seed)
    grid = np.stack(np.meshgrid(*([np.arange(m)] * 3), indexing="ij"), -1).reshape(-1, 3)
    x = (grid + 0.5 + 0.1 * (g.random(grid.shape) - 0.5)) * (side / m)
    v = g.normal(0.0, math.sqrt(T), size=x.shape)
    v -= v.mean(0)
    return x, v, np.diag([side] * 3)


def test_md_free_flight_is_uniform_motion():
    H = np.diag([50.0, 50.0, 50.0])
    x = np.array([[5.0, 5.0, 5.0], [30.0, 30.0, 30.0]])
    v = np.array([[0.3, -0.2, 0.1], [-0.1, 0.05, 0.2]])
    r = oracle.md_run(x, v, H, 2.5, 1.0, 1.0, 1.0, 0.01, 200)
    assert np.all(r["count"] == 0)
    assert np.abs(r["x"] - (x + 200 * 0.01 * v)).max() < 1e-12
    assert np.array_equal(r["v"], v)


def test_md_dimer_oscillates_with_the_harmonic_period():
    """Small oscillation of an LJ dimer about r_min = 2^(1/6) sigma: the
    curvature there is 72 eps / r_min^2, so T = 2 pi sqrt(mu / k) with
    mu = m / 2."""
    sigma, eps, mass, dt = 1.0, 1.0, 1.0, 0.001
    rmin = 2 ** (1 / 6) * sigma
    H = np.diag([20.0, 20.0, 20.0])
    x = np.array([[10.0, 10.0, 10.0], [10.0 + rmin + 0.002, 10.0, 10.0]])
    v = np.zeros_like(x)
    T_exact = 2 * math.pi * math.sqrt((mass / 2) / (72 * eps / rmin ** 2))
    nsteps = int(2.2 * T_exact / dt)
    xs = [x[1, 0] - x[0, 0]]
    xx, vv = x, v
    for _ in range(nsteps):  # one step at a time to record r(t)
        r = oracle.md_run(xx, vv, H, 3.0, sigma, eps, mass, dt, 1)
        xx, vv = r["x"], r["v"]
        xs.append(xx[1, 0] - xx[0, 0])
    y = np.array(xs) - rmin
    # downward zero crossings of r - r_min, linearly interpolated
    idx = np.where((y[:-1] > 0) & (y[1:] <= 0))[0]
    t = (idx + y[idx] / (y[idx] - y[idx + 1])) * dt
    assert len(t) >= 2
    assert abs((t[1] - t[0]) / T_exact - 1) < 2e-4
    # momentum stays zero (the pair forces are equal and opposite)
    assert np.abs(vv.sum(0)).max() < 1e-13


def test_md_is_time_reversible():
    x, v, H = _lj_gas(n=125, density=0.3)
    a = oracle.md_run(x, v, H, 2.5, 1.0, 1.0, 1.0, 0.002, 100)
    b = oracle.md_run(a["x"], -a["v"], H, 2.5, 1.0, 1.0, 1.0, 0.002, 100)
    assert np.abs(b["x"] - x).max() < 1e-8
    assert np.abs(b["v"] + v).max() < 1e-8


def test_md_energy_error_is_second_order_and_momentum_is_kept():
    """A 27-atom cluster whose every pair stays inside the cutoff (so the
    truncated potential never jumps): velocity Verlet keeps the total energy
    with an error of order dt^2."""
    g = W.rng(65)
    grid = np.stack(np.meshgrid(*([np.arange(3)] * 3), indexing="ij"), -1).reshape(-1, 3)
    x = 20.0 + 1.12 * grid + 0.05 * (g.random(grid.shape) - 0.5)
    v = g.normal(0.0, 0.3, size=x.shape)
    v -= v.mean(0)
    H = np.diag([40.0, 40.0, 40.0])
    errs = []
    for dt, steps in ((0.004, 250), (0.002, 500)):
        r = oracle.md_run(x, v, H, 12.0, 1.0, 1.0, 1.0, dt, steps)
        assert np.all(r["count"] == 27 * 26 // 2)
        E = r["energy"] + r["ke"]
        errs.append(np.abs(E - E[0]).max())
        p = r["v"].sum(0)
        assert np.abs(p).max() < 1e-12 * np.abs(r["v"]).sum()
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_md_rescaling_sets_the_kinetic_energy():
    x, v, H = _lj_gas(n=64, density=0.4)
    target = 100.0
    r = oracle.md_run(x, v, H, 2.5, 1.0, 1.0, 1.0, 0.002, 5, rescale_every=5, target_ke=target)
    ke = 0.5 * np.sum(np.sum(r["v"] * r["v"], axis=1))
    assert abs(ke / target - 1) < 1e-12
    assert abs(r["ke"][-1] / target - 1) > 1e-3   # recorded before the rescale


def test_md_with_a_skin_follows_the_same_trajectory():
    """Distances taken in the frame of the last rebuild are the same real
    distances: pair counts agree exactly and the trajectories to rounding."""
    x, v, H = _lj_gas(n=216, density=0.6, T=2.0)
    a = oracle.md_run(x, v, H, 2.5, 1.0, 1.0, 1.0, 0.004, 60)
    b = oracle.md_run(x, v, H, 2.5, 1.0, 1.0, 1.0, 0.004, 60, skin=0.3)
    assert np.array_equal(a["count"], b["count"])
    assert 1 < int(b["rebuilt"].sum()) < 60
    assert np.abs(a["x"] - b["x"]).max() < 1e-10
    assert np.abs(a["energy"] / b["energy"] - 1).max() < 1e-11


# ---------------------------------------------------------------- k closest pairs (Code 8)
def test_kclosest_code8_shape_against_exhaustive_enumeration():
    """Code 8's case: 100 and 1000 uniform points in a unit box, cutoff 0.1,
    the 5 closest cross pairs; every pair enumerated with all 27 images."""
    x, y = W.rng(81).random((100, 3)), W.rng(82).random((1000, 3))
    H = np.eye(3)
    i, j, d2 = oracle.kclosest(x, H, 0.1, 5, y=y)
    Ks = np.stack(np.meshgrid(*([np.arange(-1, 2)] * 3), indexing="ij"), -1).reshape(-1, 3).astype(float)
    D = (y[None, :, None, :] - x[:, None, None, :]) + Ks[None, None, :, :]
    e2 = ((D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]).min(axis=2)
    ii, jj = np.nonzero(e2 <= 0.1 * 0.1)
    order = np.lexsort((jj, ii, e2[ii, jj]))[:5]
    assert np.array_equal(i, ii[order]) and np.array_equal(j, jj[order])
    assert np.array_equal(d2, e2[ii[order], jj[order]])


def test_kclosest_ties_go_by_index_and_short_lists():
    """Equal squared distances are ordered by (i, j); with fewer than k pairs
    in the cutoff every pair is returned."""
    H = np.diag([8.0, 8.0, 8.0])
    x = np.array([[4.0, 4.0, 4.0], [1.0, 1.0, 1.0]])
    off = 0.125 * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    y = np.vstack([x[0] + off, [[4.0, 4.0, 4.0 + 0.0625]], x[1] + 2 * off[:2]])
    i, j, d2 = oracle.kclosest(x, H, 0.3, 4, y=y)
    assert list(zip(i, j)) == [(0, 6), (0, 0), (0, 1), (0, 2)]
    assert list(d2) == [0.0625 ** 2, 0.015625, 0.015625, 0.015625]
    i, j, d2 = oracle.kclosest(x, H, 0.3, 100, y=y)
    assert len(i) == 9 and list(zip(i[-2:], j[-2:])) == [(1, 7), (1, 8)]
    # single set: unordered pairs i < j
    i, j, d2 = oracle.kclosest(y, H, 0.13, 3)
    assert np.all(i < j) and np.all(np.diff(d2) >= 0)


# ---------------------------------------------------------------- non-periodic neighbour list (section 4.1)
@pytest.mark.parametrize("offset", [0.0, -37.5, 1000.0])
def test_nonperiodic_list_is_the_euclidean_pair_set(offset):
    """Two disjoint sets at water-like density (100 per nm^3, cutoff 1.2 nm):
    the bounding-box computation equals a plain Euclidean enumeration with
    no images, wherever the cloud sits."""
    g = W.rng(91)
    y = offset + 2.5 * g.random((2500, 3))          # 100 per nm^3 in a 2.5 nm cube
    x = offset + 0.6 + 1.3 * g.random((220, 3))     # a smaller set inside it
    r = oracle.neighbor_list_nonperiodic(x, 1.2, y=y)
    D = y[None, :, :] - x[:, None, :]
    e2 = (D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2]
    ii, jj = np.nonzero(e2 <= 1.2 * 1.2)
    assert r["count"] == len(ii) > 10000
    assert np.array_equal(r["nl_i"], ii) and np.array_equal(r["nl_j"], jj)
    assert np.abs(r["nl_d2"] - e2[ii, jj]).max() <= 1e-13 * (1.0 + abs(offset))
    # single set: i < j, the same on the Euclidean side
    r1 = oracle.neighbor_list_nonperiodic(x, 1.2)
    D1 = x[None, :, :] - x[:, None, :]
    f2 = (D1[..., 0] * D1[..., 0] + D1[..., 1] * D1[..., 1]) + D1[..., 2] * D1[..., 2]
    a, b = np.nonzero(np.triu(f2 <= 1.2 * 1.2, k=1))
    assert np.array_equal(r1["nl_i"], a) and np.array_equal(r1["nl_j"], b)


def test_nonperiodic_box_sides():
    x = np.array([[0.0, -1.0, 2.0], [3.0, 4.0, 2.5]])
    H = oracle.nonperiodic_box(x, 1.0)
    assert np.allclose(np.diag(H), [3.0 + 1.000001, 5.0 + 1.000001, 0.5 + 1.000001], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- weighted maps (Code 5 masses, Code 10)
def test_weighted_inverse_distance_sum():
    """Code 5's second example, sum of m_i m_j / d: unit weights give the sum
    of 1/d bit for bit, a constant weight c gives c^2 times it, and a small
    case matches an exhaustive enumeration over the 27 images."""
    H = BOXES["tric3"]
    x = W.uniform_in_box(1500, H, 95)
    rc = 4.0
    r1 = oracle.compute(x, H, rc, sum_inv_d=True, weights=(np.ones(len(x)), None))
    assert r1["sum_w_inv_d"] == r1["sum_inv_d"]
    r3 = oracle.compute(x, H, rc, weights=(np.full(len(x), 3.0), None))
    assert abs(r3["sum_w_inv_d"] / (9.0 * r1["sum_inv_d"]) - 1) < 1e-14
    # exhaustive, cross set in an orthorhombic box
    Ho = BOXES["ortho3"]
    xa, ya = W.uniform_in_box(60, Ho, 96), W.uniform_in_box(300, Ho, 97)
    wa, wb = W.rng(98).random(60), W.rng(99).random(300)
    r = oracle.compute(xa, Ho, 6.0, ya, weights=(wa, wb))
    s = 0.0
    for i in range(60):
        for j in range(300):
            d2 = exhaustive_d2(xa[i], ya[j], Ho, kmax=1)
            if d2 <= 36.0:
                s += wa[i] * wb[j] / math.sqrt(d2)
    assert abs(r["sum_w_inv_d"] / s - 1) < 1e-12


def test_distance_binned_relative_speed():
    """Code 10: pairs binned by distance with |v_j - v_i| summed per bin.  The
    counts are the plain distance histogram's; the sums match an exhaustive
    enumeration; equal velocities give zero sums."""
    H = BOXES["cube3"]
    x = W.uniform_in_box(500, H, 100)
    v = W.rng(101).normal(size=x.shape)
    rc = 5.0
    r = oracle.compute(x, H, rc, hist=(10, rc), dist_vel_hist=(10, rc), vel_x=v)
    assert np.array_equal(r["dv_hist"], r["hist"])
    sums = np.zeros(10)
    h = rc / 10
    for i in range(len(x)):
        for j in range(i + 1, len(x)):
            d2 = exhaustive_d2(x[i], x[j], H, kmax=1)
            if d2 <= rc * rc:
                b = min(int(math.ceil(math.sqrt(d2) / h)) - 1, 9) if d2 > 0 else 0
                sums[b] += np.linalg.norm(v[j] - v[i])
    assert np.allclose(r["dv_sum"], sums, rtol=1e-12, atol=0)
    r0 = oracle.compute(x, H, rc, dist_vel_hist=(10, rc), vel_x=np.ones_like(x))
    assert np.all(r0["dv_sum"] == 0.0)


# ---------------------------------------------------------------- per-particle LJ and neighbours of one particle

def _numpy_min_images(x, i, H):
    """For every j: the image K (raw coordinates) minimising |x_j - x_i + H K|
    and that squared distance, by an exhaustive numpy search of K0 + {-2..2}^dim
    around K0 = -round(H^-1 (x_j - x_i)) (independent of the oracle's search)."""
    dim = H.shape[0]
    Hi = np.linalg.inv(H)
    dr = x - x[i]
    K0 = -np.rint(dr @ Hi.T)
    rng = np.arange(-2, 3)
    off = np.stack(np.meshgrid(*([rng] * dim), indexing="ij"), -1).reshape(-1, dim)
    Ks = K0[:, None, :] + off[None, :, :]                      # (n, 5^dim, dim)
    D = dr[:, None, :] + Ks @ H.T
    d2 = (D * D).sum(-1)
    k = d2.argmin(1)
    return d2[np.arange(len(x)), k], Ks[np.arange(len(x)), k].astype(np.int64)


def _lj_pair(d2, s, e):
    """u(d) = 4 eps (x^6 - x^3), x = s^2/d^2 (paper Code 6), and
    f_s = 24 eps (2 x^6 - x^3) / d^2, the factor of D in dE/dr_i."""
    x = s * s / d2
    x3 = x ** 3
    return 4 * e * (x3 * x3 - x3), 24 * e * (2 * x3 * x3 - x3) / d2


SAMPLE_CASES = [("tric3", 500, 6.5, 0.0), ("skew3", 500, 6.0, 0.0), ("tric2", 400, 7.0, 0.0),
                ("tric3", 500, 6.5, 1.0)]


@pytest.mark.parametrize("name,n,rc,far", SAMPLE_CASES)
def test_lj_sample_against_numpy_enumeration_and_compute(name, n, rc, far):
    """E_i and dE/dr_i of lj_sample (Code 6 energy, its exact gradient) against
    (a) a numpy enumeration of each sampled particle's pairs with the
    exhaustively searched nearest image, (b) the gradient rows of compute()
    for the same particles, and (c) sum_i E_i = 2E over all particles."""
    H = BOXES[name]
    dim = H.shape[0]
    s, e = 3.0, 0.238
    x = _lattice(H, 8 if dim == 3 else 20, 171 + n)[:n]
    if far:  # far from the origin: raw coordinates many boxes away
        x = x + np.array([1000, -700, 300][:dim]) @ H.T
    full = oracle.compute(x, H, rc, lj=(s, e), lj_grad=True)
    sample = np.array([0, 7, 101, n // 2, n - 1])
    Ei, Gi = oracle.lj_sample(x, H, rc, sample, s, e)
    for k, i in enumerate(sample):
        d2, K = _numpy_min_images(x, i, H)
        m = (d2 <= rc * rc) & (np.arange(n) != i)
        D = (x[m] - x[i]) + K[m] @ H.T
        u, fs = _lj_pair((D * D).sum(1), s, e)
        assert math.isclose(Ei[k], u.sum(), rel_tol=1e-11, abs_tol=1e-12)
        gref = (fs[:, None] * D).sum(0)
        scale = np.abs(fs[:, None] * D).sum()
        assert np.abs(Gi[k] - gref).max() <= 1e-11 * scale
        assert np.abs(Gi[k] - full["lj_grad"][i]).max() <= 1e-12 * scale
    Eall, _ = oracle.lj_sample(x, H, rc, np.arange(n), s, e)
    assert math.isclose(Eall.sum(), 2 * full["lj_energy"], rel_tol=1e-12)


def test_lj_sample_sign_against_a_two_particle_closed_form():
    """Two particles on the x axis at distance d: E_0 = u(d) and dE/dr_0 =
    -u'(d) e_x (pulling 0 towards 1 lowers E beyond the minimum)."""
    H = np.diag([30.0, 30.0, 30.0])
    s, e = 3.4, 0.238
    for d in (3.2, 3.4 * 2 ** (1 / 6), 5.0):
        x = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]])
        E, G = oracle.lj_sample(x, H, 8.0, np.array([0, 1]), s, e)
        u = 4 * e * ((s / d) ** 12 - (s / d) ** 6)
        du = 4 * e * (-12 * s ** 12 / d ** 13 + 6 * s ** 6 / d ** 7)
        assert math.isclose(E[0], u, rel_tol=1e-13, abs_tol=1e-15)
        assert math.isclose(G[0, 0], -du, rel_tol=1e-12, abs_tol=1e-14)
        assert math.isclose(G[1, 0], du, rel_tol=1e-12, abs_tol=1e-14)
        assert np.abs(G[:, 1:]).max() == 0.0


@pytest.mark.parametrize("name,n,rc,far", SAMPLE_CASES)
def test_neighbors_of_against_numpy_enumeration_and_the_list(name, n, rc, far):
    """neighbors_of(i): the j with nearest-image distance <= rc and the raw
    image K with x_j - x_i + H K the nearest displacement; against a numpy
    exhaustive search (set and K exactly) and against the neighbour list of
    compute() (the pairs containing i, and their distances to rounding)."""
    H = BOXES[name]
    dim = H.shape[0]
    x = W.uniform_in_box(n, H, 181 + n)
    # every particle displaced by its own lattice vector (different wrap
    # integers per particle), and far from the origin for `far`
    x = x + W.rng(191 + n).integers(-3, 4, size=(n, dim)) @ H.T
    if far:
        x = x + np.array([1000, -700, 300][:dim]) @ H.T
    nl = oracle.compute(x, H, rc, nl=True)
    pairs_i, pairs_j, pairs_d = nl["nl_i"], nl["nl_j"], nl["nl_d"]
    for i in (0, 3, n // 3, n - 1):
        js, Ks = oracle.neighbors_of(x, H, rc, i)
        d2, Kref = _numpy_min_images(x, i, H)
        # pairs within 1e-9 rc^2 of the cutoff would be decided by rounding
        assert not np.any((np.abs(d2 - rc * rc) < 1e-9 * rc * rc) & (np.arange(n) != i))
        want = np.nonzero((d2 <= rc * rc) & (np.arange(n) != i))[0]
        assert np.array_equal(np.sort(js), want)
        order = np.argsort(js)
        assert np.array_equal(Ks[order], Kref[want])
        # the list's pairs containing i, with i's partner and distance
        sel = (pairs_i == i) | (pairs_j == i)
        other = np.where(pairs_i[sel] == i, pairs_j[sel], pairs_i[sel])
        assert np.array_equal(np.sort(other), want)
        D = (x[js] - x[i]) + Ks @ H.T
        dd = np.sqrt((D * D).sum(1))
        ref_d = dict(zip(other.tolist(), pairs_d[sel].tolist()))
        for j, dj in zip(js.tolist(), dd.tolist()):
            assert math.isclose(dj, ref_d[j], rel_tol=1e-9, abs_tol=1e-9 * (1 + 1e3 * far))


@pytest.mark.parametrize("name,n,rc,far", SAMPLE_CASES)
def test_per_particle_force_magnitude_sum_against_numpy(name, n, rc, far):
    """lj_fabs: per particle the sum over its pairs of |f_s| d (the scale of
    the per-particle force error), against a numpy enumeration, in both the
    cell-list and the brute-force loop."""
    H = BOXES[name]
    dim = H.shape[0]
    s, e = 3.0, 0.238
    x = _lattice(H, 8 if dim == 3 else 20, 271 + n)[:n]
    if far:
        x = x + np.array([1000, -700, 300][:dim]) @ H.T
    for method in (oracle.METHOD_CELLS, oracle.METHOD_BRUTE):
        r = oracle.compute(x, H, rc, lj=(s, e), lj_grad=True, lj_fabs=True, method=method)
        for i in (0, 5, n // 2, n - 1):
            d2, K = _numpy_min_images(x, i, H)
            m = (d2 <= rc * rc) & (np.arange(n) != i)
            _, fs = _lj_pair(d2[m], s, e)
            ref = (np.abs(fs) * np.sqrt(d2[m])).sum()
            assert math.isclose(r["lj_fabs"][i], ref, rel_tol=1e-11)
        # never below the magnitude of the net force
        assert np.all(r["lj_fabs"] >= np.linalg.norm(r["lj_grad"], axis=1) * (1 - 1e-12))
