"""GPU parity of the weighted maps against the CPU oracle: the sum of
w_i w_j / d (paper Code 5, masses) and the distance histogram with per-bin
sums of |v_j - v_i| (Code 10).  Pair counts and histogram counts bit-exact;
sums within 1e-12 (FP64 form) and 1e-6 (FP32+guard form) relative."""
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


CASES = {
    "cube3": (np.diag([30.0, 30.0, 30.0]), 4000, 5.0),
    "tric3": (W.triclinic_h((32.0, 30.0, 31.0), (80.0, 95.0, 100.0)), 6000, 4.0),
    "sq2": (np.diag([60.0, 60.0]), 5000, 3.0),
    "tric2": (np.array([[55.0, -12.0], [0.0, 50.0]]), 4000, 3.2),
    "small3": (W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0)), 400, 6.0),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weighted_inverse_distance(clm, name, precision):
    H, n, rc = CASES[name]
    x = W.uniform_in_box(n, H, 500 + n)
    w = 0.5 + 1.5 * W.rng(501).random(n)
    ref = oracle.compute(x, H, rc, sum_inv_d=True, weights=(w, None))
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    assert cl.box.info()["small_box"] == (name == "small3")
    s, c = cl.sum_w_inv_d(T(w))
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert int(c.item()) == ref["count"]
    assert abs(s.item() / ref["sum_w_inv_d"] - 1) < tol
    # unit weights give the plain sum of 1/d
    s1, _ = cl.sum_w_inv_d(torch.ones(n, dtype=torch.float64, device="cuda:0"))
    s0, _ = cl.sum_inv_d()
    assert abs(s1.item() / s0.item() - 1) < 1e-15
    # a smaller map cutoff
    ref2 = oracle.compute(x, H, 0.7 * rc, weights=(w, None))
    s2, c2 = cl.sum_w_inv_d(T(w), cutoff=0.7 * rc)
    assert int(c2.item()) == ref2["count"] and abs(s2.item() / ref2["sum_w_inv_d"] - 1) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_weighted_inverse_distance_cross(clm, precision):
    H = np.diag([40.0, 40.0, 40.0])
    x = np.mod(W.rng(502).normal(20.0, 4.0, size=(700, 3)), 40.0)
    y = W.uniform_in_box(20000, H, 503)
    wx, wy = W.rng(504).random(700), W.rng(505).random(20000)
    ref = oracle.compute(x, H, 3.0, y, weights=(wx, wy))
    cl = clm.CellList(T(x), clm.Box(H, 3.0, 1), y=T(y), precision=precision)
    s, c = cl.sum_w_inv_d(T(wx), T(wy))
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert int(c.item()) == ref["count"] and abs(s.item() / ref["sum_w_inv_d"] - 1) < tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_distance_binned_relative_speed(clm, name, precision):
    H, n, rc = CASES[name]
    dim = H.shape[0]
    x = W.uniform_in_box(n, H, 600 + n)
    v = W.rng(601).normal(size=(n, dim))
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for nb, hi in [(10, rc), (37, 0.8 * rc)]:
        ref = oracle.compute(x, H, rc, dist_vel_hist=(nb, hi), vel_x=v)
        h, sums, c = cl.dist_vel_histogram(T(v), nb, hi)
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["dv_hist"]), (nb, hi)
        assert int(c.item()) == ref["count"]
        rs = ref["dv_sum"]
        assert np.all(np.abs(sums.cpu().numpy() - rs) <= tol * np.abs(rs) + 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_distance_binned_relative_speed_cross(clm, precision):
    H = np.diag([40.0, 40.0, 40.0])
    x = np.mod(W.rng(602).normal(20.0, 4.0, size=(700, 3)), 40.0)
    y = W.uniform_in_box(20000, H, 603)
    vx, vy = W.rng(604).normal(size=(700, 3)), W.rng(605).normal(size=(20000, 3))
    ref = oracle.compute(x, H, 3.0, y, dist_vel_hist=(12, 3.0), vel_x=vx, vel_y=vy)
    cl = clm.CellList(T(x), clm.Box(H, 3.0, 1), y=T(y), precision=precision)
    h, sums, c = cl.dist_vel_histogram(T(vx), 12, 3.0, vy=T(vy))
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["dv_hist"])
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert np.all(np.abs(sums.cpu().numpy() - ref["dv_sum"]) <= tol * np.abs(ref["dv_sum"]))
