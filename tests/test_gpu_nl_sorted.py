"""Neighbour lists in canonical order (ascending i, then j) sorted on the
device, and the synchronous capacity check, through the C-ABI.

The pair set of section 4.1's neighbour list is compared with the oracle's
bit for bit, in the oracle's own (i, j) order, so the device order must be
exactly the lexicographic one; FP64 distances are the canonical sqrt and
must match bit for bit too."""
import ctypes

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


def _check_sorted(pairs, dist, ref, exact_d):
    p = pairs.cpu().numpy().astype(np.int64)
    assert len(p) == ref["count"]
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    if dist is not None:
        d = dist.cpu().numpy()
        if exact_d:
            assert np.array_equal(d, ref["nl_d"])
        else:
            assert np.abs(d - ref["nl_d"]).max() <= 2e-6 * ref["nl_d"].max()


CASES = {
    "tric3": (W.triclinic_h((32.0, 30.0, 31.0), (80.0, 95.0, 100.0)), 6000, 4.0),
    "ortho3": (np.diag([28.0, 34.0, 31.0]), 5000, 4.5),
    "tric2": (np.array([[55.0, -12.0], [0.0, 50.0]]), 4000, 3.2),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lcell", [1, 2])
def test_sorted_neighbor_list_single_set(clm, name, precision, lcell):
    H, n, rc = CASES[name]
    x = W.uniform_in_box(n, H, 700 + n)
    ref = oracle.compute(x, H, rc, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, lcell), precision=precision)
    print(f"case {name} {precision} lcell={lcell}", flush=True)
    pairs, dist = cl.neighbor_list(sorted=True)
    _check_sorted(pairs, dist, ref, precision == "fp64")
    pairs, dist = cl.neighbor_list(sorted=True, distances=False)
    _check_sorted(pairs, None, ref, True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sorted_neighbor_list_cross_set_and_small_box(clm, precision):
    H = np.diag([40.0, 40.0, 40.0])
    x = np.mod(W.rng(1).normal(20.0, 4.0, size=(700, 3)), 40.0)
    y = W.uniform_in_box(20000, H, 2)
    ref = oracle.compute(x, H, 3.0, y, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, 3.0, 1), y=T(y), precision=precision)
    pairs, dist = cl.neighbor_list(sorted=True)
    _check_sorted(pairs, dist, ref, precision == "fp64")
    Hs = W.triclinic_h((10.0, 11.0, 10.5), (85.0, 95.0, 100.0))
    xs = W.uniform_in_box(300, Hs, 51)
    ref = oracle.compute(xs, Hs, 7.0, nl=True)
    box = clm.Box(Hs, 7.0, 1)
    assert box.info()["small_box"]
    cl = clm.CellList(T(xs), box, precision=precision)
    pairs, dist = cl.neighbor_list(sorted=True)
    _check_sorted(pairs, dist, ref, True)


def _sort_call(clm, pairs, dist, count, n_i, n_j, capacity):
    L = clm._lib
    need = ctypes.c_size_t(0)
    L.check(L.lib().clm_pairs_sort_workspace_bytes(capacity, int(dist is not None), ctypes.byref(need)))
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device="cuda:0")
    pad = (-ws.data_ptr()) % 256
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    L.check(L.lib().clm_pairs_sort(clm._context(torch.device("cuda:0")), n_i, n_j, ptr(pairs), ptr(dist),
                                   ptr(count), capacity, ctypes.c_void_p(ws.data_ptr() + pad),
                                   int(need.value)))
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,n_i,n_j", [(0, 10, 10), (1, 1, 1), (2047, 5000, 5000), (2049, 300, 70000),
                                      (100_003, 2**31, 2**31), (300_000, 2**20, 3)])
def test_pairs_sort_random_unique_keys(clm, m, n_i, n_j):
    """Random distinct (i, j) in random order, index ranges from 1 to 2^31
    (1 to 8 radix passes), distances carried along."""
    g = W.rng(m + n_j)
    keys = np.unique(g.integers(0, n_i * n_j, size=int(1.3 * m) + 4, dtype=np.int64))
    keys = g.permutation(keys)[:m]
    m = len(keys)
    ij = np.stack([keys // n_j, keys % n_j], 1).astype(np.int32)
    d = g.random(m)
    cap = m + 5
    pairs = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda:0")
    pairs[:m] = T(ij)
    dist = torch.full((cap,), -1.0, dtype=torch.float64, device="cuda:0")
    dist[:m] = T(d)
    count = torch.tensor([m], dtype=torch.int64, device="cuda:0")
    print(f"case m={m} n_i={n_i} n_j={n_j}", flush=True)
    _sort_call(clm, pairs, dist, count, n_i, n_j, cap)
    order = np.lexsort((ij[:, 1], ij[:, 0]))
    assert np.array_equal(pairs[:m].cpu().numpy(), ij[order])
    assert np.array_equal(dist[:m].cpu().numpy(), d[order])
    assert (pairs[m:].cpu().numpy() == -7).all() and (dist[m:].cpu().numpy() == -1.0).all()


def test_pairs_sort_overflowed_list_sorts_the_written_part(clm):
    """count > capacity (an overflowed list): the capacity pairs that were
    written are sorted, nothing past them is touched."""
    g = W.rng(5)
    m, cap = 5000, 3000
    ij = np.stack([g.permutation(m), g.integers(0, 9000, size=m)], 1).astype(np.int32)
    pairs = torch.full((cap + 8, 2), -3, dtype=torch.int32, device="cuda:0")
    pairs[:cap] = T(ij[:cap])
    count = torch.tensor([m], dtype=torch.int64, device="cuda:0")
    _sort_call(clm, pairs, None, count, m, 9000, cap)
    w = ij[:cap]
    assert np.array_equal(pairs[:cap].cpu().numpy(), w[np.lexsort((w[:, 1], w[:, 0]))])
    assert (pairs[cap:].cpu().numpy() == -3).all()


def test_capacity_check_returns_capacity_error_with_the_true_count(clm):
    L = clm._lib
    H, n, rc = CASES["tric3"]
    x = W.uniform_in_box(n, H, 77)
    ref = oracle.compute(x, H, rc, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision="fp32")
    cap = ref["count"] // 3
    pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda:0")
    c = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    P = L.MapParams(capacity=cap, check_capacity=1)
    O = L.MapOut(pairs_dev=ctypes.c_void_p(pairs.data_ptr()), count_dev=ctypes.c_void_p(c.data_ptr()))
    st = L.lib().clm_map(cl._h, L.MAP_KINDS["neighbor_list"], ctypes.byref(P), ctypes.byref(O))
    assert st == L.STATUS_CODES["CLM_E_CAPACITY"]
    assert int(c.item()) == ref["count"]
    P.capacity = ref["count"]
    pairs = torch.empty((ref["count"], 2), dtype=torch.int32, device="cuda:0")
    O.pairs_dev = ctypes.c_void_p(pairs.data_ptr())
    assert L.lib().clm_map(cl._h, L.MAP_KINDS["neighbor_list"], ctypes.byref(P), ctypes.byref(O)) == 0
    # the Python list grows from a too-small capacity through the same error
    p2, _ = cl.neighbor_list(capacity=10, sorted=True)
    _check_sorted(p2, None, ref, True)


def test_sorted_lists_in_a_batch(clm):
    L = clm._lib
    jobs = []
    for k, (name, lcell) in enumerate([("tric3", 2), ("ortho3", 1), ("tric3", 1)]):
        H, n, rc = CASES[name]
        x = W.uniform_in_box(n - 500 * k, H, 900 + k)
        jobs.append((x, H, rc, clm.CellList(T(x), clm.Box(H, rc, lcell), precision="fp32")))
    nj = len(jobs)
    cls = (ctypes.c_void_p * nj)(*[j[3]._h for j in jobs])
    Ps = (L.MapParams * nj)()
    Os = (L.MapOut * nj)()
    keep = []
    for k, (x, H, rc, cl) in enumerate(jobs):
        cap = 40 * len(x)
        pairs = torch.empty((cap, 2), dtype=torch.int32, device="cuda:0")
        dist = torch.empty(cap, dtype=torch.float64, device="cuda:0")
        c = torch.empty(1, dtype=torch.int64, device="cuda:0")
        need = ctypes.c_size_t(0)
        L.check(L.lib().clm_pairs_sort_workspace_bytes(cap, 1, ctypes.byref(need)))
        ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device="cuda:0")
        Ps[k] = L.MapParams(capacity=cap, with_distances=1, sorted=1, check_capacity=1,
                            scratch_dev=ctypes.c_void_p(ws.data_ptr() + (-ws.data_ptr()) % 256),
                            scratch_bytes=int(need.value))
        Os[k] = L.MapOut(pairs_dev=ctypes.c_void_p(pairs.data_ptr()), dist_dev=ctypes.c_void_p(dist.data_ptr()),
                         count_dev=ctypes.c_void_p(c.data_ptr()))
        keep.append((pairs, dist, c, ws))
    need = ctypes.c_size_t(0)
    L.check(L.lib().clm_map_batch_workspace_bytes(nj, cls, ctypes.byref(need)))
    bw = torch.empty(int(need.value) + 256, dtype=torch.uint8, device="cuda:0")
    L.check(L.lib().clm_map_batch(nj, cls, L.MAP_KINDS["neighbor_list"], Ps, Os,
                                  ctypes.c_void_p(bw.data_ptr() + (-bw.data_ptr()) % 256), int(need.value)))
    torch.cuda.synchronize()
    for (x, H, rc, cl), (pairs, dist, c, ws) in zip(jobs, keep):
        ref = oracle.compute(x, H, rc, nl=True)
        m = int(c.item())
        _check_sorted(pairs[:m], dist[:m], ref, False)


def test_sorted_needs_a_scratch(clm):
    L = clm._lib
    H, n, rc = CASES["ortho3"]
    x = W.uniform_in_box(n, H, 5)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision="fp64")
    pairs = torch.empty((1000, 2), dtype=torch.int32, device="cuda:0")
    c = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    P = L.MapParams(capacity=1000, sorted=1)
    O = L.MapOut(pairs_dev=ctypes.c_void_p(pairs.data_ptr()), count_dev=ctypes.c_void_p(c.data_ptr()))
    st = L.lib().clm_map(cl._h, L.MAP_KINDS["neighbor_list"], ctypes.byref(P), ctypes.byref(O))
    assert st == L.STATUS_CODES["CLM_E_WORKSPACE"]
    torch.cuda.synchronize()
    assert int(c.item()) == -1, "nothing was launched"
