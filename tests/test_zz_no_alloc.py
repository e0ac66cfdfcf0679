"""clm_map_static (no allocation, no workspace argument) against the
workspace path clm_celllist_create + clm_celllist_build + clm_map, called
through the C-ABI: two calls in a row on each map kind, the second with a
smaller input.  Each build sorts the particles of a cell in the order of
their atomic ranks, so the order of FP64 summation (and of the neighbour
list) may differ between two builds: integers are compared exactly (pair
sets sorted), floating-point results within the parity tolerances (FP64
form 1e-12 relative for sums and energies, 1e-11 per-particle force error
relative to the sum of the pair-force magnitudes; FP32+guard form 1e-6 and
1e-5), each path against the oracle and the two paths against each other.
Also: the capacity error for an input beyond the static scratch."""
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


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _outputs(kind, n, dim, cap, nbins):
    dev = "cuda:0"
    o = {"count": torch.full((1,), -1, dtype=torch.int64, device=dev)}
    if kind in ("lj_ef", "sum_inv_d"):
        o["energy"] = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    if kind == "lj_ef":
        o["forces"] = torch.full((n, dim), np.nan, dtype=torch.float64, device=dev)
        o["grad_box"] = torch.full((dim, dim), np.nan, dtype=torch.float64, device=dev)
        o["virial"] = torch.full((dim, dim), np.nan, dtype=torch.float64, device=dev)
    if kind == "hist_dist":
        o["hist"] = torch.full((nbins + 1,), -1, dtype=torch.int64, device=dev)
    if kind == "neighbor_list":
        o["pairs"] = torch.full((cap, 2), -7, dtype=torch.int32, device=dev)
        o["dist"] = torch.full((cap,), np.nan, dtype=torch.float64, device=dev)
    return o


def _params(clm, kind, cap, nbins):
    L = clm._lib
    if kind == "lj_ef":
        return L.MapParams(sigma=3.4, epsilon=0.238, want_virial=1)
    if kind == "hist_dist":
        return L.MapParams(nbins=nbins, hist_hi=6.0)
    if kind == "neighbor_list":
        return L.MapParams(capacity=cap, with_distances=1)
    return L.MapParams()


def _mapout(clm, o):
    return clm._lib.MapOut(
        energy_dev=_p(o.get("energy")), forces_dev=_p(o.get("forces")), virial_dev=_p(o.get("virial")),
        grad_box_dev=_p(o.get("grad_box")), hist_dev=_p(o.get("hist")), pairs_dev=_p(o.get("pairs")),
        dist_dev=_p(o.get("dist")), count_dev=_p(o["count"]))


def _run(clm, x, box, prec, kind, static, y=None):
    L = clm._lib
    lib = L.lib()
    n, dim = x.shape
    ny = 0 if y is None else y.shape[0]
    cap, nbins = 4_000_000, 64
    o = _outputs(kind, n, dim, cap, nbins)
    P = _params(clm, kind, cap, nbins)
    ctx = clm._context(x.device)
    p = L.CLM_FP32_GUARD if prec == "fp32" else L.CLM_FP64
    if static:
        L.check(lib.clm_map_static(ctx, box._h, _p(x), n, _p(y), ny, p, L.MAP_KINDS[kind],
                                   ctypes.byref(P), ctypes.byref(_mapout(clm, o))))
    else:
        nb = ctypes.c_size_t(0)
        L.check(lib.clm_celllist_workspace_bytes(box._h, n, ny, p, ctypes.byref(nb)))
        raw = torch.empty(nb.value + 256, dtype=torch.uint8, device=x.device)
        ws = raw[(-raw.data_ptr()) % 256:]
        h = ctypes.c_void_p()
        L.check(lib.clm_celllist_create(ctx, box._h, n, ny, p, _p(ws), nb.value, ctypes.byref(h)))
        try:
            L.check(lib.clm_celllist_build(h, _p(x), _p(y)))
            L.check(lib.clm_map(h, L.MAP_KINDS[kind], ctypes.byref(P), ctypes.byref(_mapout(clm, o))))
            torch.cuda.synchronize()
        finally:
            lib.clm_celllist_destroy(h)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _cases():
    H1 = W.triclinic_h((60.0, 62.0, 58.0), (80.0, 95.0, 100.0))
    H2 = W.triclinic_h((36.0, 38.0, 35.0), (85.0, 100.0, 95.0))
    return [(W.uniform_in_box(21_000, H1, 401), H1, 9.0), (W.uniform_in_box(4_500, H2, 402), H2, 7.0)]


def _force_scale(ref, n, sigma, eps):
    """Per particle: the sum over its pairs of |f_ij| (scale of the force error)."""
    d = ref["nl_d"]
    xx = (sigma / d) ** 2
    x3 = xx ** 3
    fmag = np.abs(24.0 * eps * (2 * x3 * x3 - x3) / d)
    s = np.zeros(n)
    np.add.at(s, ref["nl_i"], fmag)
    np.add.at(s, ref["nl_j"], fmag)
    return s


def _sorted_list(r):
    m = int(r["count"][0])
    p = r["pairs"][:m].astype(np.int64)
    o = np.lexsort((p[:, 1], p[:, 0]))
    return p[o], r["dist"][:m][o]


def _check(kind, prec, r, ref, x_np, H, rc):
    """One path's outputs against the oracle at the parity tolerances."""
    n, dim = x_np.shape
    assert int(r["count"][0]) == ref["count"]
    tolE = 1e-12 if prec == "fp64" else 1e-6
    if kind == "sum_inv_d":
        assert abs(r["energy"][0] / ref["sum_inv_d"] - 1) <= tolE
    if kind == "hist_dist":
        assert np.array_equal(r["hist"].astype(np.uint64), ref["hist"])
    if kind == "neighbor_list":
        p, d = _sorted_list(r)
        assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
        if prec == "fp64":
            assert np.array_equal(d, ref["nl_d"])
        else:
            assert np.abs(d - ref["nl_d"]).max() <= 2e-6 * rc
    if kind == "lj_ef":
        assert abs(r["energy"][0] - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
        scale = _force_scale(ref, n, 3.4, 0.238)
        err = np.linalg.norm(r["forces"] + ref["lj_grad"], axis=1) / np.maximum(scale, 1e-300)
        assert err.max() <= (1e-11 if prec == "fp64" else 1e-5), err.max()
        tolB = 1e-11 if prec == "fp64" else 1e-5
        bscale = np.abs(ref["dEdH"]).max()
        assert np.abs(r["grad_box"] - ref["dEdH"]).max() <= tolB * bscale
        vscale = np.abs(ref["virial"]).max()
        assert np.abs(r["virial"] - ref["virial"]).max() <= tolB * vscale


def _same(kind, prec, a, b, ref, x_np):
    """The two paths against each other: integers exactly, floats within the
    tolerances above."""
    assert int(a["count"][0]) == int(b["count"][0])
    tolE = 1e-12 if prec == "fp64" else 1e-6
    if kind == "hist_dist":
        assert np.array_equal(a["hist"], b["hist"])
    if kind == "neighbor_list":
        pa, da = _sorted_list(a)
        pb, db = _sorted_list(b)
        assert np.array_equal(pa, pb)
        if prec == "fp64":
            assert np.array_equal(da, db)
        else:
            assert np.abs(da - db).max() <= 4e-6 * np.abs(db).max()
    if kind in ("sum_inv_d", "lj_ef"):
        assert abs(a["energy"][0] - b["energy"][0]) <= tolE * abs(b["energy"][0])
    if kind == "lj_ef":
        scale = _force_scale(ref, len(x_np), 3.4, 0.238)
        err = np.linalg.norm(a["forces"] - b["forces"], axis=1) / np.maximum(scale, 1e-300)
        assert err.max() <= (1e-11 if prec == "fp64" else 2e-5), err.max()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("kind", ["lj_ef", "neighbor_list", "hist_dist", "sum_inv_d"])
def test_static_equals_workspace_path_on_two_calls(clm, prec, kind):
    for x_np, H, rc in _cases():  # the second call is smaller than the first
        print(f"case kind={kind} prec={prec} n={len(x_np)}", flush=True)
        box = clm.Box(H, rc, 2)
        x = torch.from_numpy(x_np).to("cuda:0")
        a = _run(clm, x, box, prec, kind, static=True)
        b = _run(clm, x, box, prec, kind, static=False)
        ref = oracle.compute(x_np, H, rc, count=True, sum_inv_d=kind == "sum_inv_d",
                             lj=(3.4, 0.238) if kind == "lj_ef" else None, lj_grad=kind == "lj_ef",
                             hist=(64, 6.0) if kind == "hist_dist" else None,
                             nl=kind in ("neighbor_list", "lj_ef"))
        _check(kind, prec, a, ref, x_np, H, rc)
        _check(kind, prec, b, ref, x_np, H, rc)
        _same(kind, prec, a, b, ref, x_np)


def test_static_cross_set(clm):
    H = np.diag([60.0, 60.0, 60.0])
    x_np = W.uniform_in_box(3_000, H, 403)
    y_np = W.uniform_in_box(30_000, H, 404)
    box = clm.Box(H, 6.0, 2)
    x = torch.from_numpy(x_np).to("cuda:0")
    y = torch.from_numpy(y_np).to("cuda:0")
    ref = oracle.compute(x_np, H, 6.0, y_np, nl=True)
    for prec in ("fp32", "fp64"):
        print(f"case cross prec={prec}", flush=True)
        a = _run(clm, x, box, prec, "neighbor_list", static=True, y=y)
        b = _run(clm, x, box, prec, "neighbor_list", static=False, y=y)
        _check("neighbor_list", prec, a, ref, x_np, H, 6.0)
        _same("neighbor_list", prec, a, b, ref, x_np)


def test_static_rejects_inputs_beyond_its_scratch(clm):
    L = clm._lib
    lib = L.lib()
    mx = ctypes.c_size_t(0)
    L.check(lib.clm_map_static_max_bytes(ctypes.byref(mx)))
    H = np.diag([400.0, 400.0, 400.0])
    box = clm.Box(H, 6.0, 2)
    n = 2_000_000  # > the static scratch at about 100 bytes per particle
    nb = ctypes.c_size_t(0)
    L.check(lib.clm_celllist_workspace_bytes(box._h, n, 0, L.CLM_FP32_GUARD, ctypes.byref(nb)))
    assert nb.value > mx.value
    c = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    ctx = clm._context(torch.device("cuda:0"))
    x = torch.zeros((n, 3), dtype=torch.float64, device="cuda:0")  # rejected before any launch
    st = lib.clm_map_static(ctx, box._h, _p(x), n, None, 0, L.CLM_FP32_GUARD, L.MAP_KINDS["count"],
                            ctypes.byref(L.MapParams()), ctypes.byref(L.MapOut(count_dev=_p(c))))
    assert st == L.STATUS_CODES["CLM_E_CAPACITY"]
    assert b"static scratch" in lib.clm_last_error()
    torch.cuda.synchronize()
    assert int(c.item()) == -1  # outputs untouched
