"""GPU parity of the half-shell Lennard-Jones force sweep (every pair
evaluated once, both particles' force sums kept in planes with one writer per
slot, summed per particle in FP64) in its two forms -- FP32 + FP64 guard
(FP32 planes) and plain FP64 (FP64 planes) -- against the oracle and against
the full-shell gather, through the C-ABI.

Tolerances as for every map of the form: FP32+guard energy 1e-6 relative,
per-particle force error 1e-5 relative to the sum of the pair-force
magnitudes on that particle, box gradient and virial 1e-5 of their largest
entry; FP64 1e-12, 1e-11 and 1e-11; pair counts exact."""
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


def _lattice(H, n, seed, jitter=0.3):
    dim = H.shape[0]
    m = int(round(n ** (1.0 / dim)))
    grid = np.stack(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"), -1).reshape(-1, dim)
    s = (grid + 0.5 + jitter * (W.rng(seed).random(grid.shape) - 0.5)) / m
    return s @ H.T


def _force_scale(ref, n, sigma, eps):
    d = ref["nl_d"]
    xx = (sigma / d) ** 2
    x3 = xx ** 3
    fmag = np.abs(24.0 * eps * (2 * x3 * x3 - x3) / d)
    s = np.zeros(n)
    np.add.at(s, ref["nl_i"], fmag)
    np.add.at(s, ref["nl_j"], fmag)
    return s


TOL = {"fp32": (1e-6, 1e-5), "fp64": (1e-12, 1e-11)}


def _check(out, ref, x, sigma, eps, virial=True, precision="fp32"):
    n = len(x)
    tolE, tolF = TOL[precision]
    assert int(out["count"].item()) == ref["count"]
    assert abs(out["energy"].item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    scale = _force_scale(ref, n, sigma, eps)
    err = np.linalg.norm(out["forces"].cpu().numpy() + ref["lj_grad"], axis=1) / np.maximum(scale, 1e-300)
    assert err.max() <= tolF, err.max()
    gb = out["grad_box"].cpu().numpy()
    assert np.abs(gb - ref["dEdH"]).max() <= tolF * np.abs(ref["dEdH"]).max()
    if virial:
        assert np.abs(out["virial"].cpu().numpy() - ref["virial"]).max() <= tolF * np.abs(ref["virial"]).max()


BOXES = {
    "cube3": (np.diag([30.0, 30.0, 30.0]), 5.0),
    "tric3": (W.triclinic_h((32.0, 30.0, 31.0), (80.0, 95.0, 100.0)), 4.0),
    "skew3": (W.triclinic_h((30.0, 29.0, 33.0), (70.0, 110.0, 75.0)), 4.0),
    "sq2": (np.diag([60.0, 60.0]), 3.0),
    "tric2": (np.array([[55.0, -12.0], [0.0, 50.0]]), 3.2),
}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("lcell,lcell_x", [(1, None), (2, None), (3, None), (2, 3)])
@pytest.mark.parametrize("prune", [True, False])
def test_half_shell_lattice_against_oracle(clm, name, lcell, lcell_x, prune, precision):
    H, rc = BOXES[name]
    dim = H.shape[0]
    x = _lattice(H, 6000 if dim == 3 else 5000, 11) + H @ np.array([3, -2, 5][:dim])
    sigma, eps = 1.1, 0.3
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, lcell, lcell_x), precision=precision)
    assert cl._half_scratch("lj_ef", True)[1] > 0, "the half-shell sweep applies here"
    print(f"case {name} lcell={lcell} lcell_x={lcell_x} prune={prune} {precision}", flush=True)
    _check(cl.lj_forces(sigma, eps, virial=True, half=True, prune=prune), ref, x, sigma, eps,
           precision=precision)
    _check(cl.lj_forces(sigma, eps, virial=False, half=True, prune=prune), ref, x, sigma, eps, virial=False,
           precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["tric3", "cube3", "tric2"])
@pytest.mark.parametrize("prune", [True, False])
def test_half_shell_uniform_random_near_pairs(clm, name, prune, precision):
    """Uniform random points: pairs far inside sigma (the canonical FP64
    near-pair path, forces into both particles' planes) dominate E."""
    H, rc = BOXES[name]
    x = W.uniform_in_box(6000, H, 21)
    sigma, eps = 3.4 if H.shape[0] == 3 else 1.0, 0.238
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    out = cl.lj_forces(sigma, eps, virial=True, half=True, prune=prune)
    _check(out, ref, x, sigma, eps, precision=precision)
    info = cl.info()
    assert info["near_evaluations"] > 0
    # every evaluated pair was tested; pruning drops only pairs beyond the cutoff
    assert ref["count"] <= info["half_pairs_kept"] <= info["half_pairs_tested"]
    if not prune:
        assert info["half_pairs_kept"] == info["half_pairs_tested"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_half_shell_heavy_cell_tiles(clm, precision):
    """900 particles in one cell (tiles that split a cell, so the home row's
    first block starts inside a cell) among uniform ones."""
    H = np.diag([40.0, 40.0, 40.0])
    g = W.rng(3)
    x = np.concatenate([20.0 + 0.8 * g.random((900, 3)), W.uniform_in_box(3000, H, 4)])
    sigma, eps = 0.2, 0.01
    ref = oracle.compute(x, H, 3.0, lj=(sigma, eps), lj_grad=True, nl=True)
    cl = clm.CellList(T(x), clm.Box(H, 3.0, 2), precision=precision)
    _check(cl.lj_forces(sigma, eps, virial=True, half=True), ref, x, sigma, eps, precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_half_shell_map_cutoff_and_adjoint(clm, precision):
    H, rc = BOXES["tric3"]
    x = _lattice(H, 6000, 12)
    sigma, eps = 1.1, 0.3
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    rm = 0.7 * rc
    ref = oracle.compute(x, H, rm, lj=(sigma, eps), lj_grad=True, nl=True)
    _check(cl.lj_forces(sigma, eps, virial=True, cutoff=rm, half=True), ref, x, sigma, eps, precision=precision)
    g = torch.tensor([2.5], dtype=torch.float64, device="cuda:0")
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True, nl=True)
    gx, gb, e = cl.lj_adjoint(sigma, eps, g, half=True)
    scale = _force_scale(ref, len(x), sigma, eps)
    err = np.linalg.norm(gx.cpu().numpy() - 2.5 * ref["lj_grad"], axis=1) / np.maximum(2.5 * scale, 1e-300)
    tolF = TOL[precision][1]
    assert err.max() <= tolF
    assert np.abs(gb.cpu().numpy() - 2.5 * ref["dEdH"]).max() <= tolF * 2.5 * np.abs(ref["dEdH"]).max()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_half_shell_equals_full_shell_and_repeats_bitwise(clm, precision):
    H, rc = BOXES["skew3"]
    x = W.uniform_in_box(8000, H, 31)
    sigma, eps = 2.0, 0.2
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision=precision)
    a = cl.lj_forces(sigma, eps, virial=True, half=True)
    b = cl.lj_forces(sigma, eps, virial=True, half=True)
    for k in ("energy", "forces", "grad_box", "virial", "count"):
        assert a[k].cpu().numpy().tobytes() == b[k].cpu().numpy().tobytes(), k
    f = cl.lj_forces(sigma, eps, virial=True, half=False)
    assert int(f["count"].item()) == int(a["count"].item())
    ref = oracle.compute(x, H, rc, lj=(sigma, eps), lj_grad=True, nl=True)
    _check(a, ref, x, sigma, eps, precision=precision)
    _check(f, ref, x, sigma, eps, precision=precision)


def test_half_shell_scratch_errors(clm):
    import ctypes
    L = clm._lib
    H, rc = BOXES["cube3"]
    x = _lattice(H, 3000, 13)
    cl = clm.CellList(T(x), clm.Box(H, rc, 2), precision="fp32")
    sp, need = cl._half_scratch("lj_ef", True)
    e = torch.empty(1, dtype=torch.float64, device="cuda:0")
    c = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    f = torch.empty((len(x), 3), dtype=torch.float64, device="cuda:0")
    P = L.MapParams(sigma=1.0, epsilon=0.1, scratch_dev=sp, scratch_bytes=need - 1)
    o = L.MapOut(energy_dev=ctypes.c_void_p(e.data_ptr()), forces_dev=ctypes.c_void_p(f.data_ptr()),
                 count_dev=ctypes.c_void_p(c.data_ptr()))
    st = L.lib().clm_map(cl._h, L.MAP_KINDS["lj_ef"], ctypes.byref(P), ctypes.byref(o))
    assert st == L.STATUS_CODES["CLM_E_WORKSPACE"]
    P.scratch_dev = ctypes.c_void_p(sp.value + 8)
    P.scratch_bytes = need
    st = L.lib().clm_map(cl._h, L.MAP_KINDS["lj_ef"], ctypes.byref(P), ctypes.byref(o))
    assert st == L.STATUS_CODES["CLM_E_WORKSPACE"]
    torch.cuda.synchronize()
    assert int(c.item()) == -1
    # the FP64 form keeps FP64 planes: twice the plane bytes; where the
    # sweep does not apply (a cross set) the scratch is 0 bytes
    cl64 = clm.CellList(T(x), clm.Box(H, rc, 2), precision="fp64")
    assert cl64._half_scratch("lj_ef", True)[1] > need
    clx = clm.CellList(T(x), clm.Box(H, rc, 2), y=T(x[:100]), precision="fp32")
    assert clx._half_scratch("lj_ef", True) == (None, 0)


def test_automatic_choice_between_half_and_full_shell(clm):
    """half=None: the half-shell sweep when the grid gives at least 4096
    (cell row, neighbour row) work items, or when a cell row holds no more
    64-particle tiles on average than a gather tile visits rows
    ((2l+1)^2 in 3D); the full-shell gather otherwise (long rows, few
    items).  The two forms round differently, so the choice shows bit for
    bit."""
    sigma, eps = 1.1, 0.3
    cases = ((30.0, 3000, 2, True),    # 1872 items, 0.3 tiles a row
             (60.0, 20000, 2, True),   # 7488 items
             (30.0, 30000, 1, False))  # 180 items, 13 tiles a row > 9
    for L_box, n, lcell, want_half in cases:
        H = np.diag([L_box] * 3)
        x = _lattice(H, n, 14)
        box = clm.Box(H, 5.0, lcell)
        rows = 1
        for g in box.info()["grid"][1:]:
            rows *= g
        nr = 2 * lcell * lcell + 2 * lcell + 1
        reach = (2 * lcell + 1) ** 2
        assert (rows * nr >= 4096 or n / (64 * rows) <= reach) == want_half
        cl = clm.CellList(T(x), box, precision="fp32")
        auto = cl.lj_forces(sigma, eps, virial=True)
        forced = cl.lj_forces(sigma, eps, virial=True, half=want_half)
        other = cl.lj_forces(sigma, eps, virial=True, half=not want_half)
        fa, ff, fo = (r["forces"].cpu().numpy() for r in (auto, forced, other))
        assert fa.tobytes() == ff.tobytes()
        assert fa.tobytes() != fo.tobytes()
        ref = oracle.compute(x, H, 5.0, lj=(sigma, eps), lj_grad=True, nl=True)
        _check(auto, ref, x, sigma, eps)
