"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark uses (lcell 2, FP32+guard and FP64), against the
CPU oracle on the same seeded inputs:

  uniform-1e4 cube 46.42 rc 8        neighbour list + sum 1/d (plain FP64)
  uniform-1e6 triclinic 215.4 rc 12  LJ energy, forces (100 sampled particles,
                                     finite differences), far-from-origin copy
  cross 5e3 blob x 5e5 uniform rc 5  cross-set neighbour list
  2D clustered 2e6 rc 0.01           256-bin relative-speed histogram
"""
import math

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


def _sorted(pairs):
    p = pairs.cpu().numpy().astype(np.int64)
    o = np.lexsort((p[:, 1], p[:, 0]))
    return p[o], o


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config1_neighbor_list_and_inverse_distance_sum(clm, precision):
    c = W.config1()
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], nl=True, sum_inv_d=True)
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision=precision)
    pairs, dist = cl.neighbor_list()
    p, o = _sorted(pairs)
    assert len(p) == ref["count"] and np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])
    if precision == "fp64":
        assert np.array_equal(dist.cpu().numpy()[o], ref["nl_d"])
    s, cnt = cl.sum_inv_d()
    assert int(cnt.item()) == ref["count"]
    assert abs(s.item() / ref["sum_inv_d"] - 1) < (1e-12 if precision == "fp64" else 1e-6)


@pytest.fixture(scope="module")
def cfg2():
    c = W.config2()
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], lj=(c["sigma"], c["epsilon"]), lj_grad=True,
                         lj_fabs=True)
    return c, ref


def _force_err(F, ref):
    """Per-particle force error relative to the sum of the pair-force
    magnitudes on the particle (forces = -dE/dr)."""
    return np.linalg.norm(F + ref["lj_grad"], axis=1) / np.maximum(ref["lj_fabs"], 1e-300)


@pytest.mark.parametrize("form", ["fp32-half", "fp32-full", "fp64"])
def test_config2_all_forces_element_by_element(clm, cfg2, form):
    """All 10^6 forces of the headline workload against the oracle's, each
    particle's error measured against the sum of its pair-force magnitudes:
    FP32+guard <= 1e-5 (both the half-shell sweep and the full-shell
    gather), plain FP64 <= 1e-11; energies 1e-6 / 1e-12, the box gradient
    1e-5 / 1e-11 of its largest entry."""
    c, ref = cfg2
    s, e = c["sigma"], c["epsilon"]
    prec = "fp64" if form == "fp64" else "fp32"
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision=prec)
    out = cl.lj_forces(s, e, half=form != "fp32-full")
    assert int(out["count"].item()) == ref["count"]
    tol = 1e-11 if form == "fp64" else 1e-5
    tolE = 1e-12 if form == "fp64" else 1e-6
    err = _force_err(out["forces"].cpu().numpy(), ref)
    print(f"{form}: max per-particle force error {err.max():.3e}, mean {err.mean():.3e}", flush=True)
    assert err.max() <= tol, err.max()
    assert abs(out["energy"].item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    gb = out["grad_box"].cpu().numpy()
    assert np.abs(gb - ref["dEdH"]).max() <= tol * np.abs(ref["dEdH"]).max()


def test_config2_lattice_fp32_energy_and_forces(clm):
    """The jittered-lattice variant (no overlapping pairs; the pairs beyond
    sigma, most of them, are evaluated in FP32): energy within 1e-6 and
    every particle's force within 1e-5, half-shell sweep."""
    c = W.config2(variant="lattice")
    s, e = c["sigma"], c["epsilon"]
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], lj=(s, e), lj_grad=True, lj_fabs=True)
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision="fp32")
    out = cl.lj_forces(s, e)
    assert int(out["count"].item()) == ref["count"]
    rel = abs(out["energy"].item() - ref["lj_energy"]) / abs(ref["lj_energy"])
    err = _force_err(out["forces"].cpu().numpy(), ref)
    print(f"lattice fp32: energy rel err {rel:.3e}, max force err {err.max():.3e}", flush=True)
    assert rel <= 1e-6
    assert err.max() <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config2_lj_energy_forces(clm, cfg2, precision):
    c, ref = cfg2
    s, e = c["sigma"], c["epsilon"]
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision=precision)
    out = cl.lj_forces(s, e)
    assert int(out["count"].item()) == ref["count"]
    tolE = 1e-6 if precision == "fp32" else 1e-12
    assert abs(out["energy"].item() - ref["lj_energy"]) <= tolE * abs(ref["lj_energy"])
    # forces on 100 particles drawn with seed 102, against brute force over all j
    sample = W.rng(102).choice(len(c["x"]), 100, replace=False)
    _, g = oracle.lj_sample(c["x"], c["H"], c["cutoff"], sample, s, e)
    F = out["forces"].cpu().numpy()[sample]
    denom = np.empty(len(sample))
    for k, i in enumerate(sample):
        js, Ks = oracle.neighbors_of(c["x"], c["H"], c["cutoff"], int(i))
        D = c["x"][js] - c["x"][i] + Ks @ c["H"].T
        d2 = (D * D).sum(1)
        x3 = (s * s / d2) ** 3
        denom[k] = np.abs(24 * e * (2 * x3 * x3 - x3) / np.sqrt(d2)).sum()
    err = np.linalg.norm(F + g, axis=1) / denom
    assert err.max() <= (1e-5 if precision == "fp32" else 1e-11), err.max()


def test_config2_forces_finite_differences(clm, cfg2):
    """Adjoint forces vs central differences of each particle's own energy
    E_i = sum_j u(d_ij) with the pair set frozen (the LJ potential has no
    switch at the cutoff, so a pair crossing it would dominate a plain FD)."""
    c, _ = cfg2
    s, e, H = c["sigma"], c["epsilon"], c["H"]
    cl = clm.CellList(T(c["x"]), clm.Box(H, c["cutoff"], 2), precision="fp32")
    up = torch.ones(1, dtype=torch.float64, device="cuda:0")
    gx, _, _ = cl.lj_adjoint(s, e, up)
    gx = gx.cpu().numpy()
    sample = W.rng(102).choice(len(c["x"]), 100, replace=False)
    worst = 0.0
    for i in sample:
        js, Ks = oracle.neighbors_of(c["x"], H, c["cutoff"], int(i))
        img = c["x"][js] + Ks @ H.T  # frozen images of the partners

        def Ei(xi):
            D = img - xi
            d2 = (D * D).sum(1)
            x3 = (s * s / d2) ** 3
            return (4 * e * (x3 * x3 - x3)).sum()

        dmin = np.sqrt(((img - c["x"][i]) ** 2).sum(1).min())
        h = 1e-6 * max(1.0, dmin)
        fd = np.zeros(3)
        for a in range(3):
            xp = c["x"][i].copy(); xp[a] += h
            xm = c["x"][i].copy(); xm[a] -= h
            fd[a] = (Ei(xp) - Ei(xm)) / (2 * h)
        rel = np.linalg.norm(fd - gx[i]) / max(np.linalg.norm(fd), 1e-300)
        worst = max(worst, rel)
    assert worst <= 1e-6, worst


@pytest.mark.parametrize("variant", ["far", "lattice"])
def test_config2_variants(clm, variant):
    c = W.config2(variant=variant)
    s, e = c["sigma"], c["epsilon"]
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], lj=(s, e))
    for precision in ("fp32", "fp64"):
        cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision=precision)
        E, cnt = cl.lj_energy(s, e)
        assert int(cnt.item()) == ref["count"]
        tol = 1e-6 if precision == "fp32" else 1e-12
        assert abs(E.item() - ref["lj_energy"]) <= tol * abs(ref["lj_energy"]), (precision, E.item(), ref["lj_energy"])
        del cl


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config3_cross_set_pairs(clm, precision):
    c = W.config3()
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], c["y"], nl=True)
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), y=T(c["y"]), precision=precision)
    pairs, _ = cl.neighbor_list()
    p, _ = _sorted(pairs)
    assert len(p) == ref["count"]
    assert np.array_equal(p[:, 0], ref["nl_i"]) and np.array_equal(p[:, 1], ref["nl_j"])


@pytest.fixture(scope="module")
def cfg4():
    c = W.config4()
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], rel_hist=(c["rel_nbins"], c["rel_hi"]), vel_x=c["v"])
    return c, ref


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config4_relative_speed_histogram(clm, cfg4, precision):
    c, ref = cfg4
    cl = clm.CellList(T(c["x"]), clm.Box(c["H"], c["cutoff"], 2), precision=precision)
    h, sums, cnt = cl.relspeed_histogram(T(c["v"]), c["rel_nbins"], c["rel_hi"])
    assert int(cnt.item()) == ref["count"] > 2 ** 32
    assert np.array_equal(h.cpu().numpy().astype(np.uint64), ref["rel_hist"])
    rs = ref["rel_sum"]
    tol = 1e-6 if precision == "fp32" else 1e-12
    assert np.all(np.abs(sums.cpu().numpy() - rs) <= tol * np.abs(rs) + 1e-300)
