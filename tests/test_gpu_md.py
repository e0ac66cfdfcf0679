"""GPU parity of the molecular-dynamics calls (include/clmap_md.h) against the
CPU oracle: the Verlet list's pair set, energy, forces and virial in the
frame of its last rebuild, its device-side rebuild decisions, and whole
velocity-Verlet trajectories (Verlet list and rebuild-every-step forms)
against ``oracle.md_run``.  Integers (pair counts) are compared exactly;
the list path is FP64 throughout (energies 1e-12, forces 1e-11 of the
per-particle sum of pair-force magnitudes)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SIG, EPS = W.NEON["sigma"], W.NEON["epsilon"]
RC = W.NEON["cutoff"]


@pytest.fixture(scope="module")
def md():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2202_06427_amd.md as md
    return md


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _force_scale(ref, n, sigma, eps):
    d = ref["nl_d"]
    x3 = (sigma / d) ** 6
    fm = np.abs(24.0 * eps * (2 * x3 * x3 - x3) / d)
    s = np.zeros(n)
    np.add.at(s, ref["nl_i"], fm)
    np.add.at(s, ref["nl_j"], fm)
    return s


def _lj_outputs(vl, n, dim):
    F = torch.empty((n, dim), dtype=torch.float64, device="cuda:0")
    E = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    Wv = torch.zeros((dim, dim), dtype=torch.float64, device="cuda:0")
    C = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    vl.lj(SIG, EPS, F, E, virial=Wv, count=C)
    return F.cpu().numpy(), E.item(), Wv.cpu().numpy(), int(C.item())


def _check_against_oracle(x, H, frame, F, E, Wv, C, rc=RC):
    ref = oracle.compute(x, H, rc, lj=(SIG, EPS), lj_grad=True, nl=True, frame=frame)
    assert C == ref["count"]
    assert abs(E - ref["lj_energy"]) <= 1e-12 * abs(ref["lj_energy"])
    err = np.linalg.norm(F + ref["lj_grad"], axis=1) / _force_scale(ref, len(x), SIG, EPS)
    assert err.max() <= 1e-11, err.max()
    assert np.abs(Wv - ref["virial"]).max() <= 1e-11 * np.abs(ref["virial"]).max()


@pytest.mark.parametrize("lcell", [1, 2])
def test_vlist_forces_at_a_rebuild(md, lcell):
    w = W.neon_fluid(8000, seed=11)
    x, H = w["x"], w["H"]
    xd = T(x)
    vl = md.VerletList(xd, H, RC, 0.2, lcell=lcell)
    vl.update(xd)
    F, E, Wv, C = _lj_outputs(vl, len(x), 3)
    info = vl.info()
    assert info["rebuilds"] == 1 and info["updates"] == 1 and info["overflow"] == 0
    assert info["entries"] >= 2 * C
    _check_against_oracle(x, H, oracle.wrap(x, H)[2], F, E, Wv, C)


def test_vlist_forces_at_a_rebuild_large(md):
    """Above 400k particles the list is built one wave per tile (one pass)."""
    w = W.neon_fluid(420_000, seed=17)
    x, H = w["x"], w["H"]
    xd = T(x)
    vl = md.VerletList(xd, H, RC, 0.1, lcell=2)
    vl.update(xd)
    F, E, Wv, C = _lj_outputs(vl, len(x), 3)
    assert vl.info()["overflow"] == 0
    _check_against_oracle(x, H, oracle.wrap(x, H)[2], F, E, Wv, C)


def test_vlist_forces_at_a_rebuild_1e6(md):
    """The benchmark's largest Neon case (10^6 atoms, skin 0.1 nm): per-tile
    build, 4 lanes per row.  Pair count exact, energy and virial 1e-12; forces
    per particle within 1e-10 of the largest reference force (the list path
    is FP64 throughout)."""
    w = W.neon_fluid(1_000_000, seed=6)
    x, H = w["x"], w["H"]
    xd = T(x)
    vl = md.VerletList(xd, H, RC, 0.1, lcell=2)
    vl.update(xd)
    F, E, Wv, C = _lj_outputs(vl, len(x), 3)
    info = vl.info()
    assert info["overflow"] == 0 and info["rebuilds"] == 1
    ref = oracle.compute(x, H, RC, lj=(SIG, EPS), lj_grad=True, frame=oracle.wrap(x, H)[2])
    assert C == ref["count"]
    assert abs(E - ref["lj_energy"]) <= 1e-12 * abs(ref["lj_energy"])
    Fr = -ref["lj_grad"]
    assert np.abs(F - Fr).max() <= 1e-10 * np.abs(Fr).max()
    assert np.abs(Wv - ref["virial"]).max() <= 1e-11 * np.abs(ref["virial"]).max()


def test_vlist_between_rebuilds_and_across_the_box_faces(md):
    """Displacements below half the skin keep the list (no rebuild); the
    distances are taken in the frame of the rebuild, also for particles that
    crossed a face of the box.  A larger displacement triggers a rebuild."""
    w = W.neon_fluid(6000, seed=12)
    x0, H = w["x"].copy(), w["H"]
    L = H[0, 0]
    g = W.rng(13)
    # 60 particles just inside the upper x face; they cross it below
    near = g.choice(len(x0), 60, replace=False)
    x0[near, 0] = L - 0.01 * g.random(60)
    skin = 0.2
    xd = T(x0)
    vl = md.VerletList(xd, H, RC, skin, lcell=2)
    vl.update(xd)
    frame0 = oracle.wrap(x0, H)[2]
    d = g.normal(size=x0.shape)
    d *= (0.45 * skin * g.random((len(x0), 1))) / np.linalg.norm(d, axis=1, keepdims=True)
    d[near] = [0.03, 0.0, 0.0]
    x1 = x0 + d
    assert not np.array_equal(oracle.wrap(x1, H)[2], frame0)   # some wraps changed
    xd.copy_(T(x1))
    vl.update(xd)
    F, E, Wv, C = _lj_outputs(vl, len(x1), 3)
    assert vl.info()["rebuilds"] == 1
    _check_against_oracle(x1, H, frame0, F, E, Wv, C)
    # one particle beyond half the skin: rebuild in the new canonical frame
    x2 = x1.copy()
    x2[7] += [0.0, 0.0, 0.6 * skin]
    xd.copy_(T(x2))
    vl.update(xd)
    F, E, Wv, C = _lj_outputs(vl, len(x2), 3)
    assert vl.info()["rebuilds"] == 2 and vl.info()["updates"] == 3
    _check_against_oracle(x2, H, oracle.wrap(x2, H)[2], F, E, Wv, C)


def test_vlist_row_overflow_is_reported(md):
    w = W.neon_fluid(6000, seed=14)
    xd = T(w["x"])
    vl = md.VerletList(xd, w["H"], RC, 0.2, lcell=2, capacity=16)
    vl.update(xd)
    F = torch.empty((6000, 3), dtype=torch.float64, device="cuda:0")
    E = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    vl.lj(SIG, EPS, F, E)
    info = vl.info()
    assert info["overflow"] == 1 and info["max_row"] > 16


def _md_case(n=6000, seed=15):
    w = W.neon_fluid(n, seed=seed)
    ndof = 3 * n - 3
    target = 0.5 * ndof * W.KB * w["temperature"]
    return w, target


@pytest.mark.parametrize("mode,graph", [("verlet", False), ("verlet", True), ("rebuild", False)])
def test_md_trajectory_matches_the_oracle(md, mode, graph):
    w, target = _md_case()
    nsteps = 30
    skin = 0.2 if mode == "verlet" else 0.0
    ref = oracle.md_run(w["x"], w["v"], w["H"], RC, SIG, EPS, w["mass"], w["dt"], nsteps,
                        skin=skin, rescale_every=10, target_ke=target)
    x, v = T(w["x"]), T(w["v"])
    out = md.run(x, v, w["H"], cutoff=RC, sigma=SIG, epsilon=EPS, mass=w["mass"], dt=w["dt"],
                 nsteps=nsteps, mode=mode, skin=max(skin, 0.2), rescale_every=10, target_ke=target,
                 precision="fp64", graph=graph)
    torch.cuda.synchronize()
    assert np.array_equal(out["count"].cpu().numpy(), ref["count"])
    E = out["energy"].cpu().numpy()
    assert np.abs(E - ref["energy"]).max() <= 1e-10 * np.abs(ref["energy"]).max()
    KE = out["ke"].cpu().numpy()
    assert np.abs(KE - ref["ke"]).max() <= 1e-10 * np.abs(ref["ke"]).max()
    assert np.abs(x.cpu().numpy() - ref["x"]).max() < 1e-10
    assert np.abs(v.cpu().numpy() - ref["v"]).max() < 1e-9 * np.abs(ref["v"]).max()
    if mode == "verlet":
        info = out["list"].info()
        assert info["updates"] == nsteps + 1 and info["overflow"] == 0
        assert info["rebuilds"] == int(ref["rebuilt"].sum())


def test_md_rebuild_mode_fp32_guard(md):
    """The paper's protocol with FP32+guard forces.  The trajectory is another
    rounding of the FP64 one (FP32 forces), so a pair within ~1e-10 nm of the
    cutoff may sit on different sides in the two runs; the pair set of each
    step is therefore checked exactly against the oracle at the positions the
    GPU step itself used, and the trajectory against the FP64 oracle run
    within the FP32 force tolerance."""
    w, target = _md_case(5000, seed=16)
    nsteps = 20
    ref = oracle.md_run(w["x"], w["v"], w["H"], RC, SIG, EPS, w["mass"], w["dt"], nsteps,
                        rescale_every=10, target_ke=target)
    x, v = T(w["x"]), T(w["v"])
    traj = torch.empty((nsteps + 1,) + tuple(x.shape), dtype=torch.float64, device="cuda:0")
    out = md.run(x, v, w["H"], cutoff=RC, sigma=SIG, epsilon=EPS, mass=w["mass"], dt=w["dt"],
                 nsteps=nsteps, mode="rebuild", rescale_every=10, target_ke=target, precision="fp32",
                 trajectory=traj)
    torch.cuda.synchronize()
    counts = out["count"].cpu().numpy()
    E = out["energy"].cpu().numpy()
    tr = traj.cpu().numpy()
    for k in range(nsteps + 1):
        own = oracle.compute(tr[k], w["H"], RC, lj=(SIG, EPS))
        assert counts[k] == own["count"], k
        assert abs(E[k] - own["lj_energy"]) <= 1e-6 * abs(own["lj_energy"]), k
    assert np.abs(E - ref["energy"]).max() <= 1e-6 * np.abs(ref["energy"]).max()
    assert np.abs(x.cpu().numpy() - ref["x"]).max() < 1e-9
    assert np.abs(tr[nsteps] - x.cpu().numpy()).max() == 0.0
