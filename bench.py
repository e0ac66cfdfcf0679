"""Benchmark: within-cutoff pairs/s of the cell-list hot path on one MI355X.

Workload (the headline configuration): 1,000,000 uniform-random particles in
a triclinic periodic box (lengths 215.4, angles 80/95/100 degrees), cutoff
12, Lennard-Jones energy + forces (sigma 3.4, epsilon 0.238) through the
adjoint sweep.  One step = one pass of the whole hot path over the resident
positions: build (wrap and cell index with LDS bucket counts, prefix scan,
bucket pass, per-bucket placement, tiles) + the LJ
sweep with fused energy/force/box-gradient reduction (the half-shell sweep,
every pair once, in both forms: FP32+guard with FP32 force planes, plain FP64
with FP64 planes) +
per-particle force gather + finalize.  The FP32+guard form is the headline
value; the plain FP64 form is reported beside it.

Prints ONE JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks used as roofline denominators
HBM_PEAK_GBS = 8000.0
VALU_FP32_NONPACKED_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
VALU_FP32_PACKED_TFLOPS = 157.3     # needs packed FP32, which this build does not emit
VALU_FP64_TFLOPS = 78.6

# algorithmic work per unit (what the method must do)
FLOPS_PER_CANDIDATE = 8        # 3 sub, 3 mul, 2 add (distance test)
FLOPS_PER_LJ_PAIR = 20         # 1 reciprocal + ~19 flops: energy + force on both particles
BUILD_BYTES_PER_PARTICLE = 44  # 24 read + 16 (FP32 record) + 4 (index) written, 3D


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_half_lj_forces_uniform1e6_hbm_traffic.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2202_06427_amd", "csrc", "sweep_half.hip")


def measured_traffic():
    """HBM bytes per launch of the headline sweep from the committed counter
    summary, or None when the sweep source has changed since it was taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        sha = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines() if ": " in l and not l.startswith(("-", "|", "`")))
    if fields.get("sweep_half.hip sha256 prefix", "").strip() != sha:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lcell", type=int, default=2)
    ap.add_argument("--lcell-x", type=int, default=6,
                    help="cell reach along the row axis (thinner cells along the row; 0: lcell)")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--serve-requests", type=int, default=10_000)
    ap.add_argument("--serve-fracs", type=str, default="0.5,0.8,0.95",
                    help="Poisson arrival rates of the served mix as fractions of the measured "
                         "closed-loop capacity")
    ap.add_argument("--build-n-large", type=int, default=16_000_000,
                    help="particle count of the second build-bandwidth point (0: skip)")
    ap.add_argument("--md-steps", type=int, default=200,
                    help="velocity-Verlet steps per Neon MD case (0: skip the MD section)")
    ap.add_argument("--kclosest", type=int, default=1, help="0: skip the k-closest-pairs section")
    ap.add_argument("--weighted", type=int, default=1, help="0: skip the weighted-map section")
    ap.add_argument("--nonperiodic", type=int, default=1, help="0: skip the non-periodic list section")
    ap.add_argument("--md-only", type=int, default=0, metavar="N",
                    help="run only --steps Verlet-list MD steps of N Neon atoms (profiling)")
    ap.add_argument("--calibrate", type=int, default=1,
                    help="0: skip the measured device rates (FMA loops, copy kernel)")
    ap.add_argument("--sweep-forms", type=int, default=1,
                    help="0: skip timing the unpruned half-shell and full-shell sweeps")
    ap.add_argument("--step-samples", type=int, default=20,
                    help="individually timed steps for the median / min step time (0: skip)")
    ap.add_argument("--pruning", type=int, default=1,
                    help="0: skip the pruning section (sweep forms at lcell 1/2/3, 2D clustered)")
    ap.add_argument("--section", choices=["kclosest", "nonperiodic", "weighted", "pruning"], default=None,
                    help="run only this section and print its JSON (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--build-only", type=int, default=0, metavar="N",
                    help="only time cell-list builds of N uniform particles (profiling)")
    return ap.parse_args()


def copy_calibration(mib, reps=4):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    counter readings give the scale factor for the sweep's readings."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read_per_copy": n * 4,
                      "copy_calibration_bytes_written_per_copy": n * 4, "copies": reps}), flush=True)


def time_steps(clm, cl, xt, steps, warmup, sigma, eps, samples=0):
    import torch
    for _ in range(warmup):
        cl.build(xt)
        out = cl.lj_forces(sigma, eps)
    # the timed steps run without the library's phase events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        cl.build(xt)
        out = cl.lj_forces(sigma, eps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same steps again with the library's events around the build and
    # the sweep (phase times; the sweep's is the roofline's kernel time)
    clm.set_timing(True)
    clm.stats(reset=True)
    for _ in range(steps):
        cl.build(xt)
        cl.lj_forces(sigma, eps)
    torch.cuda.synchronize()
    st = clm.stats(reset=True)
    clm.set_timing(False)
    per_step = []
    for _ in range(samples):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        cl.build(xt)
        cl.lj_forces(sigma, eps)
        e1.record()
        e1.synchronize()
        per_step.append(e0.elapsed_time(e1))
    per_step.sort()
    return {
        "step_ms_median": per_step[len(per_step) // 2] if per_step else None,
        "step_ms_min": per_step[0] if per_step else None,
        "ms_per_step": ev0.elapsed_time(ev1) / steps,
        "wall_ms_per_step": 1e3 * wall / steps,
        "sweep_ms": st["sweep_ms"] / max(st["sweeps"], 1),
        "build_ms": st["build_ms"] / max(st["builds"], 1),
        "count": int(out["count"].item()),
        "energy": float(out["energy"].item()),
    }


def served(n_requests, fracs, seed=5, budget=8 << 30):
    """Served mix: closed-loop capacity (every job available at once), then
    Poisson arrivals at each fraction of that capacity, with p50/p99
    latency (arrival -> results complete on the device).  Results other than
    counts and energies are dropped when a job completes (keep_results off),
    as a server that hands them on would."""
    import numpy as np

    import workloads as W
    from paper_2202_06427_amd.serve import Job, Server

    import torch
    reqs = W.serve_requests(seed=seed, count=n_requests)
    # request payloads arrive in pinned host memory (as from a network stack):
    # one pinned buffer, a view per request
    sizes = [r["n"] * 3 for r in reqs]
    buf = torch.empty(sum(sizes), dtype=torch.float64, pin_memory=True)
    xs, off = [], 0
    for r, sz in zip(reqs, sizes):
        v = buf[off: off + sz].view(r["n"], 3)
        v.copy_(torch.from_numpy(W.request_positions(r)))
        xs.append(v)
        off += sz

    def jobs(rate):
        g = np.random.Generator(np.random.PCG64(seed + 1))
        t, out = 0.0, []
        for r, x in zip(reqs, xs):
            t += g.exponential(1.0 / rate) if rate else 0.0
            out.append(Job(r["id"], x, r["H"], r["cutoff"], r["kind"], arrival=t))
        return out

    warm = Server(hbm_budget=budget, keep_results=False)
    warm.run(jobs(None)[: min(64, n_requests)], realtime=False)
    closed = Server(hbm_budget=budget, keep_results=False).run(jobs(None), realtime=False)
    cap = closed["jobs_per_s"]
    out = {"requests": n_requests, "capacity_jobs_per_s": cap, "hbm_budget_bytes": budget,
           "closed_loop": {k: closed[k] for k in ("p50_ms", "p99_ms", "mean_batch", "failed",
                                                  "rejected", "nl_retries", "peak_hbm_bytes")},
           "rates": []}
    for f in fracs:
        r = Server(hbm_budget=budget, keep_results=False).run(jobs(f * cap), realtime=True)
        out["rates"].append({"frac_of_capacity": f, "rate_jobs_per_s": f * cap, "p50_ms": r["p50_ms"],
                             "p99_ms": r["p99_ms"], "mean_ms": r["mean_ms"],
                             "mean_admission_wait_ms": r["mean_admission_wait_ms"],
                             "mean_batch": r["mean_batch"], "pairs_per_s": r["pairs_per_s"],
                             "jobs": r["jobs"], "failed": r["failed"], "rejected": r["rejected"],
                             "nl_retries": r["nl_retries"], "peak_hbm_bytes": r["peak_hbm_bytes"]})
        log(f"served at {f:.2f} x capacity: {out['rates'][-1]}")
    del buf, xs
    return out


def sweep_forms(clm, cl, xt, sigma, eps, reps=5):
    """Sweep-kernel time of the FP32+guard LJ forces in its three forms:
    the half-shell sweep (every pair once) with and without the pruning of
    candidates by the tile's bounding box, and the full-shell gather."""
    import torch
    out = {}
    for key, kw in (("half_pruned_ms", dict(half=True, prune=True)),
                    ("half_unpruned_ms", dict(half=True, prune=False)),
                    ("full_shell_ms", dict(half=False))):
        cl.lj_forces(sigma, eps, **kw)
        torch.cuda.synchronize()
        clm.set_timing(True)
        clm.stats(reset=True)
        for _ in range(reps):
            cl.lj_forces(sigma, eps, **kw)
        st = clm.stats(reset=True)
        clm.set_timing(False)
        out[key] = st["sweep_ms"] / max(st["sweeps"], 1)
        if key == "half_pruned_ms":
            info = cl.info()
            out["half_pairs_tested"] = info["half_pairs_tested"]
            out["half_pairs_kept"] = info["half_pairs_kept"]
    return out


def build_roofline(clm, W, n, lcell, steps=5, lcell_x=None):
    """Build-only timing (count + scan + bucket + place + tiles) of n uniform particles
    in the headline triclinic box shape scaled to the same density."""
    import numpy as np
    import torch
    c = W.config2(n=1000)
    H = c["H"] * (n / 1_000_000) ** (1.0 / 3.0)
    x = W.uniform_in_box(n, H, 21)
    xt = torch.from_numpy(x).to("cuda:0")
    del x
    cl = clm.CellList(xt, clm.Box(H, c["cutoff"], lcell, lcell_x), precision="fp32")
    for _ in range(2):
        cl.build(xt)
    torch.cuda.synchronize()
    clm.set_timing(True)
    clm.stats(reset=True)
    for _ in range(steps):
        cl.build(xt)
    torch.cuda.synchronize()
    st = clm.stats(reset=True)
    clm.set_timing(False)
    ms = st["build_ms"] / max(st["builds"], 1)
    gbs = BUILD_BYTES_PER_PARTICLE * n / (ms * 1e-3) / 1e9
    del cl, xt
    torch.cuda.empty_cache()
    return {"n": n, "build_ms": ms, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}


def md_cases(steps):
    """Neon fluid MD (100 atoms/nm^3, rc 1.2 nm, 1 fs, rescaling every 10
    steps) at 10^4, 10^5 and 10^6 atoms: the paper's protocol (cell list rebuilt
    every step, FP32+guard sweep forces) against the Verlet pair list (skin
    0.1 nm, FP64 forces), timed on the host clock around `steps` steps."""
    import time
    import torch
    import paper_2202_06427_amd.md as md
    import workloads as W
    out = {}
    for n in (10_000, 100_000, 1_000_000):
        w = W.neon_fluid(n, seed=6)
        target = 0.5 * (3 * n - 3) * W.KB * w["temperature"]
        row = {}
        for mode in ("rebuild", "verlet"):
            kw = dict(cutoff=w["cutoff"], sigma=w["sigma"], epsilon=w["epsilon"], mass=w["mass"],
                      dt=w["dt"], mode=mode, skin=0.1, rescale_every=10, target_ke=target,
                      precision="fp32")
            x = torch.from_numpy(w["x"]).to("cuda:0")
            v = torch.from_numpy(w["v"]).to("cuda:0")
            md.run(x, v, w["H"], nsteps=20, **kw)  # warm-up (kernels loaded)
            x = torch.from_numpy(w["x"]).to("cuda:0")
            v = torch.from_numpy(w["v"]).to("cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = md.run(x, v, w["H"], nsteps=steps, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            pairs = int(r["count"][1:].sum().item())
            e = {"ms_per_step": 1e3 * dt / steps, "ns_per_day": steps * w["dt"] * 1e-3 / dt * 86400,
                 "pairs_per_s": pairs / dt}
            if mode == "verlet":
                info = r["list"].info()
                e.update({"skin_nm": 0.1, "rebuilds": info["rebuilds"], "list_entries": info["entries"],
                          "overflow": info["overflow"]})
            row[mode] = e
        row["verlet_speedup"] = row["rebuild"]["ms_per_step"] / row["verlet"]["ms_per_step"]
        out[w["name"]] = row
    return out


def kclosest_cases(reps=5):
    """k closest cross pairs (Code 8) on the cross-set workload (5000 blob
    particles against 5*10^5 uniform ones, box 170, cutoff 5), FP32+guard
    cell list: milliseconds per query (cell list built once)."""
    import time
    import torch
    import paper_2202_06427_amd as clm
    import workloads as W
    cfg = W.config3()
    x = torch.from_numpy(cfg["x"]).to("cuda:0")
    y = torch.from_numpy(cfg["y"]).to("cuda:0")
    cl = clm.CellList(x, clm.Box(cfg["H"], cfg["cutoff"], 2), y=y, precision="fp32")
    pairs = int(cl.count().item())
    out = {"workload": cfg["name"], "pairs_within_cutoff": pairs}
    for k in (5, 1000):
        cl.kclosest(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            i, j, d2 = cl.kclosest(k)
        torch.cuda.synchronize()
        out[f"k{k}_ms"] = 1e3 * (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        cl.count()
    torch.cuda.synchronize()
    out["one_count_sweep_ms"] = 1e3 * (time.perf_counter() - t0) / reps
    return out


def nonperiodic_cases(reps=5):
    """The neighbour-list benchmark of section 4.1: pairs within 1.2 nm
    between a set of 10..10^5 particles and one of 10^6 (100 per nm^3, no
    periodic boundaries).  Whole call (extrema, bounding box, cell lists of
    both sets, list with distances), FP32+guard, host clock."""
    import time
    import torch
    import paper_2202_06427_amd as clm
    import workloads as W
    out = {}
    for n_small in (10, 100, 1000, 10_000, 100_000):
        w = W.e1_sets(n_small)
        x = torch.from_numpy(w["x"]).to("cuda:0")
        y = torch.from_numpy(w["y"]).to("cuda:0")
        pairs, _ = clm.neighbor_list_nonperiodic(x, w["cutoff"], y=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pairs, _ = clm.neighbor_list_nonperiodic(x, w["cutoff"], y=y)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[str(n_small)] = {"ms": 1e3 * dt, "pairs": int(pairs.shape[0]), "pairs_per_s": pairs.shape[0] / dt}
    return {"workload": "e1 sets vs 10^6 (section 4.1), rc 1.2, 100/nm^3, non-periodic", "points": out}


def weighted_cases(reps=5):
    """The weighted maps: sum of m_i m_j / d (Code 5) on the 10^6-particle
    triclinic workload next to the plain sum of 1/d, and Code 10's
    distance-binned mean relative speed (10 bins) on the 2D clustered
    workload (2*10^6 points); FP32+guard, host clock around `reps` maps."""
    import time
    import torch
    import paper_2202_06427_amd as clm
    import workloads as W

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = f()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    out = {}
    cfg = W.config2()
    x = torch.from_numpy(cfg["x"]).to("cuda:0")
    cl = clm.CellList(x, clm.Box(cfg["H"], cfg["cutoff"], 2), precision="fp32")
    m = torch.from_numpy(W.rng(7).random(x.shape[0]) + 0.5).to("cuda:0")
    (e, c), dtw = timed(lambda: cl.sum_w_inv_d(m))
    (_, _), dtu = timed(lambda: cl.sum_inv_d())
    pairs = int(c.item())
    out["sum_w_inv_d"] = {"workload": cfg["name"] if "name" in cfg else "uniform-1e6-triclinic-rc12",
                          "ms": 1e3 * dtw, "pairs_per_s": pairs / dtw, "unweighted_ms": 1e3 * dtu}
    del cl
    cfg4 = W.config4()
    x4 = torch.from_numpy(cfg4["x"]).to("cuda:0")
    v4 = torch.from_numpy(cfg4["v"]).to("cuda:0")
    cl4 = clm.CellList(x4, clm.Box(cfg4["H"], cfg4["cutoff"], 2), precision="fp32")
    (h, sums, c4), dtv = timed(lambda: cl4.dist_vel_histogram(v4, 10))
    pairs4 = int(c4.item())
    out["dist_vel_hist"] = {"workload": cfg4["name"] if "name" in cfg4 else "2d-clustered-2e6",
                            "bins": 10, "ms": 1e3 * dtv, "pairs_per_s": pairs4 / dtv,
                            "mean_speed_first_bins": (sums[:3] / h[:3].to(torch.float64)).tolist()}
    return out


def pruning_cases(reps=5):
    """Candidate pruning of the half-shell LJ force sweep (FP32+guard): sweep
    time with and without pruning and of the full-shell gather, on the
    headline workload at lcell 1, 2 and 3, at lcell 2 with row-axis reach
    4, 6 and 8 (thinner cells along the row), and on the 2D clustered workload
    (2*10^6 points, rc 0.01, sigma 1e-4: about the spacing inside a
    cluster), with the half-shell candidate count of each grid."""
    import torch
    import paper_2202_06427_amd as clm
    import workloads as W

    out = {}
    cfg = W.config2()
    x = torch.from_numpy(cfg["x"]).to("cuda:0")
    for lc, lx in ((1, None), (2, None), (3, None), (2, 4), (2, 6), (2, 8)):
        cl = clm.CellList(x, clm.Box(cfg["H"], cfg["cutoff"], lc, lx), precision="fp32")
        forms = sweep_forms(clm, cl, x, cfg["sigma"], cfg["epsilon"], reps)
        info = cl.info()
        key = f"headline_lcell{lc}" + (f"_x{lx}" if lx else "")
        out[key] = {**forms, "half_shell_candidates": info["candidate_pairs"], "ntiles": info["ntiles"]}
        del cl
    del x
    cfg4 = W.config4()
    x4 = torch.from_numpy(cfg4["x"]).to("cuda:0")
    cl4 = clm.CellList(x4, clm.Box(cfg4["H"], cfg4["cutoff"], 2), precision="fp32")
    forms = sweep_forms(clm, cl4, x4, 1e-4, 1.0, reps)
    info = cl4.info()
    c = int(cl4.count().item())
    out["clustered2d_lcell2"] = {**forms, "half_shell_candidates": info["candidate_pairs"], "pairs": c,
                                 "near_evaluations": info["near_evaluations"]}
    return out


def md_only(n, steps):
    """Verlet-list MD of n Neon atoms (skin 0.1 nm) for `steps` steps."""
    import torch
    import paper_2202_06427_amd.md as md
    import workloads as W
    w = W.neon_fluid(n, seed=6)
    target = 0.5 * (3 * n - 3) * W.KB * w["temperature"]
    x = torch.from_numpy(w["x"]).to("cuda:0")
    v = torch.from_numpy(w["v"]).to("cuda:0")
    r = md.run(x, v, w["H"], cutoff=w["cutoff"], sigma=w["sigma"], epsilon=w["epsilon"], mass=w["mass"],
               dt=w["dt"], nsteps=steps, mode="verlet", skin=0.1, rescale_every=10, target_ke=target)
    torch.cuda.synchronize()
    print(json.dumps({"md_only": w["name"], "steps": steps, **r["list"].info()}), flush=True)


def measured_peaks(clm):
    """Device rates measured by the library's microbenchmarks (FMA chains
    without packed FP32, FP64 FMA chains, a 1 GiB device copy)."""
    out = {}
    for kind, key in (("fma_f32", "valu_fp32_tflops"), ("fma_f64", "valu_fp64_tflops"),
                      ("copy", "copy_GBs")):
        ms, work, rate = clm.calibrate(kind, nbytes=1 << 30, reps=10)
        out[key] = rate
        out[key.rsplit("_", 1)[0] + "_ms"] = ms
    return out


def cpu_model():
    """The CPU model string (lscpu's "Model name", else /proc/cpuinfo)."""
    import subprocess
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.strip().startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def usable_cpus():
    """CPUs this process may run on (what nproc prints)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def per_core_sample(W):
    """The headline density (10^6 particles per 215.4-box) in a box of half
    the lattice-vector lengths: 125,000 particles, the same angles, cutoff and
    LJ parameters, for the oracle on one thread."""
    H = 0.5 * W.triclinic_h(W.CFG2_LENGTHS, W.CFG2_ANGLES)
    x = W.rng(2).random((125_000, 3)) @ H.T
    return {"x": x, "H": H, "cutoff": 12.0, "sigma": 3.4, "epsilon": 0.238}


def lattice_accuracy(clm, W, nthreads):
    """FP32+guard LJ energy and forces (half-shell sweep) on the jittered
    lattice of the headline box against the oracle: energy relative error and
    the largest per-particle force error relative to the sum of that
    particle's pair-force magnitudes."""
    import numpy as np
    import torch

    import oracle
    c = W.config2(variant="lattice")
    s, e = c["sigma"], c["epsilon"]
    xt = torch.from_numpy(c["x"]).to("cuda:0")
    cl = clm.CellList(xt, clm.Box(c["H"], c["cutoff"], 2), precision="fp32")
    out = cl.lj_forces(s, e)
    F = out["forces"].cpu().numpy()
    E = out["energy"].item()
    ref = oracle.compute(c["x"], c["H"], c["cutoff"], lj=(s, e), lj_grad=True, lj_fabs=True,
                         nthreads=nthreads)
    err = np.linalg.norm(F + ref["lj_grad"], axis=1) / np.maximum(ref["lj_fabs"], 1e-300)
    return {"workload": c["name"], "energy_rel_err": abs(E - ref["lj_energy"]) / abs(ref["lj_energy"]),
            "max_force_err": float(err.max()), "mean_force_err": float(err.mean()),
            "near_pair_evaluations": cl.info()["near_evaluations"], "pairs": ref["count"]}


def cpu_baseline(cfg, nthreads):
    import oracle
    t0 = time.perf_counter()
    r = oracle.compute(cfg["x"], cfg["H"], cfg["cutoff"], lj=(cfg["sigma"], cfg["epsilon"]),
                       lj_grad=True, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return r, dt


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.build_only:
        import paper_2202_06427_amd as clm
        import workloads as W
        print(json.dumps({"build_only": build_roofline(clm, W, args.build_only, args.lcell,
                                                       lcell_x=args.lcell_x or None)}), flush=True)
        return
    if args.md_only:
        md_only(args.md_only, args.steps)
        return
    if args.section:
        f = {"kclosest": kclosest_cases, "nonperiodic": nonperiodic_cases, "weighted": weighted_cases,
             "pruning": pruning_cases}
        print(json.dumps({"section": args.section, **f[args.section]()}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (single-GPU workload; no collectives). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2202_06427_amd as clm
    import workloads as W

    cfg = W.config2(n=args.n)
    sigma, eps = cfg["sigma"], cfg["epsilon"]
    xt = torch.from_numpy(cfg["x"]).to("cuda:0")
    box = clm.Box(cfg["H"], cfg["cutoff"], args.lcell, args.lcell_x or None)
    binfo = box.info()
    log(f"box grid {binfo['grid']} lcell {binfo['lcell']} lcell_x {binfo['lcell_x']} "
        f"band {binfo['guard_band']:.3e}")

    res = {}
    for prec in (["fp32"] if args.no_fp64 else ["fp32", "fp64"]):
        cl = clm.CellList(xt, box, precision=prec)
        r = time_steps(clm, cl, xt, args.steps, args.warmup, sigma, eps, args.step_samples)
        info = cl.info()  # after the timed steps: re-evaluation counts of the last map
        r["info"] = info
        if prec == "fp32" and args.sweep_forms:
            r["forms"] = sweep_forms(clm, cl, xt, sigma, eps)
            log(f"fp32 sweep forms: {r['forms']}")
        res[prec] = r
        log(f"{prec}: {r['ms_per_step']:.3f} ms/step (sweep {r['sweep_ms']:.3f} ms, build "
            f"{r['build_ms']:.3f} ms) pairs {r['count']} cand(half) {info['candidate_pairs']}")
        del cl
        torch.cuda.empty_cache()

    main_r = res["fp32"]
    pairs = main_r["count"]
    guard = main_r["info"]
    value = pairs / (main_r["ms_per_step"] * 1e-3)
    cand = main_r["info"]["candidate_pairs"]
    flops = cand * FLOPS_PER_CANDIDATE + pairs * FLOPS_PER_LJ_PAIR
    achieved = flops / (main_r["sweep_ms"] * 1e-3) / 1e12
    line = {
        "metric": "within-cutoff pairs/s at 1M particles, FP32 vs FP64; served p50/p99 latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "uniform-1e6-triclinic-215.4-80/95/100-rc12 LJ energy+forces (bin + sweep + reduce)",
            "n": args.n, "cutoff": cfg["cutoff"], "lcell": binfo["lcell"], "lcell_x": binfo["lcell_x"],
            "grid": binfo["grid"],
            "sigma": sigma, "epsilon": eps, "pairs": pairs, "candidate_pairs_half_shell": cand,
        },
        "phases_ms": {"build": main_r["build_ms"], "sweep": main_r["sweep_ms"]},
        "roofline": {
            "bound": "alu",
            "kernel": "half_lj_kernel<3,false> (FP32+guard LJ forces, half shell, pruned)",
            "achieved": achieved,
            "peak": VALU_FP32_NONPACKED_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / VALU_FP32_NONPACKED_TFLOPS,
            "traffic": measured_traffic(),
            "traffic_unit": "bytes/launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "flops_per_launch": flops,
            "frac_in_cutoff_only": pairs * FLOPS_PER_LJ_PAIR / (main_r["sweep_ms"] * 1e-3) / 1e12
            / VALU_FP32_NONPACKED_TFLOPS,
            "peak_if_packed_fp32": VALU_FP32_PACKED_TFLOPS,
            "target_frac": 0.5,
            "target_met": achieved / VALU_FP32_NONPACKED_TFLOPS >= 0.5,
        },
        "sweep_forms_ms": main_r.get("forms"),
        "half_sweep_pairs": {"tested": guard["half_pairs_tested"], "kept_after_pruning": guard["half_pairs_kept"],
                             "kept_fraction": guard["half_pairs_kept"] / max(guard["half_pairs_tested"], 1),
                             "in_cutoff_fraction_of_kept": pairs / max(guard["half_pairs_kept"], 1)},
        "guard": {"band_retests": guard["guard_retests"], "near_pair_evaluations": guard["near_evaluations"],
                  "fraction_of_pairs": (guard["guard_retests"] + guard["near_evaluations"]) / max(2 * pairs, 1)},
    }
    b1 = {"n": args.n, "build_ms": main_r["build_ms"],
          "algorithmic_GBs": BUILD_BYTES_PER_PARTICLE * args.n / (main_r["build_ms"] * 1e-3) / 1e9}
    b1["frac"] = b1["algorithmic_GBs"] / HBM_PEAK_GBS
    line["build_roofline"] = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "bytes_per_particle": BUILD_BYTES_PER_PARTICLE, "points": [b1]}
    if args.build_n_large > 0:
        log(f"build-only timing at n={args.build_n_large} ...")
        line["build_roofline"]["points"].append(build_roofline(clm, W, args.build_n_large, args.lcell,
                                                               lcell_x=args.lcell_x or None))
    line["step_ms_median"] = main_r["step_ms_median"]
    line["step_ms_min"] = main_r["step_ms_min"]
    if args.calibrate:
        log("measured device rates (FMA chains, copy) ...")
        mp = measured_peaks(clm)
        line["measured_peaks"] = mp
        line["roofline"]["frac_of_measured_peak"] = achieved / mp["valu_fp32_tflops"]
        line["build_roofline"]["frac_of_measured_copy"] = b1["algorithmic_GBs"] / mp["copy_GBs"]
        log(f"measured: {mp}")
    if "fp64" in res:
        r64 = res["fp64"]
        line["fp64"] = {
            "value": r64["count"] / (r64["ms_per_step"] * 1e-3),
            "ms_per_step": r64["ms_per_step"],
            "sweep_ms": r64["sweep_ms"],
            "build_ms": r64["build_ms"],
            "pairs": r64["count"],
            "energy": r64["energy"],
            "step_ms_median": r64["step_ms_median"],
            "step_ms_min": r64["step_ms_min"],
        }
        a64 = flops / (r64["sweep_ms"] * 1e-3) / 1e12
        line["fp64"]["roofline"] = {"bound": "alu", "achieved": a64, "peak": VALU_FP64_TFLOPS,
                                    "unit": "TFLOP/s", "frac": a64 / VALU_FP64_TFLOPS}
        if "measured_peaks" in line:
            line["fp64"]["roofline"]["frac_of_measured_peak"] = a64 / line["measured_peaks"]["valu_fp64_tflops"]
        line["fp32_over_fp64"] = value / line["fp64"]["value"]
        line["energy_rel_diff_fp32_fp64"] = abs(main_r["energy"] - r64["energy"]) / abs(r64["energy"])
    if args.serve_requests > 0:
        log(f"served mix: {args.serve_requests} requests ...")
        fracs = [float(f) for f in args.serve_fracs.split(",") if f]
        line["served"] = served(args.serve_requests, fracs)
        log(f"served: {line['served']}")
    if args.md_steps > 0:
        log(f"Neon MD: {args.md_steps} steps at 1e4, 1e5 and 1e6 atoms ...")
        line["md"] = md_cases(args.md_steps)
        log(f"md: {line['md']}")
    if args.weighted:
        log("weighted maps ...")
        line["weighted_maps"] = weighted_cases()
        log(f"weighted: {line['weighted_maps']}")
    if args.pruning:
        log("pruning: sweep forms at lcell 1/2/3 and on the 2D clustered workload ...")
        line["pruning"] = pruning_cases()
        log(f"pruning: {line['pruning']}")
    if args.kclosest:
        log("k closest pairs ...")
        line["kclosest"] = kclosest_cases()
        log(f"kclosest: {line['kclosest']}")
    if args.nonperiodic:
        log("non-periodic neighbour lists ...")
        line["nonperiodic_nl"] = nonperiodic_cases()
        log(f"nonperiodic: {line['nonperiodic_nl']}")
    if not args.no_cpu_baseline:
        nproc = usable_cpus()
        nth = args.cpu_threads or nproc
        log(f"cpu baseline: oracle on the full workload with {nth} threads ...")
        r, dt = cpu_baseline(cfg, nth)
        line["cpu_baseline"] = {
            "value": r["count"] / dt,
            "unit": "pairs/s",
            "cores": nth,
            "kind": "oracle",
            "sample": f"the full workload once (n={args.n}, LJ energy+forces, FP64 plain cell list), {dt:.1f} s",
            "pairs": r["count"],
            "pairs_match_gpu": r["count"] == pairs,
            "energy_rel_err_fp32": abs(main_r["energy"] - r["lj_energy"]) / abs(r["lj_energy"]),
            "nproc": nproc,
            "os_cpu_count": os.cpu_count(),
            "cpu_model": cpu_model(),
        }
        if nth != 16 and nproc >= 16:
            r16, dt16 = cpu_baseline(cfg, 16)
            line["cpu_baseline"]["threads_16"] = {"value": r16["count"] / dt16, "unit": "pairs/s",
                                                  "seconds": dt16}
        log("cpu baseline: oracle on one thread (per-core figure) ...")
        pc = per_core_sample(W)
        r1, dt1 = cpu_baseline(pc, 1)
        line["cpu_baseline"]["per_core"] = {
            "value": r1["count"] / dt1, "unit": "pairs/s", "threads": 1,
            "sample": f"125,000 particles at the headline density (box of half the lengths), {dt1:.1f} s",
            "pairs": r1["count"]}
        # the FP32 accuracy where FP32 evaluates most pairs: the jittered
        # lattice (on uniform points the energy is a few overlapping pairs,
        # evaluated in FP64 by the near-pair guard)
        log("fp32 accuracy on the jittered-lattice variant against the oracle ...")
        line["cpu_baseline"]["fp32_accuracy_lattice"] = lattice_accuracy(clm, W, nth)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
