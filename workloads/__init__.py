"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the pair-map method: it only draws
positions, velocities, boxes and request streams (numpy PCG64 streams with
fixed seeds).  Both the GPU library's tests/benchmark and the CPU oracle
consume these arrays.  The paper's own toy generators (``xatomic``,
``xgalactic``, section 3) are not defined in the paper, so these stand-ins
reproduce only the shapes the paper describes: water-like atomic density
(sections 4.1, 4.2, 4.4), clustered galaxy-like points with velocities
(section 4.3), and two disjoint sets (section 4.1).
"""
import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def triclinic_h(lengths, angles_deg):
    """Unit-cell matrix (columns = lattice vectors) from lengths and angles.

    alpha = angle(b, c), beta = angle(a, c), gamma = angle(a, b); a along x,
    b in the xy plane (the usual crystallographic construction).
    """
    la, lb, lc = (float(v) for v in lengths)
    al, be, ga = (math.radians(float(v)) for v in angles_deg)
    cy = (math.cos(al) - math.cos(be) * math.cos(ga)) / math.sin(ga)
    cz2 = 1.0 - math.cos(be) ** 2 - cy ** 2
    if cz2 <= 0:
        raise ValueError("invalid cell angles")
    a = [la, 0.0, 0.0]
    b = [lb * math.cos(ga), lb * math.sin(ga), 0.0]
    c = [lc * math.cos(be), lc * cy, lc * math.sqrt(cz2)]
    return np.array([a, b, c], dtype=np.float64).T.copy()


def uniform_in_box(n, H, seed):
    """n points uniform in the cell spanned by H: r = H s, s ~ U[0,1)^dim."""
    g = rng(seed)
    dim = H.shape[0]
    s = g.random((n, dim))
    return np.ascontiguousarray(s @ np.asarray(H, dtype=np.float64).T)


def config1(seed=1):
    """Plain FP64 case: 10^4 uniform points in a cube of side 46.42, rc 8."""
    g = rng(seed)
    side = 46.42
    x = side * g.random((10_000, 3))
    return {"name": "uniform-1e4-cube46.42-rc8", "x": x, "H": np.diag([side] * 3),
            "cutoff": 8.0}


CFG2_LENGTHS = (215.4, 215.4, 215.4)
CFG2_ANGLES = (80.0, 95.0, 100.0)


def config2(seed=2, n=1_000_000, variant="uniform"):
    """10^6 uniform points in a triclinic cell (215.4; 80/95/100 deg), rc 12, LJ.

    variant "far": the same points shifted by H (1000, -700, 300);
    variant "lattice": a jittered simple-cubic-like lattice in fractional
    coordinates (no near-coincident pairs), same box and count.
    """
    g = rng(seed)
    H = triclinic_h(CFG2_LENGTHS, CFG2_ANGLES)
    if variant == "lattice":
        m = int(round(n ** (1.0 / 3.0)))
        grid = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                        axis=-1).reshape(-1, 3).astype(np.float64)
        s = (grid + 0.5 + 0.1 * (g.random(grid.shape) - 0.5)) / m
    else:
        s = g.random((n, 3))
    x = s @ H.T
    if variant == "far":
        x = x + (H @ np.array([1000.0, -700.0, 300.0]))[None, :]
    return {"name": f"uniform-{len(x)}-triclinic215.4-rc12-{variant}", "x": np.ascontiguousarray(x),
            "H": H, "cutoff": 12.0, "sigma": 3.4, "epsilon": 0.238}


def config3(seed=3, n_solute=5000, n_solvent=500_000):
    """Cross set: Gaussian solute blob (sigma 10) and uniform solvent, cube 170, rc 5."""
    g = rng(seed)
    side = 170.0
    x = np.mod(g.normal(85.0, 10.0, size=(n_solute, 3)), side)
    y = side * g.random((n_solvent, 3))
    return {"name": "cross-5e3blob-5e5uniform-cube170-rc5", "x": x, "y": y,
            "H": np.diag([side] * 3), "cutoff": 5.0}


def config4(seed=4, n=2_000_000, n_clusters=200, sigma=0.005, background=0.2):
    """2D clustered points in the unit square with N(0,1) velocities, rc 0.01."""
    g = rng(seed)
    n_bg = int(round(background * n))
    per = (n - n_bg) // n_clusters
    n_cl = per * n_clusters
    centres = g.random((n_clusters, 2))
    pts = centres[np.repeat(np.arange(n_clusters), per)] + g.normal(0.0, sigma, size=(n_cl, 2))
    bg = g.random((n - n_cl, 2))
    x = np.mod(np.concatenate([pts, bg]), 1.0)
    perm = g.permutation(n)
    x = np.ascontiguousarray(x[perm])
    v = g.normal(0.0, 1.0, size=(n, 2))
    return {"name": "2d-clustered-2e6-unitsquare-rc0.01", "x": x, "v": v, "H": np.eye(2),
            "cutoff": 0.01, "rel_nbins": 256, "rel_hi": 8.0}


def random_box(g, dim, volume, triclinic):
    """A random orthorhombic or triclinic box of the given volume."""
    aspect = np.exp(g.uniform(-0.2, 0.2, size=dim))
    if not triclinic:
        L = aspect * (volume / np.prod(aspect)) ** (1.0 / dim)
        return np.diag(L)
    while True:
        if dim == 2:
            ang = g.uniform(70.0, 110.0)
            la, lb = aspect
            H = np.array([[la, lb * math.cos(math.radians(ang))],
                          [0.0, lb * math.sin(math.radians(ang))]])
        else:
            ang = g.uniform(70.0, 110.0, size=3)
            try:
                H = triclinic_h(aspect, ang)
            except ValueError:
                continue
        scale = (volume / abs(np.linalg.det(H))) ** (1.0 / dim)
        return H * scale


def serve_requests(seed=5, count=10_000, density=0.1, n_lo=1_000, n_hi=200_000,
                   rc_lo=6.0, rc_hi=12.0):
    """Request stream descriptors for the served mix (positions drawn lazily).

    Each request: particle count log-uniform in [n_lo, n_hi], a random
    orthorhombic or triclinic box at the given density, a cutoff uniform in
    [rc_lo, rc_hi], a map kind uniform over {lj, nl, gr}, and a position
    seed.  Inter-arrival times are drawn by the caller for a chosen rate.
    """
    g = rng(seed)
    reqs = []
    for k in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        tri = bool(g.random() < 0.5)
        H = random_box(g, 3, n / density, tri)
        rc = float(g.uniform(rc_lo, rc_hi))
        kind = ("lj", "nl", "gr")[int(g.integers(0, 3))]
        reqs.append({"id": k, "n": n, "H": H, "cutoff": rc, "kind": kind,
                     "pos_seed": int(g.integers(0, 2 ** 62))})
    return reqs


def request_positions(req):
    return uniform_in_box(req["n"], req["H"], req["pos_seed"])


# Neon fluid of the paper's MD comparison (section 4.2): 100 atoms per nm^3,
# orthorhombic (cubic) periodic box, cutoff 1.2 nm, time step 1 fs, velocity
# rescaling every 10 steps.  Units: nm, ps, amu, kJ/mol (force kJ/mol/nm, so
# force / mass is in nm/ps^2).  The paper names CHARMM parameters without
# giving values; these are common Neon Lennard-Jones values.
NEON = {"sigma": 0.2749, "epsilon": 0.2960, "mass": 20.1797, "cutoff": 1.2, "dt": 0.001,
        "density": 100.0, "temperature": 300.0, "rescale_every": 10}
KB = 0.0083144626  # kJ/mol/K


def neon_fluid(n, seed=6, jitter=0.02):
    """n Neon atoms in a cube at 100 atoms/nm^3: n distinct sites drawn from
    the smallest simple-cubic lattice with at least n sites, each displaced
    by up to +-jitter/2 of the lattice spacing, with Maxwell-Boltzmann
    velocities at 300 K and zero total momentum.  Returns x (n, 3), v (n, 3),
    H (3, 3) and the parameters."""
    g = rng(seed)
    m = int(round(n ** (1.0 / 3.0)))
    while m ** 3 < n:
        m += 1
    side = (n / NEON["density"]) ** (1.0 / 3.0)
    a = side / m
    grid = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                    -1).reshape(-1, 3).astype(np.float64)
    grid = grid[np.sort(g.choice(m ** 3, size=n, replace=False))]
    x = (grid + 0.5 + jitter * (g.random((n, 3)) - 0.5)) * a
    sd = math.sqrt(KB * NEON["temperature"] / NEON["mass"])
    v = g.normal(0.0, sd, size=(n, 3))
    v -= v.mean(axis=0)
    return {"name": f"neon-{n}-rho100-rc1.2", "x": np.ascontiguousarray(x),
            "v": np.ascontiguousarray(v), "H": np.diag([side] * 3), **NEON}


def e1_sets(n_small, n_large=1_000_000, seed=9, density=100.0):
    """The neighbour-list benchmark of the paper's section 4.1: two disjoint
    sets at 100 particles per nm^3 (cutoff 1.2 nm) without periodic
    boundaries: n_large points uniform in a cube of side (n_large /
    density)^(1/3) nm and n_small points uniform in a cube of side
    (n_small / density)^(1/3) nm centred in it."""
    g = rng(seed)
    big = (n_large / density) ** (1.0 / 3.0)
    small = (n_small / density) ** (1.0 / 3.0)
    y = big * g.random((n_large, 3))
    x = 0.5 * (big - small) + small * g.random((n_small, 3))
    return {"name": f"e1-{n_small}-vs-{n_large}-rho100-rc1.2-nonperiodic", "x": x, "y": y,
            "cutoff": 1.2}
