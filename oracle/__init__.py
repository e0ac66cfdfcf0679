"""Plain FP64 CPU oracle for the cell-list pair map (arXiv 2202.06427).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  The
arithmetic lives in ``clmo.cpp`` (plain C++17 + OpenMP, FP64, no fused
multiply-add); this module only marshals numpy arrays through ctypes.

Every function follows the paper's statement of the problem: a periodic box
with unit-cell matrix H whose columns are the lattice vectors (section 2.5,
Code 3), a cutoff, and a map applied to every pair within the cutoff under
the minimum-image convention (sections 2.3 and 2.8), reduced per call.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

W_COUNT, W_SUM_D, W_SUM_INV_D, W_LJ, W_HIST_DIST, W_HIST_REL, W_NL = 1, 2, 4, 8, 16, 32, 64
W_SUM_W_INV_D, W_HIST_DIST_VEL = 128, 256
METHOD_AUTO, METHOD_BRUTE, METHOD_CELLS = -1, 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)


class _Request(ctypes.Structure):
    _fields_ = [
        ("want", ctypes.c_int), ("method", ctypes.c_int), ("nthreads", ctypes.c_int),
        ("sigma", ctypes.c_double), ("epsilon", ctypes.c_double),
        ("hist_nbins", ctypes.c_int), ("hist_hi", ctypes.c_double),
        ("rel_nbins", ctypes.c_int), ("rel_hi", ctypes.c_double),
        ("vel_x", _dp), ("vel_y", _dp), ("nl_capacity", ctypes.c_int64),
        ("frame_x", _i64p), ("weights_x", _dp), ("weights_y", _dp),
        ("dv_nbins", ctypes.c_int), ("dv_hi", ctypes.c_double),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64), ("sum_d", ctypes.c_double), ("sum_inv_d", ctypes.c_double),
        ("lj_energy", ctypes.c_double), ("virial", ctypes.c_double * 9),
        ("dEdH", ctypes.c_double * 9), ("lj_grad", _dp), ("hist", _u64p),
        ("rel_hist", _u64p), ("rel_sum", _dp), ("nl_i", _i64p), ("nl_j", _i64p),
        ("nl_d", _dp), ("nl_count", ctypes.c_uint64), ("method_used", ctypes.c_int),
        ("nl_d2", _dp), ("sum_w_inv_d", ctypes.c_double), ("dv_hist", _u64p), ("dv_sum", _dp),
        ("lj_fabs", _dp),
    ]


_lib = None


def lib():
    """Load liboracle.so (built by ``oracle/build.py``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library missing: {_LIB_PATH} (run oracle/build.py)")
        L = ctypes.CDLL(_LIB_PATH)
        L.clmo_box_inverse.argtypes = [ctypes.c_int, _dp, _dp]
        L.clmo_box_widths.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.clmo_box_from_lengths_angles.argtypes = [_dp, _dp, _dp]
        L.clmo_wrap.argtypes = [ctypes.c_int, _dp, ctypes.c_int64, _dp, _dp, _dp, _i64p]
        L.clmo_pair_d2.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _ip]
        L.clmo_pair_d2.restype = ctypes.c_double
        L.clmo_compute.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, ctypes.c_int64, _dp,
                                   ctypes.c_int64, ctypes.POINTER(_Request), ctypes.POINTER(_Result)]
        L.clmo_lj_sample.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, ctypes.c_int64, _i64p,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     _dp, _dp]
        L.clmo_neighbors_of.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, _i64p, _ip, _i64p]
        L.clmo_paper_ghost_grid.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {rc})")


def box_inverse(H):
    H = _f64(H)
    dim = H.shape[0]
    out = np.zeros((dim, dim))
    _check(lib().clmo_box_inverse(dim, _p(H), _p(out)), "box_inverse")
    return out


def box_widths(H):
    H = _f64(H)
    dim = H.shape[0]
    w = np.zeros(dim)
    V = ctypes.c_double(0.0)
    _check(lib().clmo_box_widths(dim, _p(H), _p(w), ctypes.byref(V)), "box_widths")
    return w, V.value


def box_from_lengths_angles(lengths, angles_deg):
    L = _f64(lengths)
    A = _f64(angles_deg)
    H = np.zeros((3, 3))
    _check(lib().clmo_box_from_lengths_angles(_p(L), _p(A), _p(H)), "box_from_lengths_angles")
    return H


def wrap(x, H):
    """Canonical wrap: (wrapped positions, fractional coordinates, wrap ints)."""
    x = _f64(x)
    H = _f64(H)
    n, dim = x.shape
    xw = np.zeros_like(x)
    fr = np.zeros_like(x)
    w = np.zeros((n, dim), dtype=np.int64)
    _check(lib().clmo_wrap(dim, _p(H), n, _p(x), _p(xw), _p(fr), _p(w, _i64p)), "wrap")
    return xw, fr, w


def pair_d2(xi, xj, H, reach):
    """Minimum-image squared distance of one pair and its raw-coordinate image K."""
    H = _f64(H)
    dim = H.shape[0]
    xi = _f64(xi)
    xj = _f64(xj)
    K = np.zeros(dim, dtype=np.intc)
    d2 = lib().clmo_pair_d2(dim, _p(H), _p(xi), _p(xj), float(reach), _p(K, _ip))
    return d2, K


def compute(x, H, cutoff, y=None, *, count=True, sum_d=False, sum_inv_d=False, lj=None,
            lj_grad=False, hist=None, rel_hist=None, vel_x=None, vel_y=None, nl=False,
            nl_capacity=None, method=METHOD_AUTO, nthreads=0, frame=None, weights=None,
            dist_vel_hist=None, lj_fabs=False):
    """Run the oracle; returns a dict of the requested outputs.

    lj = (sigma, epsilon); hist = (nbins, hi); rel_hist = (nbins, hi) with
    vel_x (and vel_y for a cross set).  Neighbour-list indices are 0-based,
    sorted by (i, j); single set has i < j.  frame: (nx, dim) integers that
    replace the canonical wrap integers (positions kept in the wrap of an
    earlier step; single set only).  weights = (w_x, w_y or None): the sum
    of w_i w_j / d (Code 5).  dist_vel_hist = (nbins, hi) with vel_x (and
    vel_y): pairs per distance bin and the per-bin sum of |v_j - v_i| (Code 10).
    lj_fabs (with lj_grad): per particle, the sum over its pairs of the pair-force
    magnitude |f_s| d -- the scale against which per-particle force errors are measured.
    """
    x = _f64(x)
    H = _f64(H)
    nx, dim = x.shape
    if H.shape != (dim, dim):
        raise ValueError("H must be dim x dim")
    yy = None if y is None else _f64(y)
    ny = 0 if yy is None else yy.shape[0]
    req = _Request()
    want = 0
    if count:
        want |= W_COUNT
    if sum_d:
        want |= W_SUM_D
    if sum_inv_d:
        want |= W_SUM_INV_D
    if lj is not None:
        want |= W_LJ
        req.sigma, req.epsilon = float(lj[0]), float(lj[1])
    if hist is not None:
        want |= W_HIST_DIST
        req.hist_nbins, req.hist_hi = int(hist[0]), float(hist[1])
    vx = vy = None
    if rel_hist is not None:
        want |= W_HIST_REL
        req.rel_nbins, req.rel_hi = int(rel_hist[0]), float(rel_hist[1])
        vx = _f64(vel_x)
        req.vel_x = _p(vx)
        if yy is not None:
            vy = _f64(vel_y)
            req.vel_y = _p(vy)
    if nl:
        want |= W_NL
    wx = wy = None
    if weights is not None:
        want |= W_SUM_W_INV_D
        wx = _f64(weights[0])
        req.weights_x = _p(wx)
        if yy is not None:
            wy = _f64(weights[1])
            req.weights_y = _p(wy)
    if dist_vel_hist is not None:
        want |= W_HIST_DIST_VEL
        req.dv_nbins, req.dv_hi = int(dist_vel_hist[0]), float(dist_vel_hist[1])
        if vx is None:
            vx = _f64(vel_x)
            req.vel_x = _p(vx)
            if yy is not None:
                vy = _f64(vel_y)
                req.vel_y = _p(vy)
    req.want = want
    req.method = method
    req.nthreads = nthreads
    fr = None
    if frame is not None:
        fr = np.ascontiguousarray(frame, dtype=np.int64)
        if fr.shape != (nx, dim):
            raise ValueError("frame must be (nx, dim) integers")
        req.frame_x = _p(fr, _i64p)
    res = _Result()
    keep = []
    grad = None
    fabs = None
    if lj is not None and lj_grad:
        grad = np.zeros((nx, dim))
        res.lj_grad = _p(grad)
        if lj_fabs:
            fabs = np.zeros(nx)
            res.lj_fabs = _p(fabs)
    h = None
    if hist is not None:
        h = np.zeros(req.hist_nbins + 1, dtype=np.uint64)
        res.hist = _p(h, _u64p)
    rh = rs = None
    if rel_hist is not None:
        rh = np.zeros(req.rel_nbins + 1, dtype=np.uint64)
        rs = np.zeros(req.rel_nbins)
        res.rel_hist = _p(rh, _u64p)
        res.rel_sum = _p(rs)
    nli = nlj = nld = None
    if nl:
        cap = int(nl_capacity) if nl_capacity is not None else None
        if cap is None:
            # first pass for the count, then the list
            r0 = compute(x, H, cutoff, yy, count=True, method=method, nthreads=nthreads,
                         frame=frame)
            cap = int(r0["count"])
        req.nl_capacity = cap
        nli = np.zeros(max(cap, 1), dtype=np.int64)
        nlj = np.zeros(max(cap, 1), dtype=np.int64)
        nld = np.zeros(max(cap, 1))
        nld2 = np.zeros(max(cap, 1))
        res.nl_i, res.nl_j, res.nl_d, res.nl_d2 = _p(nli, _i64p), _p(nlj, _i64p), _p(nld), _p(nld2)
    dvh = dvs = None
    if dist_vel_hist is not None:
        dvh = np.zeros(req.dv_nbins + 1, dtype=np.uint64)
        dvs = np.zeros(req.dv_nbins)
        res.dv_hist = _p(dvh, _u64p)
        res.dv_sum = _p(dvs)
    keep.append((vx, vy, fr, wx, wy))
    rc = lib().clmo_compute(dim, _p(H), float(cutoff), _p(x), nx, _p(yy), ny,
                            ctypes.byref(req), ctypes.byref(res))
    _check(rc, "compute")
    out = {"count": int(res.count), "method": int(res.method_used)}
    if sum_d:
        out["sum_d"] = res.sum_d
    if sum_inv_d:
        out["sum_inv_d"] = res.sum_inv_d
    if lj is not None:
        out["lj_energy"] = res.lj_energy
        out["virial"] = np.array(res.virial[: dim * dim]).reshape(dim, dim)
        out["dEdH"] = np.array(res.dEdH[: dim * dim]).reshape(dim, dim)
        if grad is not None:
            out["lj_grad"] = grad
        if fabs is not None:
            out["lj_fabs"] = fabs
    if weights is not None:
        out["sum_w_inv_d"] = res.sum_w_inv_d
    if dist_vel_hist is not None:
        out["dv_hist"] = dvh
        out["dv_sum"] = dvs
    if hist is not None:
        out["hist"] = h
    if rel_hist is not None:
        out["rel_hist"] = rh
        out["rel_sum"] = rs
    if nl:
        m = min(int(res.nl_count), req.nl_capacity)
        out["nl_count"] = int(res.nl_count)
        out["nl_i"], out["nl_j"], out["nl_d"], out["nl_d2"] = nli[:m], nlj[:m], nld[:m], nld2[:m]
    return out


def lj_sample(x, H, cutoff, sample, sigma, epsilon, nthreads=0):
    """Per-particle energy E_i and gradient dE/dr_i for sampled i (brute force)."""
    x = _f64(x)
    H = _f64(H)
    n, dim = x.shape
    s = np.ascontiguousarray(sample, dtype=np.int64)
    e = np.zeros(len(s))
    g = np.zeros((len(s), dim))
    _check(lib().clmo_lj_sample(dim, _p(H), float(cutoff), _p(x), n, _p(s, _i64p), len(s),
                                float(sigma), float(epsilon), int(nthreads), _p(e), _p(g)),
           "lj_sample")
    return e, g


def neighbors_of(x, H, cutoff, i, cap=100000):
    """Neighbours j of particle i within the cutoff with raw-coordinate images K."""
    x = _f64(x)
    H = _f64(H)
    n, dim = x.shape
    js = np.zeros(cap, dtype=np.int64)
    Ks = np.zeros((cap, dim), dtype=np.intc)
    cnt = ctypes.c_int64(0)
    _check(lib().clmo_neighbors_of(dim, _p(H), float(cutoff), _p(x), n, int(i), cap,
                                   _p(js, _i64p), _p(Ks, _ip), ctypes.byref(cnt)), "neighbors_of")
    m = int(cnt.value)
    if m > cap:
        return neighbors_of(x, H, cutoff, i, cap=m)
    return js[:m], Ks[:m].astype(np.int64)


def paper_ghost_grid(H, cutoff, lcell=1):
    """The paper's printed computing-cell grid convention (Code 3), lcell 1 only."""
    H = _f64(H)
    dim = H.shape[0]
    n = np.zeros(dim, dtype=np.intc)
    s = np.zeros(dim)
    _check(lib().clmo_paper_ghost_grid(dim, _p(H), float(cutoff), int(lcell), _p(n, _ip), _p(s)),
           "paper_ghost_grid")
    return n.astype(int), s


# ---------------------------------------------------------------- molecular dynamics
def md_run(x, v, H, cutoff, sigma, epsilon, mass, dt, nsteps, *, skin=0.0, rescale_every=0,
           target_ke=None, nthreads=0):
    """Velocity-Verlet trajectory with Lennard-Jones forces (paper section 4.2:
    a Neon fluid with LJ interactions only, fixed time step, velocity
    rescaling every few steps).  Plain FP64, test infrastructure.

    Step k = 1..nsteps, with h = (dt / 2) / mass:
      v = v + h F;  x = x + dt v;  F = -dE/dx (pairs within `cutoff`);
      v = v + h F;  KE = mass / 2 * sum_i |v_i|^2;
      if rescale_every and k % rescale_every == 0: v = sqrt(target_ke / KE) v.
    Positions are never wrapped (the pair map wraps them).  With skin > 0
    the pair distances are taken in the frame of the last rebuild: a rebuild
    (frame = the canonical wrap integers of x) happens at k = 0 and whenever
    some particle has moved by more than skin / 2 since the last one
    (|x - x_ref|^2 > (skin / 2)^2).  Returns a dict with x, v, F and
    per-step arrays energy (potential), ke, count and rebuilt."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    H = _f64(H)
    n, dim = x.shape
    h = (0.5 * dt) / mass
    lim2 = (0.5 * skin) * (0.5 * skin)

    def forces(frame):
        r = compute(x, H, cutoff, lj=(sigma, epsilon), lj_grad=True, nthreads=nthreads,
                    frame=frame)
        return -r["lj_grad"], r["lj_energy"], r["count"]

    frame = wrap(x, H)[2] if skin > 0 else None
    xref = x.copy()
    F, E, c = forces(frame)
    rec = {"energy": [E], "ke": [0.5 * mass * float(np.sum(np.sum(v * v, axis=1)))],
           "count": [c], "rebuilt": [True]}
    for k in range(1, nsteps + 1):
        v = v + h * F
        x = x + dt * v
        rebuilt = False
        if skin > 0:
            d = x - xref
            if float(np.max(np.sum(d * d, axis=1))) > lim2:
                frame = wrap(x, H)[2]
                xref = x.copy()
                rebuilt = True
        F, E, c = forces(frame)
        v = v + h * F
        ke = 0.5 * mass * float(np.sum(np.sum(v * v, axis=1)))
        rec["energy"].append(E)
        rec["ke"].append(ke)
        rec["count"].append(c)
        rec["rebuilt"].append(rebuilt)
        if rescale_every and k % rescale_every == 0:
            v = np.sqrt(target_ke / ke) * v
    out = {"x": x, "v": v, "F": F}
    for key, val in rec.items():
        out[key] = np.array(val)
    return out


# ---------------------------------------------------------------- k closest pairs
def kclosest(x, H, cutoff, k, y=None, nthreads=0):
    """The k pairs with the smallest squared distance among the pairs within
    the cutoff (paper Code 8: the closest pairs between two sets, merged
    across threads by a custom reduction), in ascending (d2, i, j) order;
    fewer than k when fewer pairs are within the cutoff.  Plain definition:
    every pair within the cutoff, one sort.  Returns (i, j, d2)."""
    r = compute(x, H, cutoff, y, nl=True, nthreads=nthreads)
    i, j, d2 = r["nl_i"], r["nl_j"], r["nl_d2"]
    order = np.lexsort((j, i, d2))[:k]
    return i[order], j[order], d2[order]


# ---------------------------------------------------------------- non-periodic neighbour list
def nonperiodic_box(x, cutoff, y=None):
    """The bounding box of the paper's non-periodic neighbour list (section
    4.1: a box from the extrema of the points, large enough that no periodic
    image comes within the cutoff): orthorhombic, side (max - min) + 1.000001
    cutoff along each axis over both sets.  Every image of a displacement is
    then farther than the cutoff, so the canonical periodic pair set is the
    set of Euclidean distances <= cutoff."""
    pts = _f64(x) if y is None else np.vstack([_f64(x), _f64(y)])
    lo, hi = pts.min(axis=0), pts.max(axis=0)
    return np.diag((hi - lo) + 1.000001 * float(cutoff))


def neighbor_list_nonperiodic(x, cutoff, y=None, nthreads=0):
    """Pairs within the cutoff without periodic boundaries (paper section 4.1):
    the canonical pair set in ``nonperiodic_box``.  Returns the ``compute``
    dict (nl_i, nl_j, nl_d, nl_d2, count)."""
    H = nonperiodic_box(x, cutoff, y)
    return compute(x, H, cutoff, y, nl=True, nthreads=nthreads)
