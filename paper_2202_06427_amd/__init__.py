"""Cell-list pair mapping on AMD MI355X (after CellListMap.jl, arXiv 2202.06427).

Python binding over ``libclmap.so`` (include/clmap.h).  This module only
marshals arguments: PyTorch provides device memory and the current stream;
binning, the cell-pair sweep and every reduction run in the library's HIP
kernels.  The user-facing steps mirror the paper (section 2.1): a ``Box``
(geometry and cutoff, section 2.5), a ``CellList`` (section 2.6) and a map
over the pairs within the cutoff that returns the reduced result (sections
2.3 and 2.7), with the user's closure replaced by a fixed map kind.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import ClmError

__all__ = ["Box", "CellList", "LJEnergy", "lj_energy", "ClmError", "extrema",
           "neighbor_list_nonperiodic", "calibrate"]

_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- contexts
_contexts = {}


def _context(device):
    """The library context of a device, following torch's current stream."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _contexts.get(idx)
    if h is None:
        h = ctypes.c_void_p()
        L.check(L.lib().clm_context_create(idx, None, ctypes.byref(h)))
        _contexts[idx] = h
    L.check(L.lib().clm_context_set_stream(h, ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream)))
    return h


def set_timing(enable, device=None):
    """Record HIP events around every build and sweep kernel on `device`."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    L.check(L.lib().clm_context_set_timing(_context(dev), int(bool(enable))))


def stats(reset=True, device=None):
    """Accumulated build / sweep kernel times (ms) since the last reset (synchronizes)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    st = L.Stats()
    L.check(L.lib().clm_stats_get(_context(dev), ctypes.byref(st), int(bool(reset))))
    return {k: getattr(st, k) for k, _ in L.Stats._fields_}


def _rc(cutoff):
    return 0.0 if cutoff is None else float(cutoff)


# ---------------------------------------------------------------- box
class Box:
    """Periodic box: H with the lattice vectors as columns (paper Code 3), a
    cutoff, and lcell (cell side about cutoff/lcell, paper section 2.8).
    lcell_x (default: lcell) sets the cell thickness along the first
    fractional axis separately; the pair set does not depend on it."""

    def __init__(self, H, cutoff, lcell=2, lcell_x=None):
        H = np.ascontiguousarray(np.asarray(H, dtype=np.float64))
        if H.ndim != 2 or H.shape[0] != H.shape[1]:
            raise ValueError("H must be a square matrix")
        self.dim = H.shape[0]
        self.H = H
        self.cutoff = float(cutoff)
        self.lcell_requested = int(lcell)
        h = ctypes.c_void_p()
        L.check(L.lib().clm_box_create_ex(self.dim, H.ctypes.data_as(_dp), self.cutoff, int(lcell),
                                          int(lcell_x or 0), ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_lengths_angles(cls, lengths, angles_deg, cutoff, lcell=2):
        la = np.ascontiguousarray(lengths, dtype=np.float64)
        an = np.ascontiguousarray(angles_deg, dtype=np.float64)
        h = ctypes.c_void_p()
        L.check(L.lib().clm_box_from_lengths_angles(la.ctypes.data_as(_dp), an.ctypes.data_as(_dp),
                                                    float(cutoff), int(lcell), ctypes.byref(h)))
        b = cls.__new__(cls)
        b._h = h
        info = b.info()
        b.dim = 3
        b.H = np.array(info["H"])
        b.cutoff = float(cutoff)
        b.lcell_requested = int(lcell)
        return b

    @classmethod
    def nonperiodic(cls, lo, hi, cutoff, lcell=2):
        """Bounding box of a non-periodic computation (paper section 4.1):
        side (hi - lo) + 1.000001 cutoff per axis, so that no periodic image
        comes within the cutoff."""
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        h = ctypes.c_void_p()
        L.check(L.lib().clm_box_nonperiodic(len(lo), lo.ctypes.data_as(_dp), hi.ctypes.data_as(_dp),
                                            float(cutoff), int(lcell), ctypes.byref(h)))
        b = cls.__new__(cls)
        b._h = h
        info = b.info()
        b.dim = info["dim"]
        b.H = np.array(info["H"])
        b.cutoff = float(cutoff)
        b.lcell_requested = int(lcell)
        return b

    def info(self):
        bi = L.BoxInfo()
        L.check(L.lib().clm_box_info_get(self._h, ctypes.byref(bi)))
        d = bi.dim
        return {
            "dim": d, "lcell_requested": bi.lcell_requested, "lcell": bi.lcell, "lcell_x": bi.lcell_x,
            "small_box": bool(bi.small_box), "grid": list(bi.grid[:d]), "ncells": bi.ncells,
            "H": np.array(bi.H[: d * d]).reshape(d, d), "Hinv": np.array(bi.Hinv[: d * d]).reshape(d, d),
            "widths": list(bi.widths[:d]), "volume": bi.volume, "cutoff": bi.cutoff, "rc2": bi.rc2,
            "guard_band": bi.guard_band,
        }

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L is not None and L._lib is not None:
            L._lib.clm_box_destroy(h)
            self._h = None


def _half_mode(half):
    """clm_map_params.half_shell for lj_forces / lj_adjoint's half argument."""
    return 0 if half is None else (1 if half else -1)


def _as_coords(x, dim, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on a GPU")
    if not x.is_cuda:
        raise ValueError(f"{name} must live on a GPU")
    if x.ndim != 2 or x.shape[1] != dim:
        raise ValueError(f"{name} must have shape (n, {dim})")
    return x.detach().to(torch.float64).contiguous()


# ---------------------------------------------------------------- cell list
class CellList:
    """Cell list of one set (or of two sets x and y, paper section 3.2).

    precision: "fp32" (FP32 coordinates and distances with FP64 guard bands
    and FP64 accumulation) or "fp64" (plain method).  Results of every map
    are torch tensors on the device, valid in stream order.
    """

    def __init__(self, x, box, y=None, precision="fp32"):
        self.box = box
        self.dim = box.dim
        x = _as_coords(x, self.dim, "x")
        self.device = x.device
        self.nx = x.shape[0]
        self.ny = 0 if y is None else int(y.shape[0])
        self.cross = y is not None
        if precision not in ("fp32", "fp64"):
            raise ValueError("precision must be 'fp32' or 'fp64'")
        self.precision = precision
        p = L.CLM_FP32_GUARD if precision == "fp32" else L.CLM_FP64
        nbytes = ctypes.c_size_t(0)
        L.check(L.lib().clm_celllist_workspace_bytes(box._h, self.nx, self.ny, p, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        raw = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        pad = (-raw.data_ptr()) % 256
        self._raw = raw
        self._ws = raw[pad: pad + self.workspace_bytes]
        ctx = _context(self.device)
        h = ctypes.c_void_p()
        L.check(L.lib().clm_celllist_create(ctx, box._h, self.nx, self.ny, p, _ptr(self._ws),
                                            self.workspace_bytes, ctypes.byref(h)))
        self._h = h
        self.build(x, y)

    def build(self, x, y=None):
        """(Re)bin positions of the same sizes (paper section 2.6)."""
        x = _as_coords(x, self.dim, "x")
        if x.shape[0] != self.nx:
            raise ValueError("x has a different particle count than this cell list")
        yy = None
        if self.cross:
            if y is None:
                raise ValueError("cross-set cell list needs y")
            yy = _as_coords(y, self.dim, "y")
            if yy.shape[0] != self.ny:
                raise ValueError("y has a different particle count than this cell list")
        _context(self.device)
        L.check(L.lib().clm_celllist_build(self._h, _ptr(x), _ptr(yy)))
        self._keep = (x, yy)  # inputs stay alive until the build has run
        return self

    def info(self):
        ci = L.CellListInfo()
        _context(self.device)
        L.check(L.lib().clm_celllist_info_get(self._h, ctypes.byref(ci)))
        return {k: getattr(ci, k) for k, _ in L.CellListInfo._fields_}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L is not None and L._lib is not None:
            L._lib.clm_celllist_destroy(h)
            self._h = None

    # ------------------------------------------------------------ maps
    def _map(self, kind, params, out):
        _context(self.device)
        L.check(L.lib().clm_map(self._h, L.MAP_KINDS[kind], ctypes.byref(params), ctypes.byref(out)))

    def _scalars(self):
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        c = torch.empty(1, dtype=torch.int64, device=self.device)
        return e, c

    # Every map takes an optional cutoff <= the box cutoff (None: the box's);
    # the cell grid stays the box's.
    def count(self, cutoff=None):
        """Number of pairs within the cutoff (device tensor, int64[1])."""
        _, c = self._scalars()
        o = L.MapOut(count_dev=_ptr(c))
        self._map("count", L.MapParams(cutoff=_rc(cutoff)), o)
        return c

    def sum_d(self, cutoff=None):
        """Sum of d over the pairs (paper Code 1)."""
        e, c = self._scalars()
        self._map("sum_d", L.MapParams(cutoff=_rc(cutoff)), L.MapOut(energy_dev=_ptr(e), count_dev=_ptr(c)))
        return e, c

    def sum_inv_d(self, cutoff=None):
        """Sum of 1/d over the pairs (paper Code 5)."""
        e, c = self._scalars()
        self._map("sum_inv_d", L.MapParams(cutoff=_rc(cutoff)),
                  L.MapOut(energy_dev=_ptr(e), count_dev=_ptr(c)))
        return e, c

    def sum_w_inv_d(self, w, wy=None, cutoff=None):
        """Sum of w_i w_j / d over the pairs (paper Code 5, with masses as the
        weights); w (and wy for a cross set) are per-particle device tensors."""
        w = w.detach().to(device=self.device, dtype=torch.float64).reshape(-1).contiguous()
        if w.shape[0] != self.nx:
            raise ValueError("w must have one weight per particle of x")
        wyy = None
        if self.cross:
            if wy is None:
                raise ValueError("a cross set needs wy")
            wyy = wy.detach().to(device=self.device, dtype=torch.float64).reshape(-1).contiguous()
            if wyy.shape[0] != self.ny:
                raise ValueError("wy must have one weight per particle of y")
        e, c = self._scalars()
        P = L.MapParams(cutoff=_rc(cutoff), weights_x_dev=_ptr(w), weights_y_dev=_ptr(wyy))
        self._map("sum_w_inv_d", P, L.MapOut(energy_dev=_ptr(e), count_dev=_ptr(c)))
        self._keep_w = (w, wyy)
        return e, c

    def dist_vel_histogram(self, v, nbins, hi=None, vy=None, cutoff=None):
        """Pairs per distance bin on (0, hi] and, per bin, the sum of
        |v_j - v_i| (paper Code 10: the mean pairwise speed as a function of
        distance is sums / counts).  Returns (counts with the overflow slot,
        sums, pair count)."""
        rc = self.box.cutoff if cutoff is None else float(cutoff)
        hi = rc if hi is None else float(hi)
        vx = _as_coords(v, self.dim, "v")
        vyy = _as_coords(vy, self.dim, "vy") if self.cross else None
        h = torch.empty(nbins + 1, dtype=torch.int64, device=self.device)
        sums = torch.empty(nbins, dtype=torch.float64, device=self.device)
        _, c = self._scalars()
        P = L.MapParams(nbins=nbins, hist_hi=hi, vel_x_dev=_ptr(vx), vel_y_dev=_ptr(vyy), cutoff=_rc(cutoff))
        self._map("hist_dist_vel", P, L.MapOut(hist_dev=_ptr(h), hist_sums_dev=_ptr(sums), count_dev=_ptr(c)))
        self._keep_v = (vx, vyy)
        return h, sums, c

    def lj_energy(self, sigma, epsilon, near_factor=1.0, cutoff=None):
        """Lennard-Jones energy 4 eps ((s/d)^12 - (s/d)^6) (paper Code 6)."""
        e, c = self._scalars()
        P = L.MapParams(sigma=sigma, epsilon=epsilon, near_factor=near_factor, cutoff=_rc(cutoff))
        self._map("lj_e", P, L.MapOut(energy_dev=_ptr(e), count_dev=_ptr(c)))
        return e, c

    def _half_scratch(self, kind, half):
        """(pointer, bytes) of the map scratch that selects the half-shell LJ
        force sweep (every pair once), or (None, 0) when half is False or the
        sweep does not apply to this cell list."""
        if not half:
            return None, 0
        nbytes = ctypes.c_size_t(0)
        L.check(L.lib().clm_map_scratch_bytes(self._h, L.MAP_KINDS[kind], ctypes.byref(nbytes)))
        need = int(nbytes.value)
        if need == 0:
            return None, 0
        buf = getattr(self, "_scratch", None)
        if buf is None or buf[1] < need:
            raw = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            self._scratch = (raw, need)
        raw = self._scratch[0]
        return ctypes.c_void_p(raw.data_ptr() + (-raw.data_ptr()) % 256), need

    def lj_forces(self, sigma, epsilon, near_factor=1.0, virial=False, cutoff=None, half=None,
                  prune=True):
        """Energy, forces (-dE/dr, paper Code 7), dE/dH and optionally the virial.
        half (FP32 form only): True evaluates every pair once (the half-shell
        sweep, with map scratch), False from both ends (the full-shell
        gather), None lets the library choose (the half-shell sweep when the
        cell grid gives it enough work items); prune: the half-shell sweep
        skips candidates farther than the cutoff from the tile's bounding box
        (same results)."""
        e, c = self._scalars()
        f = torch.empty((self.nx, self.dim), dtype=torch.float64, device=self.device)
        gb = torch.empty((self.dim, self.dim), dtype=torch.float64, device=self.device)
        w = torch.empty((self.dim, self.dim), dtype=torch.float64, device=self.device) if virial else None
        sp, sb = self._half_scratch("lj_ef", half is not False)
        P = L.MapParams(sigma=sigma, epsilon=epsilon, near_factor=near_factor, want_virial=int(virial),
                        cutoff=_rc(cutoff), scratch_dev=sp, scratch_bytes=sb, no_prune=int(not prune),
                        half_shell=_half_mode(half))
        o = L.MapOut(energy_dev=_ptr(e), forces_dev=_ptr(f), grad_box_dev=_ptr(gb),
                     virial_dev=_ptr(w), count_dev=_ptr(c))
        self._map("lj_ef", P, o)
        return {"energy": e, "forces": f, "grad_box": gb, "virial": w, "count": c}

    def lj_adjoint(self, sigma, epsilon, upstream, near_factor=1.0, cutoff=None, half=None):
        """g dE/dr and g dE/dH for an upstream gradient g (device float64[1])."""
        e, c = self._scalars()
        up = upstream.detach().to(device=self.device, dtype=torch.float64).reshape(1).contiguous()
        gx = torch.empty((self.nx, self.dim), dtype=torch.float64, device=self.device)
        gb = torch.empty((self.dim, self.dim), dtype=torch.float64, device=self.device)
        sp, sb = self._half_scratch("lj_adjoint", half is not False)
        P = L.MapParams(sigma=sigma, epsilon=epsilon, near_factor=near_factor, upstream_dev=_ptr(up),
                        cutoff=_rc(cutoff), scratch_dev=sp, scratch_bytes=sb, half_shell=_half_mode(half))
        o = L.MapOut(energy_dev=_ptr(e), forces_dev=_ptr(gx), grad_box_dev=_ptr(gb), count_dev=_ptr(c))
        self._map("lj_adjoint", P, o)
        self._keep_up = up
        return gx, gb, e

    def histogram(self, nbins, hi=None, cutoff=None):
        """Histogram of d on (0, hi] (right-closed bins, paper Code 10); the
        last slot counts pairs beyond hi."""
        rc = self.box.cutoff if cutoff is None else float(cutoff)
        hi = rc if hi is None else float(hi)
        h = torch.empty(nbins + 1, dtype=torch.int64, device=self.device)
        _, c = self._scalars()
        P = L.MapParams(nbins=nbins, hist_hi=hi, cutoff=_rc(cutoff))
        self._map("hist_dist", P, L.MapOut(hist_dev=_ptr(h), count_dev=_ptr(c)))
        return h, c

    def relspeed_histogram(self, v, nbins, hi, vy=None, sums=True, cutoff=None):
        """Histogram of |v_j - v_i| over the pairs and per-bin sums (paper Code 10)."""
        vx = _as_coords(v, self.dim, "v")
        vyy = _as_coords(vy, self.dim, "vy") if self.cross else None
        h = torch.empty(nbins + 1, dtype=torch.int64, device=self.device)
        s = torch.empty(nbins, dtype=torch.float64, device=self.device) if sums else None
        _, c = self._scalars()
        P = L.MapParams(nbins=nbins, hist_hi=float(hi), vel_x_dev=_ptr(vx), vel_y_dev=_ptr(vyy),
                        want_sums=int(sums), cutoff=_rc(cutoff))
        self._map("hist_relspeed", P, L.MapOut(hist_dev=_ptr(h), hist_sums_dev=_ptr(s), count_dev=_ptr(c)))
        self._keep_v = (vx, vyy)
        return h, s, c

    def kclosest(self, k, capacity=None):
        """The k pairs with the smallest distance within the cutoff (paper
        Code 8), ascending by (d2, i, j): device tensors i, j (int32) and d2
        (float64) of length min(k, pairs within the cutoff).  Synchronizes."""
        k = int(k)
        cap = int(capacity) if capacity is not None else max(8192, 4 * k)
        nbytes = ctypes.c_size_t(0)
        L.check(L.lib().clm_kclosest_workspace_bytes(self._h, k, cap, ctypes.byref(nbytes)))
        raw = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        pad = (-raw.data_ptr()) % 256
        ws = raw[pad: pad + int(nbytes.value)]
        i = torch.empty(k, dtype=torch.int32, device=self.device)
        j = torch.empty(k, dtype=torch.int32, device=self.device)
        d2 = torch.empty(k, dtype=torch.float64, device=self.device)
        found = ctypes.c_int64(0)
        _context(self.device)
        st = L.lib().clm_kclosest(self._h, k, cap, _ptr(ws), int(nbytes.value), _ptr(i), _ptr(j),
                                  _ptr(d2), ctypes.byref(found))
        if st == L.STATUS_CODES["CLM_E_CAPACITY"] and capacity is None:
            return self.kclosest(k, capacity=int(found.value))
        L.check(st)
        m = int(found.value)
        return i[:m], j[:m], d2[:m]

    def neighbor_list(self, capacity=None, distances=True, cutoff=None, sorted=False):
        """Pairs (i, j) within the cutoff (single set: i < j) and their d;
        with ``sorted`` in ascending (i, j) order (sorted on the device).

        Synchronizes (the library's capacity check); grows the buffers and
        re-runs when the list has more pairs than the capacity."""
        cap = int(capacity) if capacity is not None else max(1024, 64 * self.nx)
        while True:
            pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
            dist = torch.empty(max(cap, 1), dtype=torch.float64, device=self.device) if distances else None
            _, c = self._scalars()
            P = L.MapParams(capacity=cap, with_distances=int(distances), cutoff=_rc(cutoff),
                            sorted=int(bool(sorted)), check_capacity=1)
            ws = None
            if sorted:
                need = ctypes.c_size_t(0)
                L.check(L.lib().clm_pairs_sort_workspace_bytes(cap, int(distances), ctypes.byref(need)))
                ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=self.device)
                P.scratch_dev = ctypes.c_void_p(ws.data_ptr() + (-ws.data_ptr()) % 256)
                P.scratch_bytes = int(need.value)
            try:
                self._map("neighbor_list", P, L.MapOut(pairs_dev=_ptr(pairs), dist_dev=_ptr(dist),
                                                       count_dev=_ptr(c)))
            except L.ClmError as e:
                if e.status != L.STATUS_CODES["CLM_E_CAPACITY"]:
                    raise
                cap = int(c.item())
                continue
            n = int(c.item())
            return pairs[:n], (dist[:n] if distances else None)


# ---------------------------------------------------------------- device rates
def calibrate(kind, nbytes=1 << 30, reps=10, device="cuda:0"):
    """Measured device rate of a microbenchmark (include/clmap_calib.h):
    ``"fma_f32"`` / ``"fma_f64"`` (vector FMA chains) or ``"copy"`` (a
    device copy of ``nbytes``).  Returns (ms per launch, work per launch,
    rate) with the rate in TFLOP/s for FMA and GB/s (read + written) for the
    copy.  Synchronizes."""
    k = L.CALIB_KINDS[kind]
    dev = torch.device(device)
    need = ctypes.c_size_t(0)
    L.check(L.lib().clm_calibrate_scratch_bytes(k, ctypes.byref(need)))
    if kind == "copy":
        nbytes = int(nbytes) // 16 * 16
        if nbytes < 16:
            raise ValueError("copy calibration needs at least 16 bytes")
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        src.fill_(1)
        dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    else:
        src, nbytes = None, int(need.value)
        dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    ms, work = ctypes.c_double(0.0), ctypes.c_double(0.0)
    L.check(L.lib().clm_calibrate(_context(dev), k, _ptr(src), _ptr(dst), nbytes, int(reps),
                                  ctypes.byref(ms), ctypes.byref(work)))
    rate = work.value / (ms.value * 1e-3) / (1e9 if kind == "copy" else 1e12)
    return ms.value, work.value, rate


# ---------------------------------------------------------------- non-periodic neighbour list
def extrema(x):
    """Per-axis minima and maxima of device coordinates (n, dim), computed by
    the library's reduction kernels (synchronizes)."""
    x = _as_coords(x, x.shape[1] if x.ndim == 2 else -1, "x")
    n, dim = x.shape
    nbytes = ctypes.c_size_t(0)
    L.check(L.lib().clm_extrema_workspace_bytes(n, ctypes.byref(nbytes)))
    raw = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=x.device)
    pad = (-raw.data_ptr()) % 256
    lo, hi = np.zeros(dim), np.zeros(dim)
    L.check(L.lib().clm_extrema(_context(x.device), dim, _ptr(x), n, ctypes.c_void_p(raw.data_ptr() + pad),
                                int(nbytes.value), lo.ctypes.data_as(_dp), hi.ctypes.data_as(_dp)))
    return lo, hi


def neighbor_list_nonperiodic(x, cutoff, y=None, lcell=2, precision="fp32", distances=True,
                              capacity=None):
    """Pairs within the cutoff without periodic boundaries (paper section 4.1):
    the extrema of the points set a bounding box large enough that no periodic
    image comes within the cutoff (``Box.nonperiodic``), then the cell list
    of one set (or of x and y) and the neighbour-list map.  Returns the pairs
    (int32, (m, 2); single set i < j) and, with ``distances``, d (float64)."""
    lo, hi = extrema(x)
    if y is not None:
        lo2, hi2 = extrema(y)
        lo, hi = np.minimum(lo, lo2), np.maximum(hi, hi2)
    box = Box.nonperiodic(lo, hi, cutoff, lcell)
    cl = CellList(x, box, y=y, precision=precision)
    if capacity is None:
        # ideal-gas estimate over the bounding box of the partner set
        vol = float(np.prod(np.maximum(hi - lo, 1e-300)))
        ball = 4.0 / 3.0 * np.pi * cutoff ** 3 if box.dim == 3 else np.pi * cutoff ** 2
        partners = (cl.ny if y is not None else cl.nx) / vol * ball
        pairs = cl.nx * partners * (1.0 if y is not None else 0.5)
        capacity = int(1.25 * min(pairs, cl.nx * max(cl.ny, cl.nx))) + 1024
    return cl.neighbor_list(capacity=capacity, distances=distances)


# ---------------------------------------------------------------- autograd
class LJEnergy(torch.autograd.Function):
    """E(x, H) = sum over pairs of 4 eps ((s/d)^12 - (s/d)^6); backward runs the
    library's adjoint sweep (g dE/dx and g dE/dH at fixed Cartesian x)."""

    @staticmethod
    def forward(ctx, x, H, sigma, epsilon, cutoff, lcell=2, precision="fp32"):
        Hn = H.detach().cpu().numpy() if isinstance(H, torch.Tensor) else np.asarray(H)
        box = Box(Hn, cutoff, lcell)
        cl = CellList(x.detach(), box, precision=precision)
        e, _ = cl.lj_energy(sigma, epsilon)
        ctx.cl = cl
        ctx.params = (sigma, epsilon)
        ctx.h_is_tensor = isinstance(H, torch.Tensor)
        ctx.h_device = H.device if ctx.h_is_tensor else None
        return e.reshape(())

    @staticmethod
    def backward(ctx, gE):
        sigma, epsilon = ctx.params
        gx, gb, _ = ctx.cl.lj_adjoint(sigma, epsilon, gE.reshape(1))
        gH = gb.to(ctx.h_device) if (ctx.h_is_tensor and ctx.needs_input_grad[1]) else None
        return gx, gH, None, None, None, None, None


def lj_energy(x, H, sigma, epsilon, cutoff, lcell=2, precision="fp32"):
    return LJEnergy.apply(x, H, sigma, epsilon, cutoff, lcell, precision)
