"""Molecular dynamics on the cell-list library (paper section 4.2: a Neon fluid
with Lennard-Jones interactions only, velocity Verlet with a fixed time step,
velocity rescaling every few steps).

Binding of include/clmap_md.h plus a small driver.  Two ways to get the forces
of a step:

* ``"rebuild"`` -- the paper's protocol: the cell list is rebuilt at every step
  and the LJ forces come from the cell-pair sweep (``clm_map``, FP32 with FP64
  guards or FP64);
* ``"verlet"`` -- a Verlet pair list over a cell list built at cutoff + skin,
  rebuilt on the device only when some particle has moved by more than half
  the skin; forces from the list in FP64, with the second half-kick fused.

Everything in a step runs in the library's HIP kernels; this module only
allocates device memory (torch) and calls the C-ABI.  With ``graph=True`` the
driver records ten steps (one rescaling period) as a HIP graph and replays it.
"""
import ctypes
import math

import torch

from . import _lib as L
from . import Box, CellList, _context, _ptr

__all__ = ["Integrator", "VerletList", "run"]


def _workspace(nbytes, device):
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    pad = (-raw.data_ptr()) % 256
    return raw, raw[pad: pad + int(nbytes)]


class Integrator:
    """Velocity Verlet for n particles of one mass (clm_md_*)."""

    def __init__(self, n, dim, mass, dt, device):
        self.n, self.dim, self.mass, self.dt = int(n), int(dim), float(mass), float(dt)
        self.device = torch.device(device)
        b = ctypes.c_size_t(0)
        L.check(L.lib().clm_md_workspace_bytes(self.n, ctypes.byref(b)))
        self._raw, self._ws = _workspace(b.value, self.device)
        h = ctypes.c_void_p()
        L.check(L.lib().clm_md_create(_context(self.device), self.dim, self.n, self.mass, self.dt,
                                      _ptr(self._ws), int(b.value), ctypes.byref(h)))
        self._h = h

    def kick_drift(self, x, v, f, rescale_target_ke=0.0):
        """v = lambda v + h f; x += dt v (in place)."""
        _context(self.device)
        L.check(L.lib().clm_md_kick_drift(self._h, _ptr(x), _ptr(v), _ptr(f), float(rescale_target_ke)))

    def kick(self, v, f, ke=None):
        """v += h f; kinetic energy into ke (device float64[1]) if given."""
        _context(self.device)
        L.check(L.lib().clm_md_kick(self._h, _ptr(v), _ptr(f), _ptr(ke)))

    def kinetic(self, v, ke=None):
        """Kinetic energy of v into ke (device float64[1]) if given; kept
        for the next rescale."""
        _context(self.device)
        L.check(L.lib().clm_md_kinetic(self._h, _ptr(v), _ptr(ke)))

    def rescale(self, v, target_ke):
        """v = sqrt(target_ke / KE) v with the last kept kinetic energy."""
        _context(self.device)
        L.check(L.lib().clm_md_rescale(self._h, _ptr(v), float(target_ke)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L is not None and L._lib is not None:
            L._lib.clm_md_destroy(h)
            self._h = None


class VerletList:
    """Verlet pair list (clm_vlist_*): cell list at cutoff + skin, forces at
    cutoff, device-side rebuild when a particle has moved more than skin / 2.

    capacity: partners per particle the list can hold; by default 1.3 times
    the mean count within cutoff + skin at the mean density, plus 32."""

    def __init__(self, x, H, cutoff, skin, lcell=2, capacity=None):
        if not skin > 0:
            raise ValueError("skin must be > 0")
        self.box = Box(H, float(cutoff) + float(skin), lcell)
        self.cutoff, self.skin = float(cutoff), float(skin)
        self.cl = CellList(x, self.box, precision="fp64")
        self.n, self.dim, self.device = self.cl.nx, self.cl.dim, self.cl.device
        if capacity is None:
            vol = self.box.info()["volume"]
            rl = self.box.cutoff
            ball = 4.0 / 3.0 * math.pi * rl ** 3 if self.dim == 3 else math.pi * rl ** 2
            capacity = int(math.ceil(1.3 * self.n / vol * ball)) + 32
        self.capacity = int(capacity)
        b = ctypes.c_size_t(0)
        L.check(L.lib().clm_vlist_workspace_bytes(self.cl._h, self.capacity, ctypes.byref(b)))
        self.workspace_bytes = int(b.value)
        self._raw, self._ws = _workspace(b.value, self.device)
        h = ctypes.c_void_p()
        _context(self.device)
        L.check(L.lib().clm_vlist_create(self.cl._h, self.cutoff, self.capacity, _ptr(self._ws),
                                         self.workspace_bytes, ctypes.byref(h)))
        self._h = h

    def update(self, x):
        """Displacement check, rebuild when due, frame positions of this step."""
        _context(self.device)
        L.check(L.lib().clm_vlist_update(self._h, _ptr(x)))

    def lj(self, sigma, epsilon, forces, energy, virial=None, count=None, integrator=None, v=None,
           ke=None):
        """LJ energy and forces over the list (outputs are caller tensors);
        with an integrator the second half-kick of the step is fused."""
        _context(self.device)
        L.check(L.lib().clm_vlist_lj(self._h, float(sigma), float(epsilon), _ptr(forces), _ptr(energy),
                                     _ptr(virial), _ptr(count),
                                     None if integrator is None else integrator._h, _ptr(v), _ptr(ke)))

    def info(self):
        vi = L.VlistInfo()
        _context(self.device)
        L.check(L.lib().clm_vlist_info_get(self._h, ctypes.byref(vi)))
        return {k: getattr(vi, k) for k, _ in L.VlistInfo._fields_ if k != "pad"}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and L is not None and L._lib is not None:
            L._lib.clm_vlist_destroy(h)
            self._h = None


class _RebuildForces:
    """Forces of the paper's protocol: cell list rebuilt at every step, LJ
    forces from the cell-pair sweep."""

    def __init__(self, x, H, cutoff, lcell, precision):
        self.cl = CellList(x, Box(H, cutoff, lcell), precision=precision)

    def step(self, x, sigma, eps, F, E, C):
        self.cl.build(x)
        # the map scratch lets the library take the half-shell sweep where it
        # is faster (its automatic choice)
        sp, sb = self.cl._half_scratch("lj_ef", True)
        P = L.MapParams(sigma=sigma, epsilon=eps, near_factor=1.0, scratch_dev=sp, scratch_bytes=sb,
                        half_shell=0)
        o = L.MapOut(energy_dev=_ptr(E), forces_dev=_ptr(F), count_dev=_ptr(C))
        self.cl._map("lj_ef", P, o)


def run(x, v, H, *, cutoff, sigma, epsilon, mass, dt, nsteps, mode="verlet", skin=0.1,
        rescale_every=10, target_ke=None, lcell=2, precision="fp32", capacity=None, graph=False,
        trajectory=None):
    """Velocity-Verlet trajectory on the GPU (the step of ``oracle.md_run``).

    x, v: (n, dim) float64 device tensors, updated in place.  Returns a dict
    with per-step device tensors energy (potential), ke (after the second
    kick, before a rescale) and count (pairs within the cutoff), the final
    forces and, for mode "verlet", the list.  On a step k that is a multiple
    of rescale_every the velocities are scaled by sqrt(target_ke / KE); the
    scaling is applied at the start of the next step, and after the last step
    when it falls on one.  graph=True records one rescaling period of steps
    as a HIP graph (after a first period run eagerly) and replays it.
    trajectory: an optional (nsteps + 1, n, dim) float64 device tensor that
    receives a copy of the positions each step's forces and count were taken
    at (eager steps only: not with graph=True)."""
    n, dim = x.shape
    dev = x.device
    if trajectory is not None:
        if graph:
            raise ValueError("trajectory copies are not recorded into a graph")
        if tuple(trajectory.shape) != (nsteps + 1, n, dim) or trajectory.dtype != torch.float64 \
                or trajectory.device != dev:
            raise ValueError("trajectory must be a float64 (nsteps + 1, n, dim) tensor on x's device")
    if target_ke is None:
        rescale_every = 0
    integ = Integrator(n, dim, mass, dt, dev)
    F = torch.empty((n, dim), dtype=torch.float64, device=dev)
    E = torch.zeros(nsteps + 1, dtype=torch.float64, device=dev)
    KE = torch.zeros(nsteps + 1, dtype=torch.float64, device=dev)
    C = torch.zeros(nsteps + 1, dtype=torch.int64, device=dev)
    if mode == "verlet":
        vl = VerletList(x, H, cutoff, skin, lcell=lcell, capacity=capacity)

        def forces(e, ke, c, kick):
            vl.update(x)
            vl.lj(sigma, epsilon, F, e, count=c, integrator=integ if kick else None, v=v, ke=ke)
    elif mode == "rebuild":
        rf = _RebuildForces(x, H, cutoff, lcell, precision)
        vl = None

        def forces(e, ke, c, kick):
            rf.step(x, sigma, epsilon, F, e, c)
            if kick:
                integ.kick(v, F, ke)
    else:
        raise ValueError("mode must be 'verlet' or 'rebuild'")

    def one_step(k, e, ke, c):
        resc = rescale_every and k > 1 and (k - 1) % rescale_every == 0
        integ.kick_drift(x, v, F, target_ke if resc else 0.0)
        forces(e, ke, c, True)
        if trajectory is not None:
            trajectory[k].copy_(x)

    forces(E[0:1], KE[0:1], C[0:1], False)
    if trajectory is not None:
        trajectory[0].copy_(x)
    integ.kinetic(v, KE[0:1])
    k = 1
    if graph and rescale_every and nsteps >= 2 * rescale_every:
        while k <= rescale_every:           # first period eagerly: kernels loaded, no rescale at k = 1
            one_step(k, E[k:k + 1], KE[k:k + 1], C[k:k + 1])
            k += 1
        period = rescale_every
        nrep = (nsteps - k + 1) // period
        bE = torch.zeros(period, dtype=torch.float64, device=dev)
        bKE = torch.zeros(period, dtype=torch.float64, device=dev)
        bC = torch.zeros(period, dtype=torch.int64, device=dev)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.graph(g, stream=s):
            for j in range(period):          # the period's first step rescales
                one_step(k + j, bE[j:j + 1], bKE[j:j + 1], bC[j:j + 1])
        for _ in range(nrep):
            g.replay()
            E[k:k + period].copy_(bE)
            KE[k:k + period].copy_(bKE)
            C[k:k + period].copy_(bC)
            k += period
    while k <= nsteps:
        one_step(k, E[k:k + 1], KE[k:k + 1], C[k:k + 1])
        k += 1
    if rescale_every and nsteps > 0 and nsteps % rescale_every == 0:
        integ.rescale(v, target_ke)
    out = {"energy": E, "ke": KE, "count": C, "forces": F}
    if vl is not None:
        out["list"] = vl
    return out
