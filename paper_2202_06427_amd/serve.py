"""Continuous-batching request loop for pair-map jobs on one GPU.

A job is one pair map over its own particle set and box (the paper's
map_pairwise call on a fresh CellList, sections 2.6-2.7): LJ energy+forces,
a neighbour list, or a distance histogram (g(r) counts).  The loop

  * admits arrived jobs in FIFO order while their HBM footprint fits the
    budget and a slot is free (the footprint is known before any device work:
    workspace + positions + outputs);
  * uploads the positions and enqueues each admitted job's cell-list build;
  * launches every admitted job of one map kind as ONE batched sweep
    (clm_map_batch): their tiles run side by side in a single kernel;
  * keeps going while those batches run: jobs arriving meanwhile are admitted
    and launched in the next batch as budget and slots free up;
  * retires a batch when its event has completed, records each job's latency
    (arrival -> results complete on the device) and frees its footprint.

Uploads and cell-list builds of newly admitted jobs go to a second stream
(default priority) while earlier batches run; a batch's sweep waits for its
jobs' builds through an event.  A neighbour list whose estimated capacity
was too small is re-run in the next batch with the exact size (the loop
never blocks on it).  With keep_results=True a finished job's device
results stay charged to the budget until release(job); with
keep_results=False only counts and energies are kept and the device
buffers return at once.

The scheduler is host code; the executor does the device work (all pair
work runs in libclmap's kernels).
"""
import collections
import ctypes
import math
import time

import numpy as np
import torch

from . import Box, CellList, _context, _ptr
from . import _lib as L

KINDS = ("lj", "nl", "gr")


class Job:
    __slots__ = ("id", "x", "H", "cutoff", "kind", "arrival", "params", "lcell", "box", "cl",
                 "xdev", "out", "footprint", "admitted", "done", "result", "status", "capacity",
                 "retries", "host", "built", "held")

    def __init__(self, jid, x, H, cutoff, kind, arrival=0.0, params=None, lcell=2):
        if kind not in KINDS:
            raise ValueError(f"kind must be one of {KINDS}")
        self.id = jid
        self.x = x
        self.H = np.asarray(H, dtype=np.float64)
        self.cutoff = float(cutoff)
        self.kind = kind
        self.arrival = float(arrival)
        self.params = dict(params or {})
        self.lcell = lcell
        self.box = self.cl = self.xdev = self.out = None
        self.footprint = 0
        self.admitted = self.done = None
        self.result = None
        self.status = "pending"
        self.capacity = 0
        self.retries = 0
        self.host = None  # (host counts, host energies, index) of its batch
        self.built = None  # event after the upload and build (side stream)
        self.held = 0      # bytes still charged to the budget after completion


def expected_pairs(n, H, cutoff):
    """Mean pair count of n uniform points (used to size neighbour lists)."""
    dim = H.shape[0]
    V = abs(np.linalg.det(H))
    p = (4.0 / 3.0) * math.pi * cutoff ** 3 / V if dim == 3 else math.pi * cutoff ** 2 / V
    return 0.5 * n * (n - 1) * min(1.0, p)


class GpuExecutor:
    """Device work of the server: cell lists, batched sweeps, events."""

    def __init__(self, device="cuda:0", precision="fp32", lj=(3.4, 0.238), gr_bins=128):
        self.device = torch.device(device)
        self.precision = precision
        self.lj = lj
        self.gr_bins = gr_bins
        # uploads and builds of admitted jobs (default priority, like the main stream)
        self.side = torch.cuda.Stream(device=self.device)

    def result_bytes(self, job):
        """Device bytes of a job's outputs (kept after completion when the
        server keeps results)."""
        n, dim = job.x.shape
        if job.kind == "lj":
            return n * dim * 8 + dim * dim * 8 + 64
        if job.kind == "nl":
            return max(job.capacity, 1) * (8 + 8) + 64
        return (self.gr_bins + 1) * 8 + 64

    def footprint(self, job):
        """Workspace + positions + outputs + the job's share of a batch
        workspace (descriptors and tile list), known before any device work."""
        n, dim = job.x.shape
        box = Box(job.H, job.cutoff, job.lcell)
        p = L.CLM_FP32_GUARD if self.precision == "fp32" else L.CLM_FP64
        nb = ctypes.c_size_t(0)
        L.check(L.lib().clm_celllist_workspace_bytes(box._h, n, 0, p, ctypes.byref(nb)))
        if job.kind == "nl" and job.capacity == 0:
            job.capacity = int(1.25 * expected_pairs(n, job.H, job.cutoff) + 4096)
        info = box.info()
        g = info["grid"] + [1] * (3 - len(info["grid"]))
        tiles = info["ncells"] + 2 * g[1] * g[2] + 5 * ((n + 63) // 64) + 8
        batch_share = 4096 + 16 * tiles
        job.box = box
        return int(nb.value) + n * dim * 8 + self.result_bytes(job) + batch_share + 4096

    def _outputs(self, job):
        n, dim = job.x.shape
        dev = self.device
        o = {}  # energy and count are slices of the batch's buffers (launch)
        if job.kind == "lj":
            o["forces"] = torch.empty((n, dim), dtype=torch.float64, device=dev)
            o["grad_box"] = torch.empty((dim, dim), dtype=torch.float64, device=dev)
        elif job.kind == "nl":
            cap = max(job.capacity, 1)
            o["pairs"] = torch.empty((cap, 2), dtype=torch.int32, device=dev)
            o["dist"] = torch.empty(cap, dtype=torch.float64, device=dev)
        else:
            o["hist"] = torch.empty(self.gr_bins + 1, dtype=torch.int64, device=dev)
        return o

    def start(self, job):
        xt = job.x if isinstance(job.x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(job.x))
        with torch.cuda.stream(self.side):
            # a payload in pinned host memory is copied without blocking the host
            job.xdev = xt.to(self.device, non_blocking=xt.is_pinned())
            job.cl = CellList(job.xdev, job.box, precision=self.precision)  # enqueues the build
            job.built = torch.cuda.Event()
            job.built.record(self.side)
        job.out = self._outputs(job)

    def regrow(self, job, capacity):
        """New neighbour-list outputs of the exact size (the cell list stays)."""
        job.capacity = int(capacity)
        job.out = self._outputs(job)
        job.host = None

    def _params(self, job):
        o = job.out
        if job.kind == "lj":
            s, e = job.params.get("lj", self.lj)
            P = L.MapParams(sigma=s, epsilon=e)
            O = L.MapOut(energy_dev=_ptr(o["energy"]), forces_dev=_ptr(o["forces"]),
                         grad_box_dev=_ptr(o["grad_box"]), count_dev=_ptr(o["count"]))
            return L.MAP_KINDS["lj_ef"], P, O
        if job.kind == "nl":
            P = L.MapParams(capacity=job.capacity, with_distances=1)
            O = L.MapOut(pairs_dev=_ptr(o["pairs"]), dist_dev=_ptr(o["dist"]), count_dev=_ptr(o["count"]))
            return L.MAP_KINDS["neighbor_list"], P, O
        P = L.MapParams(nbins=self.gr_bins, hist_hi=job.cutoff)
        O = L.MapOut(hist_dev=_ptr(o["hist"]), count_dev=_ptr(o["count"]))
        return L.MAP_KINDS["hist_dist"], P, O

    def launch(self, jobs):
        """One batched sweep over jobs of one kind; returns a completion handle.
        The batch's counts and energies land in one device buffer each and are
        copied to pinned host memory in stream order, so retiring a batch
        never waits on work launched after it."""
        _context(self.device)
        main = torch.cuda.current_stream(self.device)
        for job in jobs:  # the builds ran on the side stream
            if job.built is not None:
                main.wait_event(job.built)
                job.built = None
        n = len(jobs)
        cnt_dev = torch.empty(n, dtype=torch.int64, device=self.device)
        e_dev = torch.empty(n, dtype=torch.float64, device=self.device)
        for k, job in enumerate(jobs):
            job.out["count"] = cnt_dev[k:k + 1]
            job.out["energy"] = e_dev[k:k + 1]
        cls = (ctypes.c_void_p * n)(*[j.cl._h for j in jobs])
        Ps = (L.MapParams * n)()
        Os = (L.MapOut * n)()
        mk = None
        for k, job in enumerate(jobs):
            mk, Ps[k], Os[k] = self._params(job)
        nb = ctypes.c_size_t(0)
        L.check(L.lib().clm_map_batch_workspace_bytes(n, cls, ctypes.byref(nb)))
        raw = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        ws = raw[(-raw.data_ptr()) % 256:]
        L.check(L.lib().clm_map_batch(n, cls, mk, Ps, Os, _ptr(ws), int(nb.value)))
        cnt_host = torch.empty(n, dtype=torch.int64, pin_memory=True)
        e_host = torch.empty(n, dtype=torch.float64, pin_memory=True)
        cnt_host.copy_(cnt_dev, non_blocking=True)
        e_host.copy_(e_dev, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        for k, job in enumerate(jobs):
            job.host = (cnt_host, e_host, k)
        return (ev, raw)

    def done(self, handle, block=False):
        ev, _ = handle
        if block:
            ev.synchronize()
            return True
        return ev.query()

    def overflow(self, job):
        """Pairs of a neighbour-list job beyond its capacity (0 otherwise)."""
        if job.kind != "nl":
            return 0
        cnt_host, _, k = job.host
        cnt = int(cnt_host[k])
        return cnt if cnt > job.capacity else 0

    def finish(self, job, keep=True):
        """Results of a job whose batch has completed (host values already
        copied); keep=False drops the device outputs (count and energy stay)."""
        o = job.out
        cnt_host, e_host, k = job.host
        cnt = int(cnt_host[k])
        res = {"count": cnt}
        if job.kind == "lj":
            res["energy"] = float(e_host[k])
            if keep:
                res["forces"] = o["forces"]
                res["grad_box"] = o["grad_box"]
        elif job.kind == "nl":
            if keep:
                res["pairs"] = o["pairs"][:cnt]
                res["dist"] = o["dist"][:cnt]
        else:
            if keep:
                res["hist"] = o["hist"]
        job.result = res
        job.out = None
        job.cl = None  # the workspace returns to the allocator (stream-ordered)
        job.xdev = None

    def drain(self):
        torch.cuda.synchronize(self.device)


class Server:
    def __init__(self, executor=None, hbm_budget=8 << 30, max_slots=256, max_batch=64,
                 keep_results=True, **kw):
        self.ex = executor if executor is not None else GpuExecutor(**kw)
        self.keep_results = bool(keep_results)
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.pending = collections.deque()
        self.ready = []           # admitted and built (enqueued), not yet mapped
        self.inflight = []        # (handle, [jobs])
        self.used = 0
        self.active = 0
        self.peak_used = 0
        self.finished = []
        self.t0 = None
        self.batch_sizes = []

    def submit(self, job):
        self.pending.append(job)

    def clock(self):
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ admission
    def _admit(self, now):
        admitted = 0
        while self.pending and self.pending[0].arrival <= now and self.active < self.max_slots:
            job = self.pending[0]
            if job.footprint == 0:
                job.footprint = self.ex.footprint(job)
            if job.footprint > self.budget:
                self.pending.popleft()
                job.status = "rejected: footprint above the HBM budget"
                job.done = now
                self.finished.append(job)
                continue
            if self.used + job.footprint > self.budget:
                if not (self.ready or self.inflight) and self.active == 0:
                    # only results the caller has not released hold the budget
                    self.pending.popleft()
                    job.status = "rejected: budget held by results not released"
                    job.done = now
                    self.finished.append(job)
                    continue
                break  # FIFO: wait until running jobs release memory
            self.pending.popleft()
            job.admitted = now
            try:
                self.ex.start(job)
            except Exception as e:  # a failing job does not stop the others
                job.status = f"failed: {e}"
                job.done = now
                self.finished.append(job)
                continue
            self.used += job.footprint
            self.peak_used = max(self.peak_used, self.used)
            self.active += 1
            job.status = "admitted"
            self.ready.append(job)
            admitted += 1
        return admitted

    def _launch(self):
        groups = collections.defaultdict(list)
        for job in self.ready:
            groups[job.kind].append(job)
        self.ready = []
        for _, jobs in groups.items():
            for s in range(0, len(jobs), self.max_batch):
                chunk = jobs[s: s + self.max_batch]
                try:
                    h = self.ex.launch(chunk)
                except Exception as e:
                    for job in chunk:
                        self._release(job, f"failed: {e}")
                    continue
                self.inflight.append((h, chunk))
                self.batch_sizes.append(len(chunk))
                for job in chunk:
                    job.status = "running"

    def _retire(self, block_first=False):
        keep = []
        for k, (h, jobs) in enumerate(self.inflight):
            if self.ex.done(h, block=block_first and k == 0):
                for job in jobs:
                    try:
                        need = self.ex.overflow(job)
                        if need:
                            # the capacity estimate was too small: the exact
                            # size goes into the next batch (no blocking here)
                            grow = 16 * (need - job.capacity)
                            self.ex.regrow(job, need)
                            job.retries += 1
                            job.footprint += grow
                            self.used += grow
                            self.peak_used = max(self.peak_used, self.used)
                            job.status = "admitted"
                            self.ready.append(job)
                            continue
                        self.ex.finish(job, keep=self.keep_results)
                        status = "done"
                    except Exception as e:
                        status = f"failed: {e}"
                    self._release(job, status)
            else:
                keep.append((h, jobs))
        self.inflight = keep

    def _release(self, job, status):
        job.done = self.clock()
        job.status = status
        held = 0
        if status == "done" and self.keep_results and hasattr(self.ex, "result_bytes"):
            held = min(job.footprint, self.ex.result_bytes(job))
        job.held = held
        self.used -= job.footprint - held
        self.active -= 1
        self.finished.append(job)

    def release(self, job):
        """Return the budget held by a finished job's device results (kept
        with keep_results=True) and drop them."""
        if job.held:
            self.used -= job.held
            job.held = 0
        if job.result is not None:
            job.result = {k: v for k, v in job.result.items() if not isinstance(v, torch.Tensor)}

    # ------------------------------------------------------------ loop
    def run(self, jobs, realtime=True):
        """Serve `jobs` (arrival times in seconds from the start).  With
        realtime=False every job is available at once (closed loop)."""
        for j in sorted(jobs, key=lambda j: j.arrival):
            if not realtime:
                j.arrival = 0.0
            self.submit(j)
        self.t0 = time.perf_counter()
        while self.pending or self.ready or self.inflight:
            self._retire()
            if self._admit(self.clock()) or self.ready:
                self._launch()
                continue
            if self.pending and self.pending[0].arrival <= self.clock():
                # the head job waits for memory or a slot: block on the oldest batch
                if self.inflight:
                    self._retire(block_first=True)
                continue
            if self.inflight:
                time.sleep(0.0001)
            elif self.pending:
                time.sleep(max(0.0, min(self.pending[0].arrival - self.clock(), 0.002)))
        self.ex.drain()
        return self.summary()

    def summary(self):
        done = [j for j in self.finished if j.status == "done"]
        failed = [j for j in self.finished if j.status.startswith("failed")]
        lat = np.array([j.done - j.arrival for j in done]) if done else np.zeros(1)
        wait = np.array([j.admitted - j.arrival for j in done]) if done else np.zeros(1)
        wall = max((j.done for j in done), default=0.0)
        pairs = sum(j.result["count"] for j in done)
        return {
            "jobs": len(done),
            "failed": len(failed),
            "rejected": len(self.finished) - len(done) - len(failed),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "mean_admission_wait_ms": float(wait.mean() * 1e3),
            "p99_admission_wait_ms": float(np.percentile(wait, 99) * 1e3),
            "wall_s": wall,
            "jobs_per_s": len(done) / wall if wall > 0 else 0.0,
            "pairs_per_s": pairs / wall if wall > 0 else 0.0,
            "batches": len(self.batch_sizes),
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "peak_hbm_bytes": self.peak_used,
            "nl_retries": sum(j.retries for j in done),
        }
