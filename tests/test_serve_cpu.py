"""Scheduling logic of the serving loop, on the CPU: a fake executor runs the
oracle synchronously, so admission by footprint, slot limits, FIFO order,
batching by kind, rejection and failure isolation are tested without a GPU."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2202_06427_amd.serve import Job, Server


class FakeExecutor:
    def __init__(self, fail_ids=(), overflow_ids=(), result_bytes=0):
        self.fail_ids = set(fail_ids)
        self.overflow_ids = set(overflow_ids)  # neighbour lists whose first capacity is too small
        self.max_active_seen = 0
        self.launched = []
        self.server = None
        self.rb = result_bytes
        self.live = 0  # bytes the fake device holds (footprints + kept results)

    def footprint(self, job):
        if job.kind == "nl" and job.capacity == 0:
            job.capacity = 10 if job.id in self.overflow_ids else 10 ** 9
        return 1000 * len(job.x)

    def result_bytes(self, job):
        return self.rb

    def start(self, job):
        if job.id in self.fail_ids:
            raise RuntimeError("injected failure")
        self.live += job.footprint

    def overflow(self, job):
        if job.kind != "nl":
            return 0
        n = oracle.compute(job.x, job.H, job.cutoff)["count"]
        return n if n > job.capacity else 0

    def regrow(self, job, capacity):
        job.capacity = capacity

    def launch(self, jobs):
        kinds = {j.kind for j in jobs}
        assert len(kinds) == 1, "a batch holds one map kind"
        self.launched.append([j.id for j in jobs])
        if self.server is not None:
            self.max_active_seen = max(self.max_active_seen, self.server.active)
            assert self.server.used <= self.server.budget
        return jobs

    def done(self, handle, block=False):
        return True

    def finish(self, job, keep=True):
        r = oracle.compute(job.x, job.H, job.cutoff, nl=job.kind == "nl",
                           lj=(3.4, 0.238) if job.kind == "lj" else None,
                           hist=(16, job.cutoff) if job.kind == "gr" else None)
        job.result = {"count": r["count"]}
        self.live -= job.footprint - (min(job.footprint, self.rb) if keep else 0)

    def drain(self):
        pass


def _jobs(n_jobs, seed=0):
    g = W.rng(seed)
    jobs = []
    for k in range(n_jobs):
        n = int(g.integers(50, 400))
        H = W.random_box(g, 3, n / 0.1, bool(k % 2))
        jobs.append(Job(k, W.uniform_in_box(n, H, 100 + k), H, 6.0, ("lj", "nl", "gr")[k % 3],
                        arrival=0.001 * k))
    return jobs


def test_all_jobs_complete_with_oracle_results():
    ex = FakeExecutor()
    srv = Server(executor=ex, hbm_budget=10 ** 9, max_slots=8)
    ex.server = srv
    jobs = _jobs(20)
    summary = srv.run(jobs, realtime=False)
    assert summary["jobs"] == 20 and summary["failed"] == 0 and summary["rejected"] == 0
    for j in jobs:
        assert j.result["count"] == oracle.compute(j.x, j.H, j.cutoff)["count"]
    assert ex.max_active_seen <= 8
    assert all(len(b) >= 1 for b in ex.launched)


def test_tiny_budget_queues_and_rejects_oversized():
    ex = FakeExecutor()
    jobs = _jobs(12, seed=1)
    biggest = max(len(j.x) for j in jobs)
    srv = Server(executor=ex, hbm_budget=1000 * biggest, max_slots=64)
    ex.server = srv
    # one job larger than the whole budget is rejected, the rest queue and finish
    huge = Job(99, W.uniform_in_box(2 * biggest, np.eye(3) * 40.0, 5), np.eye(3) * 40.0, 6.0, "gr")
    summary = srv.run(jobs + [huge], realtime=False)
    assert summary["jobs"] == 12 and summary["rejected"] == 1
    assert huge.status.startswith("rejected")
    assert srv.peak_used <= srv.budget
    for b in ex.launched:  # with room for about one job at a time, batches stay small
        assert sum(len(jobs[i].x) for i in b) <= biggest


def test_failing_job_does_not_stop_the_others():
    ex = FakeExecutor(fail_ids={3, 7})
    srv = Server(executor=ex, hbm_budget=10 ** 9, max_slots=4)
    ex.server = srv
    jobs = _jobs(10, seed=2)
    summary = srv.run(jobs, realtime=False)
    assert summary["failed"] == 2 and summary["jobs"] == 8
    assert jobs[3].status.startswith("failed") and jobs[7].status.startswith("failed")
    assert srv.used == 0 and srv.active == 0


def test_fifo_admission_and_latency_accounting():
    ex = FakeExecutor()
    srv = Server(executor=ex, hbm_budget=10 ** 9, max_slots=2)
    ex.server = srv
    jobs = _jobs(8, seed=3)
    srv.run(jobs, realtime=True)
    adm = [j.admitted for j in sorted(jobs, key=lambda j: j.arrival)]
    assert adm == sorted(adm)
    for j in jobs:
        assert j.done >= j.admitted >= j.arrival - 1e-9


def test_neighbor_list_overflow_reruns_in_a_later_batch():
    """A list whose capacity estimate is too small goes back into the next
    batch with the exact size; the loop does not block, the budget grows by
    the extra outputs, and the count is the oracle's."""
    ex = FakeExecutor(overflow_ids={1, 4})
    srv = Server(executor=ex, hbm_budget=10 ** 9, max_slots=8)
    ex.server = srv
    jobs = _jobs(9, seed=4)
    summary = srv.run(jobs, realtime=False)
    assert summary["jobs"] == 9 and summary["nl_retries"] == 2
    for j in jobs:
        assert j.result["count"] == oracle.compute(j.x, j.H, j.cutoff)["count"]
    relaunched = [b for b in ex.launched if 1 in b or 4 in b]
    assert sum(b.count(1) for b in relaunched) == 2 and sum(b.count(4) for b in relaunched) == 2
    assert srv.used >= 0


def test_kept_results_hold_the_budget_until_released():
    """keep_results=True: each finished job keeps result_bytes charged; the
    budget returns on release(); keep_results=False returns it at once."""
    jobs = _jobs(6, seed=5)
    ex = FakeExecutor(result_bytes=500)
    srv = Server(executor=ex, hbm_budget=10 ** 9, max_slots=8, keep_results=True)
    ex.server = srv
    srv.run(jobs, realtime=False)
    assert srv.used == 500 * 6 and ex.live == 500 * 6
    for j in jobs:
        srv.release(j)
    assert srv.used == 0
    ex2 = FakeExecutor(result_bytes=500)
    srv2 = Server(executor=ex2, hbm_budget=10 ** 9, max_slots=8, keep_results=False)
    ex2.server = srv2
    srv2.run(_jobs(6, seed=5), realtime=False)
    assert srv2.used == 0 and ex2.live == 0


def test_accounted_budget_bounds_what_the_device_holds():
    """Many neighbour-list jobs with kept results: what the (fake) device
    holds never exceeds the budget, and jobs the held results block are
    rejected instead of waiting forever."""
    jobs = _jobs(30, seed=6)
    biggest = max(1000 * len(j.x) for j in jobs)
    ex = FakeExecutor(result_bytes=biggest // 2)
    srv = Server(executor=ex, hbm_budget=3 * biggest, max_slots=8, keep_results=True)
    ex.server = srv
    peak = [0]
    orig = ex.launch

    def launch(js):
        peak[0] = max(peak[0], ex.live)
        return orig(js)
    ex.launch = launch
    summary = srv.run(jobs, realtime=False)
    assert peak[0] <= srv.budget
    assert summary["jobs"] + summary["rejected"] == 30
