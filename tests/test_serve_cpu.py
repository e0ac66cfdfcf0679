"""Scheduling logic of the serving loop, on the CPU: a fake executor runs the
oracle synchronously, so admission by footprint, slot limits, FIFO order,
batching by kind, rejection and failure isolation are tested without a GPU."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2202_06427_amd.serve import Job, Server


class FakeExecutor:
    def __init__(self, fail_ids=()):
        self.fail_ids = set(fail_ids)
        self.max_active_seen = 0
        self.launched = []
        self.server = None

    def footprint(self, job):
        return 1000 * len(job.x)

    def start(self, job):
        if job.id in self.fail_ids:
            raise RuntimeError("injected failure")

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

    def finish(self, job):
        r = oracle.compute(job.x, job.H, job.cutoff, nl=job.kind == "nl",
                           lj=(3.4, 0.238) if job.kind == "lj" else None,
                           hist=(16, job.cutoff) if job.kind == "gr" else None)
        job.result = {"count": r["count"]}

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
