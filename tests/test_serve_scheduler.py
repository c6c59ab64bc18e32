"""Serving scheduler on the CPU with a scripted executor: admission under the
memory budget and slot limit, batching, and the failure paths -- a job that
can never run is rejected and the rest go on, a job that does not fit yet
waits instead of exhausting memory, a cancelled job gives its memory and slot
back, and a launch or completion error fails only its own batch."""
import itertools

import pytest

from paper_2505_03269_amd import serve


class Script:
    """Executor stand-in: a batch completes after `polls` done() calls; the
    batches whose launch number is in fail_launch raise at launch, those in
    fail_done raise when polled.  Tracks memory and slots in use."""

    def __init__(self, polls=2, fail_launch=(), fail_done=()):
        self.polls, self.fail_launch, self.fail_done = polls, set(fail_launch), set(fail_done)
        self.launches = []        # (stream, [jid, ...])
        self.live_bytes = self.peak_bytes = 0
        self.live_jobs = set()
        self.released = []

    def launch(self, batch, si):
        k = len(self.launches)
        self.launches.append((si, [j.jid for j in batch]))
        if k in self.fail_launch:
            raise RuntimeError("launch %d failed" % k)
        for j in batch:
            self.live_jobs.add(j.jid)
            self.live_bytes += j.nbytes
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        return {"k": k, "left": self.polls, "batch": batch}

    def done(self, h):
        if h["k"] in self.fail_done:
            raise RuntimeError("batch %d faulted" % h["k"])
        h["left"] -= 1
        if h["left"] > 0:
            return False
        for j in h["batch"]:
            self.live_jobs.discard(j.jid)
            self.live_bytes -= j.nbytes
        return True

    def release(self, job, keep_output):
        self.released.append(job.jid)


def jobs_of(sizes, dtype=0, cancel=None):
    out = []
    for i, nb in enumerate(sizes):
        j = serve.Job(i, 0.0, dtype, 0, 256, i, cancel_at=(cancel or {}).get(i))
        j.M, j.K, j.nbytes = 64, 64, nb
        out.append(j)
    return out


class FakeClock:
    """Deterministic time: every reading advances by one microsecond."""

    def __init__(self):
        self.t = itertools.count()

    def __call__(self):
        return next(self.t) * 1e-6


def run(sched, jobs, ex):
    return sched.run(jobs, ex, clock=FakeClock(), sleep=lambda s: None)


def test_all_jobs_done_within_budget_and_slots():
    jobs = jobs_of([100] * 20)
    sched = serve.Scheduler(budget=350, max_slots=8, streams=2, max_batch=4)
    ex = Script()
    s = run(sched, jobs, ex)
    assert s["completed"] == 20 and all(j.status == serve.DONE for j in jobs)
    assert ex.peak_bytes <= 350                          # never more than the budget in flight
    assert max(sched.batch_sizes) <= 3                   # three 100-byte jobs fit 350 bytes
    assert sorted(sum((b for _, b in ex.launches), [])) == list(range(20))
    assert sorted(ex.released) == list(range(20))


def test_slot_limit_caps_batches():
    jobs = jobs_of([1] * 10)
    sched = serve.Scheduler(budget=10**9, max_slots=2, streams=3, max_batch=8)
    ex = Script()
    run(sched, jobs, ex)
    assert max(sched.batch_sizes) <= 2 and len(ex.live_jobs) == 0


def test_impossible_jobs_rejected_others_served():
    jobs = jobs_of([100, 5000, 100, 100])          # job 1 is larger than the whole budget
    jobs[3].N = 250                                # not a multiple of 8
    sched = serve.Scheduler(budget=1000, max_slots=4, streams=1,
                            validate=lambda j: "too big" if j.nbytes > 1000 else ("bad N" if j.N % 8 else None))
    s = run(sched, jobs, Script())
    assert [j.status for j in jobs] == [serve.DONE, serve.REJECTED, serve.DONE, serve.REJECTED]
    assert jobs[1].error == "too big" and jobs[3].error == "bad N"
    assert s["completed"] == 2 and s["rejected"] == 2


def test_job_waits_for_memory_instead_of_overcommitting():
    jobs = jobs_of([600, 600, 600])
    sched = serve.Scheduler(budget=1000, max_slots=8, streams=3)
    ex = Script(polls=3)
    run(sched, jobs, ex)
    assert all(j.status == serve.DONE for j in jobs)
    assert ex.peak_bytes == 600                    # one at a time, though three streams were free
    assert [b for _, b in ex.launches] == [[0], [1], [2]]


def test_cancel_before_launch_frees_memory_and_slot():
    # job 0 holds the budget; job 1 is admitted-blocked behind it and cancelled;
    # job 2 must get job 1's place
    jobs = jobs_of([600, 400, 400], cancel={1: 0.0})
    sched = serve.Scheduler(budget=1000, max_slots=2, streams=1)
    ex = Script(polls=5)
    s = run(sched, jobs, ex)
    assert [j.status for j in jobs] == [serve.DONE, serve.CANCELLED, serve.DONE]
    assert all(1 not in b for _, b in ex.launches)
    assert s["cancelled"] == 1 and s["completed"] == 2


def test_cancel_after_launch_drops_output_when_batch_completes():
    jobs = jobs_of([10, 10], cancel={0: 1e-5})     # launched at once, cancelled while in flight
    sched = serve.Scheduler(budget=100, max_slots=4, streams=1)
    ex = Script(polls=50)
    run(sched, jobs, ex)
    assert jobs[0].status == serve.CANCELLED and jobs[1].status == serve.DONE
    assert ex.launches[0][1] == [0, 1]


def test_launch_error_fails_only_that_batch():
    jobs = jobs_of([100] * 6)
    sched = serve.Scheduler(budget=200, max_slots=8, streams=1, max_batch=2)
    ex = Script(fail_launch={1})
    s = run(sched, jobs, ex)
    failed = [j.jid for j in jobs if j.status == serve.FAILED]
    assert failed == ex.launches[1][1] and len(failed) == 2
    assert s["completed"] == 4 and s["failed"] == 2
    assert "launch 1 failed" in jobs[failed[0]].error


def test_completion_error_fails_only_that_batch():
    jobs = jobs_of([100] * 6)
    sched = serve.Scheduler(budget=200, max_slots=8, streams=2, max_batch=2)
    ex = Script(fail_done={0})
    s = run(sched, jobs, ex)
    assert [j.status for j in jobs if j.jid in ex.launches[0][1]] == [serve.FAILED] * 2
    assert s["completed"] == 4


def test_arrival_order_and_latency_summary():
    jobs = jobs_of([10] * 5)
    for i, j in enumerate(jobs):
        j.arrival = 1e-4 * (4 - i)                  # listed in reverse arrival order
    sched = serve.Scheduler(budget=10, max_slots=1, streams=1)
    ex = Script(polls=1)
    s = run(sched, jobs, ex)
    assert [b for _, b in ex.launches] == [[4], [3], [2], [1], [0]]
    assert s["p99_ms"] >= s["p50_ms"] >= 0 and all(j.t_done >= j.arrival for j in jobs)
    with pytest.raises(KeyError):
        serve.summarise(jobs_of([1]))["p50_ms"]     # nothing completed: no latency figures
