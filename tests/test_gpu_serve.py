"""Serving loop (continuous batching): every job's result is the same alone
and in the mix; jobs that arrive while others run are batched and overlap;
the loop reports latency percentiles and throughput."""
import numpy as np
import pytest

import oracle
from gpu_util import check_fp_full, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402
from paper_2505_03269_amd import serve  # noqa: E402


@pytest.fixture(scope="module")
def server():
    srv = serve.Server(pool_per_dtype=3, budget_bytes=1 << 30, streams=3, max_slots=24, seed=3)
    # a serving process warms up before it takes traffic: the overlap checks
    # below are about steady state, not a fresh process's first launches
    srv.warmup()
    return srv


def test_results_same_alone_and_in_the_mix(server):
    jobs = server.make_jobs(48, rate=3000.0, seed=7)
    # a budget of 1.5 largest jobs admits every job but makes most of them
    # wait for memory held by others
    server.budget = int(1.5 * max(j.nbytes for j in jobs))
    log("serving %d jobs" % len(jobs))
    summary = server.run(jobs, keep_outputs=True)
    log("summary %s, batches %s, max in flight %d" % (summary, server.batch_sizes, server.max_inflight))
    assert summary["jobs"] == 48 and all(j.t_done is not None and j.t_done >= j.arrival for j in jobs)
    assert summary["p99_ms"] >= summary["p50_ms"] > 0 and summary["tops"] > 0
    assert max(server.batch_sizes) > 1          # arrivals during a batch were batched together
    assert server.max_inflight > 1              # batches overlapped on the device
    for job in jobs:
        alone = server.run_alone(job)
        assert torch.equal(job.out, alone), "job %d (dtype %d) differs alone and in the mix" % (job.jid, job.dtype)


def test_mixed_results_match_oracle(server):
    jobs = server.make_jobs(12, rate=None, seed=8)
    server.budget = 1 << 34
    server.run(jobs, keep_outputs=True)
    seen = set()
    for job in jobs:
        if job.dtype in seen or job.dtype == tcbf.F8_E4M3:
            continue
        seen.add(job.dtype)
        ws = server.pool[(job.dtype, job.wid)]
        X = serve.job_input(job, server.device).cpu().numpy().astype(np.float64)
        got = job.out.cpu().numpy()
        if job.dtype == tcbf.F16:
            # resident weights are receiver-blocked [1, 2, Kb, M, 32]: back to [1, 2, M, K]
            Wb = ws.A.cpu().numpy().astype(np.float64)
            W = Wb.transpose(0, 1, 3, 2, 4).reshape(1, 2, job.M, -1)[..., :job.K]
            Wc, Xc = W[:, 0] + 1j * W[:, 1], X[:, 0] + 1j * X[:, 1]
            check_fp_full(got[:, 0] + 1j * got[:, 1], oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), job.K)
        else:
            Wp = ws.A.cpu().numpy().view(np.uint32)
            Xp = tcbf.pack1bit(serve.job_input(job, server.device), k_major=False).cpu().numpy().view(np.uint32)
            rr, ri = oracle.cgemm_1bit_popc(Wp[:, 0], Wp[:, 1], Xp[:, 0], Xp[:, 1], job.K)
            assert np.array_equal(got[:, 0].astype(np.int64), rr) and np.array_equal(got[:, 1].astype(np.int64), ri)
    assert seen == {tcbf.F16, tcbf.INT1}


def test_budget_too_small_is_reported():
    """Jobs larger than the whole budget are rejected with a reason; the run
    still returns."""
    srv = serve.Server(pool_per_dtype=1, dtypes=(tcbf.F16,), budget_bytes=1 << 10, streams=1, seed=4)
    jobs = srv.make_jobs(2, rate=None, seed=9)
    summary = srv.run(jobs)
    assert summary["rejected"] == 2 and summary["completed"] == 0
    assert all(j.status == serve.REJECTED and "budget" in j.error for j in jobs)


def test_rejected_and_cancelled_jobs_leave_the_rest_intact(server):
    """A mix with an unknown weight set, an odd sample count and a job
    cancelled before it can start: those three leave with their status, every
    other job completes with the same result as alone."""
    jobs = server.make_jobs(10, rate=None, seed=12)
    server.budget = 1 << 34
    jobs[2].wid = 999
    jobs[5].N = 300
    jobs[5].nbytes = server.job_bytes(jobs[5])
    jobs[7].cancel_at = 0.0
    summary = server.run(jobs, keep_outputs=True)
    assert jobs[2].status == serve.REJECTED and jobs[5].status == serve.REJECTED
    assert jobs[7].status == serve.CANCELLED and jobs[7].out is None
    assert summary["completed"] == 7
    for job in jobs:
        if job.status == serve.DONE:
            assert torch.equal(job.out, server.run_alone(job))
