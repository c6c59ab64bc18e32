"""Serving loop (continuous batching): every job's result is the same alone
and in the mix; jobs that arrive while others run are batched, and batches on
different streams overlap in device time (timing events on the streams); the
loop reports latency percentiles and throughput; served results of every
dtype match the oracle (FP8: the FP64 oracle on the inputs dequantised by the
oracle's own quantiser)."""
import numpy as np
import pytest

import oracle
from gpu_util import U32, check_fp_full, gamma, log

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
    # batches on different streams were in progress on the device at the same
    # time (device timestamps of events recorded before the first and after
    # the last kernel of each batch on its own stream)
    ov = server.device_overlap()
    log("device overlap %s" % ov)
    assert ov["batches"] == len(server.batch_sizes)
    assert ov["overlapping_pairs"] > 0 and ov["overlap_ms"] > 0
    for job in jobs:
        alone = server.run_alone(job)
        assert torch.equal(job.out, alone), "job %d (dtype %d) differs alone and in the mix" % (job.jid, job.dtype)


def test_mixed_results_match_oracle(server):
    jobs = server.make_jobs(12, rate=None, seed=8)
    server.budget = 1 << 34
    server.run(jobs, keep_outputs=True)
    seen = set()
    for job in jobs:
        if job.dtype in seen:
            continue
        seen.add(job.dtype)
        ws = server.pool[(job.dtype, job.wid)]
        X = serve.job_input(job, server.data).cpu().numpy().astype(np.float64)
        got = job.out.cpu().numpy()
        log("served job %d dtype %d: %d x %d x %d" % (job.jid, job.dtype, job.M, job.N, job.K))
        if job.dtype == tcbf.F8_E4M3:
            # the oracle's own quantiser on the fp16 inputs (per-row scales:
            # W per beam, X per sample), exact decoding, FP64 product
            W16 = ws.source().cpu().numpy()[0].astype(np.float32)
            wr, wi, wsc = oracle.quantize_e4m3_rows(W16[0], W16[1])
            xr, xi, xsc = oracle.quantize_e4m3_rows(X[0, 0].T, X[0, 1].T)
            d = oracle.e4m3_decode
            Wd = (d(wr) + 1j * d(wi)) * np.asarray(wsc, np.float64)[:, None]
            Xd = ((d(xr) + 1j * d(xi)) * np.asarray(xsc, np.float64)[:, None]).T
            ref = oracle.cgemm(Wd[None], np.ascontiguousarray(Xd)[None])[0]
            g = got[0, 0] + 1j * got[0, 1]
            rel = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
            bound = (2.0 ** -9 + 2.0 * gamma(2 * job.K) + 4 * U32) * np.matmul(np.abs(Wd), np.abs(Xd))
            err = np.maximum(np.abs(g.real - ref.real), np.abs(g.imag - ref.imag))
            log("served FP8 job: rel Frobenius %.3e vs the dequantised-input oracle" % rel)
            assert rel <= 3e-2 and np.all(err <= bound)
        elif job.dtype == tcbf.F16:
            # the fp16 weights the resident (receiver-blocked) form was made from
            W = ws.source().cpu().numpy().astype(np.float64)
            Wc, Xc = W[:, 0] + 1j * W[:, 1], X[:, 0] + 1j * X[:, 1]
            check_fp_full(got[:, 0] + 1j * got[:, 1], oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), job.K)
        else:
            # sign bits packed by the oracle from the fp16 weights and data
            Wp = oracle.pack1bit(ws.source().cpu().numpy()[0])
            Xp = oracle.pack1bit(np.ascontiguousarray(X[0].transpose(0, 2, 1)))
            rr, ri = oracle.cgemm_1bit_popc(Wp[None, 0], Wp[None, 1], Xp[None, 0], Xp[None, 1], job.K)
            assert np.array_equal(got[:, 0].astype(np.int64), rr) and np.array_equal(got[:, 1].astype(np.int64), ri)
    assert seen == {tcbf.F16, tcbf.F8_E4M3, tcbf.INT1}


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


def test_tuned_variants_are_served():
    """With the autotuner's per-weight-set variants in use, every fp16 job
    runs in the grouped launch with the variant tuned for its weight set and
    sample count, equals its own plan with that variant bitwise, and one is
    checked against the oracle."""
    srv = serve.Server(pool_per_dtype=3, dtypes=(tcbf.F16,), budget_bytes=1 << 33, streams=2, seed=21)
    srv.tune_weights(reps=2, warmup=1)
    assert set(srv.f16_variants) == {(w, n) for w in range(3) for n in serve.Server.N_BUCKETS}
    assert all(v >= 2 for v in srv.f16_variants.values())
    log("tuned variants %s" % sorted(srv.f16_variants.items()))
    jobs = srv.make_jobs(16, rate=None, seed=22)
    summary = srv.run(jobs, keep_outputs=True)
    assert summary["completed"] == 16
    for job in jobs:
        assert srv.f16_variant(job) == srv.f16_variants[(job.wid, min(serve.Server.N_BUCKETS, key=lambda b: abs(
            np.log2(b) - np.log2(job.N))))]
        assert torch.equal(job.out, srv.run_alone(job)), "job %d" % job.jid
    job = jobs[0]
    W = srv.pool[(job.dtype, job.wid)].source().cpu().numpy().astype(np.float64)
    X = serve.job_input(job, srv.data).cpu().numpy().astype(np.float64)
    Wc, Xc = W[:, 0] + 1j * W[:, 1], X[:, 0] + 1j * X[:, 1]
    got = job.out.cpu().numpy()
    check_fp_full(got[:, 0] + 1j * got[:, 1], oracle.cgemm(Wc, Xc), np.matmul(np.abs(Wc), np.abs(Xc)), job.K)
