"""Serving loop: continuous batching of beamforming jobs on one GPU.

A job asks for B = W . X with one of the resident weight sets (fp16, FP8 or
1-bit) and its own data X of N samples.  The server

  * keeps every weight set resident on the device in the form its kernel
    reads (receiver-blocked fp16 weights; receiver-blocked e4m3 codes with
    per-row scales; packed sign words), built once at start-up;
  * admits arrived jobs in arrival order while the device-memory budget and
    the slot count allow (a job's budget is its input and output buffers);
  * launches the admitted jobs as soon as a stream is free: the jobs of a
    batch go into one grouped persistent launch per dtype
    (tcbf_group_execute), on that stream, each fp16 job with the kernel
    variant the autotuner chose for its weight set and sample count once
    tune_weights() has run (else the library's default for its shape);
  * runs several streams, so a batch formed while others are still on the
    GPU overlaps with them, and frees a job's memory and slot when the host
    sees its batch complete (an event query, no blocking wait);
  * reports per-job latency (completion seen by the host minus arrival, both
    on the host clock, queueing included), p50 / p99, and throughput as useful
    operations (8 per complex multiply-accumulate) over the makespan; and
    each batch's device-time interval (timing events on its stream), from
    which device_overlap() measures how much batches overlapped on the GPU.

A job's data is a view of a device-resident data pool (the stand-in for
samples an instrument has delivered into device memory), so the served path
runs only the library's kernels: the FP8 quantisation or sign packing of the
data and the grouped products.

Failure handling: a job that can never run (unknown dtype or weight set, a
sample count the kernels do not take, more memory than the whole budget) is
rejected when it arrives and the others go on; a job that does not fit the
memory still free waits; a job cancelled before its batch is launched gives
its memory and slot back at once (after launch, when its batch completes,
and its output is dropped); a launch or completion error fails that batch's
jobs only.  Every job ends with a status: done, rejected, cancelled or
failed.

The admission and batching logic (Scheduler) is independent of the device:
it drives an executor with launch / done / release calls.  GpuExecutor runs
the batches through the library; tests drive the scheduler with a scripted
executor on the CPU.  Every product runs in the library; this module only
schedules.
"""
import time

import numpy as np

from . import (BLOCKED, F8_E4M3, F16, INT1, GROUP_MAX, GROUP_WORKSPACE_BYTES, PLANAR, Plan, block_weights,
               group_execute, pack1bit, quantize_e4m3)

DTYPE_NAMES = {F16: "f16", F8_E4M3: "f8", INT1: "int1"}


class WeightSet:
    """One resident weight matrix (M beams x K receivers) in its kernel's form:
    receiver-blocked fp16 weights or blocked e4m3 codes (repacked once, at
    registration), packed sign words for 1-bit."""

    def __init__(self, wid, dtype, M, K, seed, device):
        self.wid, self.dtype, self.M, self.K = wid, dtype, M, K
        self.seed, self.device = seed, device
        W16 = self.source()
        self.scale = None
        if dtype == F16:
            self.A = block_weights(W16)
        elif dtype == F8_E4M3:
            self.A, self.scale = quantize_e4m3(W16, k_major=True, block=0, out_layout=BLOCKED)
        else:
            self.A = pack1bit(W16, k_major=True)
        self.bytes = self.A.numel() * self.A.element_size() + (0 if self.scale is None else
                                                               self.scale.numel() * self.scale.element_size())

    def source(self):
        """The fp16 weights [1, 2, M, K] the resident form was made from
        (unit-modulus phasors, steering-like), regenerated from the seed."""
        import torch
        g = torch.Generator(device=self.device)
        g.manual_seed(self.seed)
        phi = torch.rand((self.M, self.K), device=self.device, generator=g, dtype=torch.float64) * (2 * np.pi)
        return torch.stack([torch.cos(phi), torch.sin(phi)])[None].to(torch.float16).contiguous()


DONE, REJECTED, CANCELLED, FAILED = "done", "rejected", "cancelled", "failed"


class Job:
    __slots__ = ("jid", "arrival", "dtype", "wid", "N", "seed", "t_done", "out", "X", "xs", "nbytes", "M", "K",
                 "status", "error", "cancel_at")

    def __init__(self, jid, arrival, dtype, wid, N, seed, cancel_at=None):
        self.jid, self.arrival, self.dtype, self.wid, self.N, self.seed = jid, arrival, dtype, wid, N, seed
        self.t_done = None
        self.out = self.X = self.xs = None
        self.M = self.K = 0
        self.nbytes = 0
        self.status = self.error = None
        self.cancel_at = cancel_at   # client cancels at this time (relative, like arrival), or never

    @property
    def ops(self):
        return 8.0 * self.M * self.N * self.K


def out_dtype(dtype):
    """Element type of a job's output: fp32 complex, exact int32 for 1-bit."""
    import torch
    return torch.int32 if dtype == INT1 else torch.float32


def make_data_pool(elements, seed, device):
    """Device-resident sample data (8-bit range complex Gaussian values in
    fp16, sigma 32, clipped to +-127): the stand-in for data an instrument
    has already delivered into device memory.  Jobs take their X from it, so
    no random-number or copy kernel sits inside a job's latency."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    v = torch.randn(elements, device=device, generator=g, dtype=torch.float32) * 32.0
    return v.round().clamp(-127, 127).to(torch.float16)


def job_input(job, data):
    """The job's data X [1, 2, K, N] fp16: a view of the data pool at an
    offset fixed by the job's seed (16-byte aligned)."""
    need = 2 * job.K * job.N
    if need > data.numel():
        raise ValueError("job data larger than the data pool")
    off = (int(job.seed) % ((data.numel() - need) // 8 + 1)) * 8
    return data[off:off + need].view(1, 2, job.K, job.N)


class Server:
    # largest job data: K 2048 x N 8192 complex fp16 values (two planes)
    DATA_POOL_ELEMENTS = 2 * 2048 * 8192 * 2

    def __init__(self, pool_per_dtype=16, dtypes=(F16, F8_E4M3, INT1), budget_frac=0.5, budget_bytes=None,
                 streams=3, max_slots=64, seed=0, device=0):
        import torch
        self.device = "cuda:%d" % device
        self.dev_index = device
        torch.cuda.set_device(device)
        rng = np.random.default_rng(np.random.SeedSequence([5, 0, seed]))
        self.pool = {}
        for d in dtypes:
            for i in range(pool_per_dtype):
                M = int(-(-rng.integers(128, 4097) // 8) * 8)
                K = int(-(-rng.integers(64, 2049) // 8) * 8)
                self.pool[(d, i)] = WeightSet(i, d, M, K, seed * 1000 + d * 100 + i, self.device)
        self.dtypes = tuple(dtypes)
        self.pool_per_dtype = pool_per_dtype
        self.data = make_data_pool(self.DATA_POOL_ELEMENTS, seed * 1000 + 999, self.device)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(device)
            budget_bytes = int(free * budget_frac)
        self.budget = budget_bytes
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.workspaces = [torch.empty(GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device=self.device)
                           for _ in range(streams)]
        self.max_slots = max_slots
        self.plans = {}
        self.batch_log = []
        # fp16 kernel variants chosen by the autotuner per (weight set, N
        # bucket); used while use_tuned is set (see tune_weights)
        self.f16_variants = {}
        self.use_tuned = False

    # -- jobs ---------------------------------------------------------------
    def make_jobs(self, count, rate, seed=1):
        """`count` jobs with Poisson arrivals at `rate` jobs/s (rate None: all at
        t = 0), dtype and weight set uniform, N ~ U[256, 8192] (multiple of 8)."""
        rng = np.random.default_rng(np.random.SeedSequence([5, 1, seed]))
        gaps = rng.exponential(1.0 / rate, count) if rate else np.zeros(count)
        arrivals = np.cumsum(gaps) - (gaps[0] if rate else 0.0)
        jobs = []
        for j in range(count):
            d = self.dtypes[rng.integers(len(self.dtypes))]
            w = int(rng.integers(self.pool_per_dtype))
            N = int(-(-rng.integers(256, 8193) // 8) * 8)
            job = Job(j, float(arrivals[j]), d, w, N, int(rng.integers(2**31)))
            ws = self.pool[(d, w)]
            job.M, job.K = ws.M, ws.K
            job.nbytes = self.job_bytes(job)
            jobs.append(job)
        return jobs

    def job_bytes(self, job):
        M, N, K = job.M, job.N, job.K
        b = 2 * K * N * 2 + 8 * M * N           # fp16 data in, fp32 complex out
        if job.dtype == F8_E4M3:
            b += 2 * N * (-(-K // 64) * 64) + 4 * N   # blocked codes: whole 64-receiver blocks
        elif job.dtype == INT1:
            b += 8 * N * (-(-K // 32))
        return b

    def _plan(self, dtype, M, N, K, variant=0):
        key = (dtype, M, N, K, variant)
        p = self.plans.get(key)
        if p is None:
            lay = PLANAR if dtype == INT1 else BLOCKED   # the resident weights' layout
            p = Plan(1, M, N, K, dtype, a_layout=lay, b_layout=BLOCKED if dtype == F8_E4M3 else PLANAR,
                     variant=variant, device=self.dev_index)
            self.plans[key] = p
        return p

    # -- autotuned tile choice ------------------------------------------------
    N_BUCKETS = (256, 512, 1024, 2048, 4096, 8192)

    def tune_weights(self, cache_path=None, reps=5, warmup=2):
        """Run the autotuner for every resident fp16 weight set at each
        representative sample count of N_BUCKETS (receiver-blocked weights,
        the form kept resident) and use its choices from now on: a job's
        problem joins the grouped launch with the variant tuned for its
        weight set at the bucket nearest its N (log scale).  Choices are
        cached per exact shape under cache_path (no file: this process only)."""
        from . import tune
        for (d, wid), ws in self.pool.items():
            if d != F16:
                continue
            for n in self.N_BUCKETS:
                entry = tune.tune(1, ws.M, n, ws.K, F16, cache_path=cache_path, device=self.dev_index,
                                  operand_layout=BLOCKED, reps=reps, warmup=warmup)
                self.f16_variants[(wid, n)] = tune.group_variant(entry)
        self.use_tuned = True

    def f16_variant(self, job):
        """The kernel variant of an fp16 job: 0 (the library's default for
        its shape) unless tuned choices are in use."""
        if not self.use_tuned:
            return 0
        n = min(self.N_BUCKETS, key=lambda b: abs(np.log2(b) - np.log2(max(job.N, 1))))
        return self.f16_variants.get((job.wid, n), 0)

    def validate(self, job):
        """Why `job` can never run here, or None."""
        if job.dtype not in self.dtypes or (job.dtype, job.wid) not in self.pool:
            return "unknown dtype or weight set"
        if job.N < 1 or job.N % 8 != 0:
            return "N must be a positive multiple of 8"
        if job.nbytes > self.budget:
            return "needs %d bytes, more than the memory budget of %d" % (job.nbytes, self.budget)
        return None

    def warmup(self, count=24, seed=999):
        """Serve `count` throw-away jobs back to back (every dtype's quantise /
        pack and grouped-launch path), so one-time costs of a fresh process
        (first kernel launches, allocator growth) are paid before any
        measured run."""
        self.run(self.make_jobs(count, rate=None, seed=seed))

    def run(self, jobs, keep_outputs=False, max_batch=GROUP_MAX):
        """Serve `jobs` in real time (their arrival times are relative to the
        start of the call).  Returns a summary dict; every job gets a status,
        and job.t_done when it left the server."""
        import torch
        torch.cuda.synchronize()
        self.batch_log = []
        self.t_ref = torch.cuda.Event(enable_timing=True)
        self.t_ref.record(torch.cuda.current_stream(self.device))
        sched = Scheduler(self.budget, self.max_slots, len(self.streams), max_batch, self.validate)
        summary = sched.run(jobs, GpuExecutor(self), keep_outputs)
        self.batch_sizes, self.max_inflight = sched.batch_sizes, sched.max_inflight
        summary["by_dtype"] = {DTYPE_NAMES[d]: int(sum(1 for j in jobs if j.dtype == d)) for d in self.dtypes}
        return summary

    def device_intervals(self):
        """Device-time interval of every batch of the last run, from timing
        events recorded on its stream before its first and after its last
        kernel: [(stream index, start ms, end ms)], times relative to an
        event recorded when the run started.  Call after the run."""
        import torch
        torch.cuda.synchronize()
        return [(si, self.t_ref.elapsed_time(a), self.t_ref.elapsed_time(b)) for si, a, b in self.batch_log]

    def device_overlap(self):
        """How much the batches of the last run overlapped in device time:
        pairs of batches on different streams whose intervals intersect, and
        the total time at least two streams had a batch in progress (ms)."""
        iv = self.device_intervals()
        pairs = sum(1 for i in range(len(iv)) for j in range(i + 1, len(iv))
                    if iv[i][0] != iv[j][0] and min(iv[i][2], iv[j][2]) > max(iv[i][1], iv[j][1]))
        edges = sorted([(a, 1) for _, a, _ in iv] + [(b, -1) for _, _, b in iv])
        depth, last, multi = 0, None, 0.0
        for t, d in edges:
            if depth >= 2 and last is not None:
                multi += t - last
            depth += d
            last = t
        busy = sum(b - a for _, a, b in iv)
        return {"batches": len(iv), "overlapping_pairs": pairs, "overlap_ms": multi, "batch_ms_total": busy}

    def run_alone(self, job):
        """The job's product on its own (one plain launch), for comparison."""
        import torch
        ws = self.pool[(job.dtype, job.wid)]
        X = job_input(job, self.data)
        out = torch.empty((1, 2, job.M, job.N), dtype=out_dtype(job.dtype), device=self.device)
        if job.dtype == F16:
            self._plan(F16, job.M, job.N, job.K, self.f16_variant(job)).execute(ws.A, X, out)
        elif job.dtype == F8_E4M3:
            Xq, xs = quantize_e4m3(X, k_major=False, block=0, out_layout=BLOCKED)
            self._plan(F8_E4M3, job.M, job.N, job.K).execute(ws.A, Xq, out, ws.scale, xs)
        else:
            self._plan(INT1, job.M, job.N, job.K).execute(ws.A, pack1bit(X, k_major=False), out)
        torch.cuda.synchronize()
        return out


class GpuExecutor:
    """Runs batches through the library on the server's streams: per dtype,
    the jobs of a batch in one grouped launch (their data quantised or
    sign-packed one by one first).  A batch's handle is an event recorded
    after its launches."""

    def __init__(self, server):
        self.srv = server

    def launch(self, batch, si):
        import torch
        srv = self.srv
        s = srv.streams[si]
        with torch.cuda.stream(s):
            start = torch.cuda.Event(enable_timing=True)
            start.record(s)
            f16, f8, i1, f16v = [], [], [], []
            for job in batch:
                ws = srv.pool[(job.dtype, job.wid)]
                X = job_input(job, srv.data)
                job.out = torch.empty((1, 2, job.M, job.N), dtype=out_dtype(job.dtype), device=srv.device)
                if job.dtype == F16:
                    job.X = X
                    f16.append((ws.A, X, job.out))
                    f16v.append(srv.f16_variant(job))
                elif job.dtype == F8_E4M3:
                    job.X, job.xs = quantize_e4m3(X, k_major=False, block=0, out_layout=BLOCKED)
                    f8.append((ws.A, job.X, job.out, ws.scale, job.xs, job.K))
                else:
                    job.X = pack1bit(X, k_major=False)
                    i1.append((ws.A, job.X, job.out, job.K))
            # one workspace per stream: the grouped launches of a batch run
            # one after the other on it
            for dt, probs in ((F16, f16), (F8_E4M3, f8), (INT1, i1)):
                for i in range(0, len(probs), GROUP_MAX):
                    group_execute(probs[i:i + GROUP_MAX], workspace=srv.workspaces[si], device=srv.dev_index,
                                  dtype=dt, layout=PLANAR if dt == INT1 else BLOCKED,
                                  variants=f16v[i:i + GROUP_MAX] if dt == F16 else None)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        srv.batch_log.append((si, start, ev))
        return ev

    def done(self, handle):
        return handle.query()

    def release(self, job, keep_output):
        if not keep_output:
            job.out = None
        job.X = job.xs = None


class Scheduler:
    """Admission in arrival order under a memory budget and a slot limit,
    batching of admitted jobs, one batch in flight per stream.  `validate(job)`
    returns why a job can never run (it is rejected on arrival) or None.

    The executor provides launch(batch, stream_index) -> handle,
    done(handle) -> bool and release(job, keep_output); an exception from
    launch or done fails that batch's jobs and the loop goes on."""

    def __init__(self, budget, max_slots, streams, max_batch=GROUP_MAX, validate=None):
        self.budget, self.max_slots, self.streams, self.max_batch = budget, max_slots, streams, max_batch
        self.validate = validate or (lambda job: None)
        self.batch_sizes, self.max_inflight = [], 0

    def run(self, jobs, executor, keep_outputs=False, clock=time.perf_counter, sleep=time.sleep):
        n = len(jobs)
        order = sorted(range(n), key=lambda i: jobs[i].arrival)
        pending = []          # arrived, waiting for memory or a slot
        admitted = []         # holding memory and a slot, not yet launched
        inflight = []         # (stream index, handle, jobs)
        busy = [False] * self.streams
        used = {"bytes": 0, "slots": 0}
        nxt, left = 0, n
        cancels = any(j.cancel_at is not None for j in jobs)
        self.batch_sizes, self.max_inflight = [], 0
        t0 = clock()

        def finish(job, status, error=None, free=True):
            nonlocal left
            job.status, job.error, job.t_done = status, error, clock() - t0
            if free:
                used["bytes"] -= job.nbytes
                used["slots"] -= 1
            executor.release(job, keep_outputs and status == DONE)
            left -= 1

        while left > 0:
            now = clock() - t0
            while nxt < n and jobs[order[nxt]].arrival <= now:
                job = jobs[order[nxt]]
                nxt += 1
                why = self.validate(job)
                if why is not None:
                    finish(job, REJECTED, why, free=False)
                else:
                    pending.append(job)
            # client cancellations before launch: memory and slot come back now
            for q, holds in (((pending, False), (admitted, True)) if cancels else ()):
                for job in [j for j in q if j.cancel_at is not None and j.cancel_at <= now]:
                    q.remove(job)
                    finish(job, CANCELLED, free=holds)
            # completions
            still = []
            for si, h, batch in inflight:
                try:
                    ok, err = executor.done(h), None
                except Exception as e:  # noqa: BLE001 -- the batch fails, the server goes on
                    ok, err = True, e
                if not ok:
                    still.append((si, h, batch))
                    continue
                for job in batch:
                    if err is not None:
                        finish(job, FAILED, repr(err))
                    elif job.cancel_at is not None and job.cancel_at <= clock() - t0:
                        finish(job, CANCELLED)
                    else:
                        finish(job, DONE)
                busy[si] = False
            inflight = still
            # admission in arrival order
            while pending and used["slots"] < self.max_slots and used["bytes"] + pending[0].nbytes <= self.budget:
                job = pending.pop(0)
                used["bytes"] += job.nbytes
                used["slots"] += 1
                admitted.append(job)
            # launch on a free stream
            free = [i for i in range(self.streams) if not busy[i]]
            if admitted and free:
                si = free[0]
                batch, admitted = admitted[:self.max_batch], admitted[self.max_batch:]
                try:
                    h = executor.launch(batch, si)
                except Exception as e:  # noqa: BLE001
                    for job in batch:
                        finish(job, FAILED, repr(e))
                    continue
                busy[si] = True
                inflight.append((si, h, batch))
                self.batch_sizes.append(len(batch))
                self.max_inflight = max(self.max_inflight, len(inflight))
                continue
            if not inflight and not admitted and nxt < n:
                wait = jobs[order[nxt]].arrival - (clock() - t0)
                if wait > 2e-4:
                    sleep(wait - 1e-4)
        return summarise(jobs)


def summarise(jobs):
    """Latency and throughput over the completed jobs, counts by status."""
    ok = [j for j in jobs if j.status == DONE]
    out = {"jobs": len(jobs), "completed": len(ok)}
    for st in (REJECTED, CANCELLED, FAILED):
        out[st] = sum(1 for j in jobs if j.status == st)
    if ok:
        makespan = max(j.t_done for j in ok) - min(j.arrival for j in ok)
        lat = np.array([j.t_done - j.arrival for j in ok])
        ops = sum(j.ops for j in ok)
        out.update({"makespan_s": makespan, "tops": ops / makespan / 1e12 if makespan > 0 else 0.0,
                    "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                    "mean_ms": float(lat.mean() * 1e3)})
    return out


def serve_benchmark(warmup=1000, measured=10000, load=0.8, seed=0, device=0, server=None):
    """Closed-loop capacity run, then an open-loop Poisson run at `load` x
    capacity; returns both summaries."""
    srv = server or Server(seed=seed, device=device)
    warm = srv.make_jobs(warmup, None, seed=seed + 100)
    srv.run(warm)
    closed_jobs = srv.make_jobs(measured, None, seed=seed + 200)
    closed = srv.run(closed_jobs)
    capacity = measured / closed["makespan_s"]
    open_jobs = srv.make_jobs(measured, load * capacity, seed=seed + 300)
    opened = srv.run(open_jobs)
    return {"closed_loop": closed, "capacity_jobs_per_s": capacity, "load": load, "open_loop": opened,
            "budget_bytes": srv.budget, "streams": len(srv.streams), "max_slots": srv.max_slots}
