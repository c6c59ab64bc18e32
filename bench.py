#!/usr/bin/env python3
"""Benchmark of the batched complex beamforming product on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-secondary]
                    [--no-serving] [--sweep]

One step = one tcbf_execute of the radio-astronomy workload (256 channels,
M=1024 beams, K=576 receivers, N=4096 samples, fp16 in, fp32 complex out),
inputs resident in HBM.  Throughput is counted as 8 useful ops per complex
multiply-accumulate on the unpadded sizes.  The per-launch kernel time comes
from HIP events on the stream the library launches on (torch's current
stream).  Prints ONE JSON line; secondary workloads (1-bit, steering weights,
sign packing, ultrasound shape in fp16 and FP8) ride along in its "secondary"
list.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "complex-GEMM TeraOps/s (8 ops/cMAC) & % MFMA peak; p99 latency served, FP16 vs FP8"
# MI355X published dense peaks
PEAK_F16_TFLOPS = 2516.6
PEAK_I8_TOPS = 5033.2
PEAK_F8_TFLOPS = 5033.2
PEAK_F4_TFLOPS = 10066.3
PEAK_HBM_GBS = 8000.0
# VALU xor+popcount estimate: 256 CU x 64 lanes x 2.4 GHz lane-ops/s, each
# xor+popcount pair covers 32 real +-1 MACs = 64 ops -> 32 ops per lane-op.
# The line's peak is the rate the peak probe sustains on the part (it issues
# faster than this count assumes); the estimate is the fallback without it.
PEAK_VALU_1BIT_TOPS = 256 * 64 * 2.4e9 * 32 / 1e12
# Steering weights are bound by vector arithmetic (FP64 phase, sin/cos): the
# kernel issues about 120 lane operations per complex weight (vector
# instructions x 64 lanes / weights, from a counter run of the fp16 planar
# output), against the fp32 vector lane rate of 256 CUs x 128 lanes x 2.4 GHz
STEER_LANE_OPS_PER_WEIGHT = 120
STEER_PEAK_GWS = 256 * 128 * 2.4 / STEER_LANE_OPS_PER_WEIGHT  # Gweights/s

# the throughput goal for the radio-astronomy fp16 shape, as a fraction of
# the published fp16 dense peak
TARGET_FRAC_F16 = 0.70

# accuracy gates (relative Frobenius error against the FP64 oracle)
TOL_F16 = 2e-3
TOL_F8 = 3e-2


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources each profiled kernel is compiled from (hashed together, in order)
KERNEL_SOURCES = {
    "cgemm_f16_fast_kernel": ("cgemm_f16.hip", "tcbf_tile.h", "tcbf_internal.h"),
    "cgemm_f16_pp_kernel": ("cgemm_f16.hip", "tcbf_tile.h", "tcbf_internal.h"),
}


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2505_03269_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/hbm_traffic_<kernel>.txt, "key: value" lines), or None when there
    is none or the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic_%s.txt" % kernel)
    if not os.path.exists(p):
        return None
    rec = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if kernel not in KERNEL_SOURCES or rec.get("kernel_source_sha256_16") != kernel_source_hash(kernel):
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain 1 GiB device-to-device copy, so counter runs of this script see a
    copy kernel of known size (1 GiB read, 1 GiB written) beside the workload."""
    import torch
    src = torch.ones(1 << 29, dtype=torch.float16, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def time_launches(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps  # ms per launch


def time_graph(fn, per_graph=20, replays=5):
    """Milliseconds per call of `fn` captured `per_graph` times in one HIP
    graph (on a side stream) and replayed: the device time without the host's
    per-call enqueue cost.  Median over `replays` replays."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(per_graph):
                fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    ms = []
    stream = torch.cuda.current_stream()
    for _ in range(replays):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        g.replay()
        t1.record(stream)
        torch.cuda.synchronize()
        ms.append(t0.elapsed_time(t1) / per_graph)
    del g
    return float(np.median(ms))


def time_interleaved(fns, steps, warmup, rounds=3):
    """Median ms per launch of each callable, timed in alternating rounds (so a
    clock swing during the measurement does not favour whichever goes first)."""
    res = [[] for _ in fns]
    for _ in range(rounds):
        for i, fn in enumerate(fns):
            res[i].append(time_launches(fn, steps, warmup))
    return [float(np.median(v)) for v in res]


def measure_peak(kind, random=False, target_ms=40.0, blocks=2048):
    """Measured ceiling of one instruction kind (tcbf_peak_probe): a short
    launch sizes the run to about target_ms, then the median of three timed
    launches (HIP events on the launch stream).  The clock is the median over
    workgroups of the shader-clock counter's advance over the constant 100 MHz
    counter's during that workgroup's loop (each workgroup reads both on its
    own compute unit)."""
    import torch
    import paper_2505_03269_amd as tcbf
    stream = torch.cuda.current_stream()
    sink = torch.empty(blocks * 256 * 4 + blocks * 32, dtype=torch.uint8, device="cuda:0")

    def run(iters):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        ops, _, marks = tcbf.peak_probe(kind, blocks, iters, operand_bits=None if not random else 2025, random=random,
                                        sink=sink)
        t1.record(stream)
        torch.cuda.synchronize()
        return ops, t0.elapsed_time(t1), marks.cpu().numpy()
    iters = 256
    for _ in range(2):  # the first sizing run is dominated by launch overhead
        _, ms, _ = run(iters)
        iters = max(256, int(iters * min(target_ms / max(ms, 1e-3), 64.0)))
    runs = sorted((run(iters) for _ in range(3)), key=lambda r: r[1])
    ops, ms, m = runs[1]
    ticks = (m[:, 2] - m[:, 0]).astype(np.float64)
    real = (m[:, 3] - m[:, 1]).astype(np.float64)
    ok = real > 0
    clock = round(float(np.median(100.0 * ticks[ok] / real[ok])), 1) if ok.any() else None
    return {"tops": round(ops / (ms * 1e-3) / 1e12, 1), "ms": round(ms, 3), "iterations": iters,
            "shader_clock_mhz": clock}


def peak_probes():
    import paper_2505_03269_amd as tcbf
    kinds = (("f16", tcbf.PROBE_F16), ("i8", tcbf.PROBE_I8), ("f8_e4m3", tcbf.PROBE_F8),
             ("f4_e2m1", tcbf.PROBE_F4), ("valu_xor_popc", tcbf.PROBE_VALU_XOR_POPC))
    out = {}
    for name, kind in kinds:
        out[name] = {"uniform": measure_peak(kind), "random": measure_peak(kind, random=True)}
        log("peak probe %s: %s" % (name, out[name]))
    out["hbm_copy"] = measure_copy()
    log("device copy: %s" % out["hbm_copy"])
    return out


def measure_copy(nbytes=1 << 31):
    """The memory system's practical streaming rate: a plain device-to-device
    copy of 2 GiB (torch's copy kernel), bytes read plus written per second,
    median of five."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    b.copy_(a)
    ms = []
    for _ in range(5):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        b.copy_(a)
        t1.record(stream)
        torch.cuda.synchronize()
        ms.append(t0.elapsed_time(t1))
    del a, b
    torch.cuda.empty_cache()
    m = float(np.median(ms))
    return {"gbs": round(2 * nbytes / (m * 1e-3) / 1e9, 1), "ms": round(m, 4), "bytes_each_way": nbytes}


def launch_spread(fn, launches):
    """Per-launch durations (HIP events around each launch on the current
    stream): p10 / p50 / p90 in ms."""
    import torch
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return {"launches": launches, "p10_ms": round(float(np.percentile(ms, 10)), 4),
            "p50_ms": round(float(np.percentile(ms, 50)), 4), "p90_ms": round(float(np.percentile(ms, 90)), 4)}


def host_cpu():
    """Model and thread counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def rel_fro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def planar_out(C):
    """[..., 2, rows, N] float32 planes -> complex128 [..., rows, N]."""
    C = np.asarray(C, np.float64)
    return C[..., 0, :, :] + 1j * C[..., 1, :, :]


def cpu_baseline(W, X, C_gpu, budget_s=12.0):
    """The oracle as it stands, timed on host cores on a bounded sample of the
    radio-astronomy workload (consecutive beam rows of the first channels),
    and the GPU output of those rows compared with it (stated accuracy).
    C_gpu: host copy of the first channels of the GPU output [c, 2, M, N]."""
    import oracle
    import workloads as wl
    M, K = W.shape[2], W.shape[3]
    N = X.shape[3]
    rows_done, chans = 0, []
    err2 = {}
    ref2 = {}
    t0 = time.perf_counter()
    spent = 0.0
    c = 0
    while spent < budget_s and c < C_gpu.shape[0]:
        Wc = wl.planar_to_complex(W[c])
        Xc = wl.planar_to_complex(X[c])[None]
        r = 0
        while r < M and spent < budget_s:
            t = time.perf_counter()
            ref = oracle.cgemm(Wc[None, r:r + 64], Xc)[0]
            spent += time.perf_counter() - t
            got = planar_out(C_gpu[c, :, r:r + 64])
            err2[c] = err2.get(c, 0.0) + float(np.sum(np.abs(got - ref) ** 2))
            ref2[c] = ref2.get(c, 0.0) + float(np.sum(np.abs(ref) ** 2))
            r += 64
            rows_done += 64
        chans.append((c, r))
        c += 1
    cmacs = rows_done * N * K
    per_ch = [float(np.sqrt(err2[cc] / ref2[cc])) for cc in sorted(err2)]
    worst = max(per_ch)
    return {"value": 8.0 * cmacs / spent / 1e12, "unit": "TeraOps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(spent, 2), "host": host_cpu(),
            "scope": "sampled: %.2f%% of the workload's outputs; value = sampled ops / sampled time"
                     % (100.0 * rows_done / (W.shape[0] * M)),
            "sample": "fp64 oracle on %d beam rows (%s) of the same workload, %d x %d per row"
                      % (rows_done, ", ".join("ch%d rows 0-%d" % (cc, rr - 1) for cc, rr in chans), N, K),
            "accuracy": {"metric": "relative Frobenius error of the GPU output against the FP64 oracle, "
                                   "per sampled channel (worst)",
                         "value": worst, "per_channel": [round(v, 9) for v in per_ch],
                         "tolerance": TOL_F16, "pass": worst <= TOL_F16, "entries": rows_done * N}}


# Single-thread timing of the config-1 oracle, in a child process so the
# oracle's OpenMP pool starts with one thread (the child never touches the GPU).
_C1_ONE_THREAD = r"""
import json, sys, time
sys.path.insert(0, %r)
import numpy as np
import oracle, workloads as wl
chans = [wl.c1_channel(c) for c in range(4)]
W = wl.planar_to_complex(np.stack([w for w, _ in chans]))
X = wl.planar_to_complex(np.stack([x for _, x in chans]))
ts = []
for _ in range(3):
    t = time.perf_counter(); oracle.cgemm(W, X); ts.append(time.perf_counter() - t)
print(json.dumps({"seconds": float(np.median(ts)), "threads": oracle.num_threads()}))
"""


def cpu_leg_c1(C_gpu):
    """Config 1 (4 x 128 x 64 x 512) in full: the oracle on all host threads
    (median of 3) and on one thread, and every GPU output against it."""
    import subprocess
    import oracle
    import workloads as wl
    chans = [wl.c1_channel(c) for c in range(4)]
    W = wl.planar_to_complex(np.stack([w for w, _ in chans]))
    X = wl.planar_to_complex(np.stack([x for _, x in chans]))
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        ref = oracle.cgemm(W, X)
        ts.append(time.perf_counter() - t)
    sec = float(np.median(ts))
    ops = 8.0 * 4 * 128 * 64 * 512
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        r = subprocess.run([sys.executable, "-c", _C1_ONE_THREAD % ROOT], env=env, capture_output=True, text=True,
                           timeout=300)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
    except (OSError, subprocess.SubprocessError, ValueError):
        one = None
    got = planar_out(C_gpu)
    per_ch = [rel_fro(got[c], ref[c]) for c in range(4)]
    return {"value": ops / sec / 1e12, "unit": "TeraOps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "seconds": round(sec, 5), "scope": "full output (median of 3 runs)",
            "single_thread": None if one is None else {"seconds": round(one["seconds"], 5),
                                                       "value": ops / one["seconds"] / 1e12,
                                                       "threads": one["threads"]},
            "sample": "fp64 oracle over the whole workload (4 x 128 x 512 outputs, K = 64)",
            "accuracy": {"metric": "relative Frobenius error against the FP64 oracle, per channel (worst), "
                                   "every output", "value": max(per_ch), "tolerance": TOL_F16,
                         "pass": max(per_ch) <= TOL_F16, "entries": 4 * 128 * 512}}


def cpu_leg_c3(Wp0, Xp0, C0, K, budget_s=4.0, def_rows=16):
    """1-bit workload, channel 0: the oracle's popcount form (the paper's
    algorithm on packed words) on consecutive beam rows within a time budget,
    compared with the GPU output bit for bit; and the int64 definition on a
    few rows (cost per output entry, also compared)."""
    import oracle
    M, N = Wp0.shape[1], Xp0.shape[1]
    rows, spent, mismatches = 0, 0.0, 0
    while rows < M and spent < budget_s:
        t = time.perf_counter()
        re, im = oracle.cgemm_1bit_popc(Wp0[0, rows:rows + 64][None], Wp0[1, rows:rows + 64][None],
                                        Xp0[0][None], Xp0[1][None], K)
        spent += time.perf_counter() - t
        mismatches += int(np.count_nonzero(re[0] != C0[0, rows:rows + 64]))
        mismatches += int(np.count_nonzero(im[0] != C0[1, rows:rows + 64]))
        rows += 64
    # the definition on +-1 values (unpacking is not timed)
    wr = oracle.unpack1bit(Wp0[0, :def_rows], K)
    wi = oracle.unpack1bit(Wp0[1, :def_rows], K)
    xr = np.ascontiguousarray(oracle.unpack1bit(Xp0[0], K).T)
    xi = np.ascontiguousarray(oracle.unpack1bit(Xp0[1], K).T)
    t = time.perf_counter()
    dre, dim = oracle.cgemm_1bit_def(wr[None], wi[None], xr[None], xi[None])
    t_def = time.perf_counter() - t
    mismatches += int(np.count_nonzero(dre[0] != C0[0, :def_rows])) + int(np.count_nonzero(dim[0] != C0[1, :def_rows]))
    ops = 8.0 * rows * N * K
    return {"value": ops / spent / 1e12, "unit": "TeraOps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "seconds": round(spent, 2), "host_model": host_cpu()["model"],
            "scope": "sampled: %d of %d beam rows of channel 0 (of 64 channels); value = sampled ops / sampled time"
                     % (rows, M),
            "sample": "popcount form (Sec. III-D, packed words) on rows 0-%d of channel 0, %d samples each" % (rows - 1, N),
            "definition_ns_per_entry": round(t_def / (def_rows * N) * 1e9, 1),
            "definition_sample": "int64 definition on +-1 values, rows 0-%d of channel 0 (%d entries, K = %d)"
                                 % (def_rows - 1, def_rows * N, K),
            "accuracy": {"metric": "outputs differing from the oracle (popcount form and definition)",
                         "value": mismatches, "tolerance": 0, "pass": mismatches == 0,
                         "entries": rows * N + def_rows * N}}


def cpu_leg_c4(Ws, X, ms, outs):
    """Ultrasound workload on sampled beams: the FP64 oracle on the fp16
    inputs (timed: the CPU baseline), the fp16 product's error against it, and
    each FP8 mode's error against the oracle on the dequantised inputs (the
    oracle's own quantiser, same rules) and on the unquantised inputs.
    Ws: fp16 W planes of the sampled beams [2, len(ms), K]; X: [2, K, N]."""
    import oracle
    import workloads as wl
    K, N = X.shape[1], X.shape[2]
    Wc = wl.planar_to_complex(Ws)
    Xc = wl.planar_to_complex(X)
    t = time.perf_counter()
    ref = oracle.cgemm(Wc[None], Xc[None])[0]
    sec = time.perf_counter() - t
    acc = {}
    if "f16" in outs:
        e = rel_fro(planar_out(outs["f16"]), ref)
        acc["f16"] = {"value": e, "tolerance": TOL_F16, "pass": e <= TOL_F16,
                      "against": "FP64 oracle on the same fp16 inputs"}
    d = lambda q: oracle.e4m3_decode(q)  # noqa: E731
    for name, block in (("f8_e4m3", 0), ("mxf8_e4m3", 32)):
        if name not in outs:
            continue
        if block:
            wr, wi, wsc = oracle.quantize_e4m3_blocks(Ws[0], Ws[1])
            xr, xi, xsc = oracle.quantize_e4m3_blocks(X[0].T, X[1].T)
            ws = np.repeat(oracle.e8m0_decode(wsc), 32, axis=1)[:, :K]
            xs = np.repeat(oracle.e8m0_decode(xsc), 32, axis=1)[:, :K]
        else:
            wr, wi, wsc = oracle.quantize_e4m3_rows(Ws[0], Ws[1])
            xr, xi, xsc = oracle.quantize_e4m3_rows(X[0].T, X[1].T)
            ws = np.asarray(wsc, np.float64)[:, None]
            xs = np.asarray(xsc, np.float64)[:, None]
        Wd = (d(wr) + 1j * d(wi)) * ws
        Xd = ((d(xr) + 1j * d(xi)) * xs).T
        refd = oracle.cgemm(Wd[None], np.ascontiguousarray(Xd)[None])[0]
        got = planar_out(outs[name])
        e_d, e_u = rel_fro(got, refd), rel_fro(got, ref)
        acc[name] = {"vs_dequantised_inputs": e_d, "vs_unquantised_inputs": e_u, "tolerance": TOL_F8,
                     "pass_vs_dequantised": e_d <= TOL_F8, "pass_vs_unquantised": e_u <= TOL_F8,
                     "note": "the error against the unquantised inputs is the e4m3 rounding of both operands"}
    ops = 8.0 * len(ms) * N * K
    return {"value": ops / sec / 1e12, "unit": "TeraOps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "seconds": round(sec, 3), "host_model": host_cpu()["model"],
            "scope": "sampled: %d of 32768 beams; value = sampled ops / sampled time" % len(ms),
            "sample": "fp64 oracle on beams %s... (%d seeded beams incl. the first and last), all %d frames"
                      % (", ".join(str(int(m)) for m in ms[:4]), len(ms), N),
            "accuracy": acc}


def bench_c2(steps, warmup):
    import torch
    import paper_2505_03269_amd as tcbf
    import workloads as wl
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    t0 = time.perf_counter()
    W, X = wl.generate_c2()
    log("c2 inputs generated in %.1f s" % (time.perf_counter() - t0))
    # The weights are repacked once into the receiver-blocked layout (as the
    # paper's pipeline tiles its model matrix once, before the data stream);
    # the product is then timed on resident blocked W and planar X.  The same
    # product on planar W is timed beside it.
    plan = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16, a_layout=tcbf.BLOCKED)
    plan_p = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    info = plan.info()
    A = torch.from_numpy(W).to("cuda:0")
    B = torch.from_numpy(X).to("cuda:0")
    C = plan.empty_output()
    Ab = torch.empty(tcbf.blocked_shape(cfg["batch"], cfg["M"], cfg["K"]), dtype=torch.float16, device="cuda:0")
    ms_block = time_launches(lambda: tcbf.block_weights(A, out=Ab), 3, 1)
    ms = time_launches(lambda: plan.execute(Ab, B, C), steps, warmup)
    tops = info["useful_ops"] / (ms * 1e-3) / 1e12
    spread = launch_spread(lambda: plan.execute(Ab, B, C), max(steps, 20))
    ms_p = time_launches(lambda: plan_p.execute(A, B, C), max(3, steps // 2), 2)
    planar = {"value": round(info["useful_ops"] / (ms_p * 1e-3) / 1e12, 2), "ms_per_launch": round(ms_p, 4),
              "note": "same product with planar [batch][2][M][K] weights"}
    blocking = {"ms": round(ms_block, 4), "bytes": 2 * A.numel() * 2,
                "note": "one-time weight repack into the blocked layout (not in the timed step)"}
    # the first channels of the timed product's output, for the CPU leg's
    # accuracy check
    plan.execute(Ab, B, C)
    C_head = C[:8].cpu().numpy()
    del A, Ab, B, C
    torch.cuda.empty_cache()
    return W, X, info, ms, tops, spread, planar, blocking, C_head


def bench_c2_interleaved(W, X, steps):
    """The radio-astronomy product in the interleaved complex layouts (weights
    [batch][M][K][2] repacked once into the receiver-blocked layout, data
    [batch][K][N][2] read as is, output [batch][M][N][2]), timed against the
    planar-data product in alternating rounds."""
    import torch
    import paper_2505_03269_amd as tcbf
    import workloads as wl
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    shape = (cfg["batch"], cfg["M"], cfg["N"], cfg["K"])
    Ai = torch.from_numpy(W).to("cuda:0").permute(0, 2, 3, 1).contiguous()
    Ab = tcbf.block_weights(Ai, layout=tcbf.INTERLEAVED)
    del Ai
    B = torch.from_numpy(X).to("cuda:0")
    Bi = B.permute(0, 2, 3, 1).contiguous()
    pi = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED, b_layout=tcbf.INTERLEAVED, c_layout=tcbf.INTERLEAVED)
    pp = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED)
    pm = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED, b_layout=tcbf.INTERLEAVED)
    info = pi.info()
    Ci, Cp = pi.empty_output(), pp.empty_output()
    ms_i, ms_p, ms_m = time_interleaved([lambda: pi.execute(Ab, Bi, Ci), lambda: pp.execute(Ab, B, Cp),
                                         lambda: pm.execute(Ab, Bi, Cp)], max(steps // 2, 5), 2)
    ops = info["useful_ops"]
    tops = ops / (ms_i * 1e-3) / 1e12
    del Ab, B, Bi, Ci, Cp
    torch.cuda.empty_cache()
    return {"workload": "radio-astro-fp16 interleaved: batch=256 M=1024 K=576 N=4096", "kernel": info["kernel_name"],
            "variant": info["variant"], "value": round(tops, 1), "unit": "TeraOps/s", "ms_per_launch": round(ms_i, 4),
            "dtype": "f16",
            "layout": "W interleaved, repacked once into the receiver-blocked layout; X interleaved [K][N][2]; "
                      "output interleaved [M][N][2]",
            "planar_data_tops": round(ops / (ms_p * 1e-3) / 1e12, 1),
            "interleaved_data_planar_output_tops": round(ops / (ms_m * 1e-3) / 1e12, 1),
            "ratio_to_planar": round(ms_p / ms_i, 3),
            "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tops / PEAK_F16_TFLOPS, 4)}}


def bench_c2_bf16(W, X, steps, samples):
    """The radio-astronomy product with bfloat16 operands (the same weights
    and data rounded to bfloat16 on the device; weights repacked once into the
    receiver-blocked layout), timed against the fp16 product in alternating
    rounds; sampled outputs go to the CPU leg's accuracy check."""
    import torch
    import paper_2505_03269_amd as tcbf
    import workloads as wl
    cfg = wl.WORKLOADS["radio-astro-fp16"]
    shape = (cfg["batch"], cfg["M"], cfg["N"], cfg["K"])
    A16 = torch.from_numpy(W).to("cuda:0")
    Ab16 = tcbf.block_weights(A16)
    Abf = tcbf.block_weights(A16.to(torch.bfloat16))
    del A16
    B16 = torch.from_numpy(X).to("cuda:0")
    Bbf = B16.to(torch.bfloat16)
    pb = tcbf.Plan(*shape, tcbf.BF16, a_layout=tcbf.BLOCKED)
    ph = tcbf.Plan(*shape, tcbf.F16, a_layout=tcbf.BLOCKED)
    info = pb.info()
    Cb, Ch = pb.empty_output(), ph.empty_output()
    ms_b, ms_h = time_interleaved([lambda: pb.execute(Abf, Bbf, Cb), lambda: ph.execute(Ab16, B16, Ch)],
                                  max(steps // 2, 5), 2)
    # channel 0, beams 0..63: the GPU rows and the bfloat16-rounded inputs
    rows = 64
    samples["bf16"] = {"W": torch.from_numpy(W[0, :, :rows]).to(torch.bfloat16).float().numpy(),
                       "X": Bbf[0].float().cpu().numpy(), "C": Cb[0, :, :rows].cpu().numpy()}
    ops = info["useful_ops"]
    tops = ops / (ms_b * 1e-3) / 1e12
    del Ab16, Abf, B16, Bbf, Cb, Ch
    torch.cuda.empty_cache()
    return {"workload": "radio-astro-bf16: batch=256 M=1024 K=576 N=4096", "kernel": info["kernel_name"],
            "variant": info["variant"], "value": round(tops, 1), "unit": "TeraOps/s", "ms_per_launch": round(ms_b, 4),
            "dtype": "bf16", "layout": "W receiver-blocked (repacked once), X planar; the fp16 inputs rounded to bfloat16",
            "f16_tops": round(ops / (ms_h * 1e-3) / 1e12, 1),
            "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tops / PEAK_F16_TFLOPS, 4), "peak_is": "bf16 dense matrix peak (same as fp16)"}}


def cpu_leg_bf16(sample):
    """Accuracy of the bfloat16 line: the FP64 oracle on the bfloat16-rounded
    inputs (64 beams of channel 0, every sample) against the GPU rows."""
    import oracle
    Wz = sample["W"][0].astype(np.float64) + 1j * sample["W"][1].astype(np.float64)
    Xz = sample["X"][0].astype(np.float64) + 1j * sample["X"][1].astype(np.float64)
    ref = oracle.cgemm(Wz[None], Xz[None])[0]
    e = rel_fro(planar_out(sample["C"]), ref)
    return {"value": e, "tolerance": TOL_F16, "pass": e <= TOL_F16, "entries": int(ref.size),
            "against": "FP64 oracle on the same bfloat16 inputs (channel 0, beams 0-63)"}


def bench_c1_latency(samples, launches=200):
    """The small plain-fp16 case (4 x 128 x 64 x 512): one launch is far too
    short to fill the GPU, so what counts is latency.  Per launch: eager
    launches back to back (host enqueue included), and the same launches
    captured once in a HIP graph and replayed (one graph launch per
    `launches` products)."""
    import torch
    import paper_2505_03269_amd as tcbf
    import workloads as wl
    cfg = wl.WORKLOADS["plain-fp16-4ch"]
    chans = [wl.c1_channel(c) for c in range(cfg["batch"])]
    W = np.stack([w for w, _ in chans])
    X = np.stack([x for _, x in chans])
    plan = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    A, B = torch.from_numpy(W).to("cuda:0"), torch.from_numpy(X).to("cuda:0")
    C = plan.empty_output()
    eager = time_launches(lambda: plan.execute(A, B, C), launches, 10)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.execute(A, B, C)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(launches):
                plan.execute(A, B, C)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = time_launches(g.replay, 5, 2) / launches
    ops = plan.info()["useful_ops"]
    samples["c1"] = C.cpu().numpy()
    return {"workload": "plain-fp16 latency: batch=4 M=128 K=64 N=512", "kernel": plan.info()["kernel_name"],
            "value": round(graph * 1e3, 2), "unit": "us per product (graph replay)", "higher_is_better": False,
            "eager_us_per_launch": round(eager * 1e3, 2), "graph_us_per_product": round(graph * 1e3, 2),
            "tops_graph": round(ops / (graph * 1e-3) / 1e12, 2), "launches_per_graph": launches}


def bench_secondary(steps, samples, serving=True, copy_gbs=None, valu_peak=None):
    """Config-1 latency, the 1-bit config (all variants), steering weights,
    sign packing, a memory-bound LOFAR shape, the ultrasound shape in fp16 and
    FP8, grouped launches and the served stream.  `samples` receives host
    copies of sampled GPU outputs for the CPU legs' accuracy checks."""
    import torch
    import paper_2505_03269_amd as tcbf
    from paper_2505_03269_amd import tune
    import workloads as wl
    out = []
    st = max(3, steps // 4)
    out.append(bench_c1_latency(samples))
    # 1-bit: 64 x 2048 x 8192 x 8192 from random words
    cfg = wl.WORKLOADS["one-bit"]
    Wp, Xp = wl.generate_c3()
    A = torch.from_numpy(Wp.view(np.int32)).to("cuda:0")
    B = torch.from_numpy(Xp.view(np.int32)).to("cuda:0")
    samples["c3"] = {"W0": np.ascontiguousarray(Wp[0]), "X0": np.ascontiguousarray(Xp[0]), "K": cfg["K"]}
    del Wp, Xp
    valu = (valu_peak, "the peak probe's xor+popcount rate") if valu_peak else \
        (PEAK_VALU_1BIT_TOPS, "estimate: 256 CU x 64 lanes x 2.4 GHz x 32 ops per lane-op")
    for v, peak, bound, peak_note in ((3, PEAK_F4_TFLOPS, "mfma", "fp4 (e2m1) dense matrix peak"),
                                      (1, PEAK_I8_TOPS, "mfma", "int8 dense matrix peak"),
                                      (2, valu[0], "alu", valu[1])):
        plan = tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.INT1, variant=v)
        info = plan.info()
        C = plan.empty_output()
        ms = time_launches(lambda: plan.execute(A, B, C), st, 1)
        tops = info["useful_ops"] / (ms * 1e-3) / 1e12
        out.append({"workload": "one-bit: batch=64 M=2048 K=8192 N=8192", "variant": v,
                    "default": v == tcbf.Plan(cfg["batch"], cfg["M"], cfg["N"], cfg["K"], tcbf.INT1).info()["variant"],
                    "kernel": info["kernel_name"], "value": round(tops, 1), "unit": "TeraOps/s",
                    "ms_per_launch": round(ms, 4), "dtype": "int1",
                    "roofline": {"bound": bound, "achieved": round(tops, 1), "peak": round(peak, 1),
                                 "unit": "TOP/s", "frac": round(tops / peak, 4), "peak_is": peak_note}})
        if v == 3:
            samples["c3"]["C0"] = C[0].cpu().numpy()
            samples["c3"]["line"] = len(out) - 1
        del C
    # steering weights of the radio-astronomy geometry on the GPU (FP64 phases,
    # fp16 planar out): 256 channels x 1024 beams x 576 antennas
    ax, ay, bl, bm = wl.c2_geometry()
    pos = torch.from_numpy(np.column_stack([ax, ay, np.zeros_like(ax)])).to("cuda:0")
    dirs = torch.from_numpy(np.column_stack([bl, bm, np.zeros_like(bl)])).to("cuda:0")
    freqs = torch.tensor([wl.c2_frequency(c) for c in range(256)], dtype=torch.float64, device="cuda:0")
    Wst = torch.empty((256, 2, 1024, 576), dtype=torch.float16, device="cuda:0")
    ms = time_launches(lambda: tcbf.steering_weights(pos, dirs, freqs, wl.C0, out=Wst), st, 1)
    nbytes = Wst.numel() * 2 + (pos.numel() + dirs.numel() + freqs.numel()) * 8
    gbs = nbytes / (ms * 1e-3) / 1e9
    gws = Wst.numel() / 2 / (ms * 1e-3) / 1e9
    # the same weights written straight into the blocked layout the product reads
    Wbl = torch.empty(tcbf.blocked_shape(256, 1024, 576), dtype=torch.float16, device="cuda:0")
    ms_bl = time_launches(lambda: tcbf.steering_weights(pos, dirs, freqs, wl.C0, out=Wbl, out_layout=tcbf.BLOCKED),
                          st, 1)
    del Wbl
    out.append({"workload": "steering weights fp16: 256 ch x 1024 beams x 576 antennas (FP64 phase)",
                "kernel": "steering_kernel", "value": round(gbs, 1), "unit": "GB/s", "ms_per_launch": round(ms, 4),
                "blocked_output_ms_per_launch": round(ms_bl, 4),
                "weights_per_s": round(Wst.numel() / 2 / (ms * 1e-3), 1),
                "roofline": {"bound": "alu", "achieved": round(gws, 1), "peak": round(STEER_PEAK_GWS, 1),
                             "unit": "Gweights/s", "frac": round(gws / STEER_PEAK_GWS, 4),
                             "peak_is": "fp32 vector lane rate (78.6e12 lane operations/s) / %d lane operations "
                                        "per weight (kernel's vector instructions, counter run)"
                                        % STEER_LANE_OPS_PER_WEIGHT},
                "hbm": {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4)}})
    del Wst, pos, dirs, freqs
    # sign packing of int8 interleaved data shaped like the 1-bit X: [64][8192][8192][2]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    src = torch.randint(-128, 128, (16, cfg["K"], cfg["N"], 2), dtype=torch.int8, device="cuda:0", generator=g)
    dst = torch.empty((16, 2, cfg["N"], cfg["K"] // 32), dtype=torch.int32, device="cuda:0")
    ms = time_launches(lambda: tcbf.pack1bit(src, k_major=False, layout=tcbf.INTERLEAVED, out=dst), st, 1)
    nbytes = src.numel() + dst.numel() * 4
    gbs = nbytes / (ms * 1e-3) / 1e9
    del src, dst, A, B
    torch.cuda.empty_cache()
    # a memory-bound product the library itself runs (the LOFAR beamformer
    # shape of Sec. V-B with 64 stations: 256 x 1024 x 1024 x 64, blocked
    # weights): its algorithmic byte rate is a streaming rate this part
    # demonstrably reaches, the ceiling the packing kernel is scored against
    lofar = bench_lofar_k64(st)
    out.append(lofar)
    stream_peak = max(copy_gbs or 0.0, lofar["value"])
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "measured_peak": round(stream_peak, 1),
            "measured_peak_is": "best of a 2 GiB device copy (%s GB/s) and the LOFAR K=64 product's algorithmic "
                                "byte rate (%s GB/s)" % (copy_gbs, lofar["value"]),
            "frac_of_measured_peak": round(gbs / stream_peak, 4)}
    out.append({"workload": "pack1bit int8 interleaved [16][8192][8192][2] -> words",
                "kernel": "pack_nmajor_vec_kernel", "value": round(gbs, 1), "unit": "GB/s",
                "ms_per_launch": round(ms, 4), "roofline": roof})
    # ultrasound shape, fp16: 1 x 32768 x 8192 x 256
    cfg = wl.WORKLOADS["ultrasound-fp16"]
    W, X = wl.c4_channel(0)
    # the model matrix is tiled once before the experiment (Sec. V-A): blocked
    # weights, with the planar-weight product beside it
    plan = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], tcbf.F16, a_layout=tcbf.BLOCKED)
    plan_p = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], tcbf.F16)
    info = plan.info()
    A = torch.from_numpy(W[None]).to("cuda:0")
    B = torch.from_numpy(X[None]).to("cuda:0")
    Ab = tcbf.block_weights(A)
    C = plan.empty_output()
    # sub-millisecond launches: time enough of them to average out clock swings
    st4 = max(st, 20)
    # the autotuner's choice for this shape (blocked weights), timed beside
    # the library's default plan
    ent = tune.tune(1, cfg["M"], cfg["N"], cfg["K"], tcbf.F16, operand_layout=tcbf.BLOCKED, reps=10, warmup=3)
    v_def = info["variant"]
    plan_t = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], tcbf.F16, a_layout=tcbf.BLOCKED, variant=ent["variant"])
    if ent["variant"] == v_def:
        ms, ms_p = time_interleaved([lambda: plan.execute(Ab, B, C), lambda: plan_p.execute(A, B, C)], st4, 3)
        ms_t = ms
    else:
        ms, ms_p, ms_t = time_interleaved([lambda: plan.execute(Ab, B, C), lambda: plan_p.execute(A, B, C),
                                           lambda: plan_t.execute(Ab, B, C)], st4, 3)
    # sampled beams for the CPU leg (seeded, plus the first and the last)
    beams = np.unique(np.concatenate([[0, cfg["M"] - 1], np.random.default_rng(11).choice(cfg["M"], 62, replace=False)]))
    beams_d = torch.from_numpy(beams).to("cuda:0")
    samples["c4"] = {"ms": beams, "Ws": np.ascontiguousarray(W[:, beams]), "X": X, "outs": {}, "lines": {}}
    plan.execute(Ab, B, C)
    samples["c4"]["outs"]["f16"] = C[0][:, beams_d].cpu().numpy()
    del Ab
    tops = info["useful_ops"] / (ms * 1e-3) / 1e12
    out.append({"workload": "ultrasound-fp16: batch=1 M=32768 K=8192 N=256", "kernel": info["kernel_name"],
                "value": round(tops, 1), "unit": "TeraOps/s", "ms_per_launch": round(ms, 4), "dtype": "f16",
                "layout": "W receiver-blocked (repacked once), X planar", "variant": v_def,
                "weights_planar_tops": round(info["useful_ops"] / (ms_p * 1e-3) / 1e12, 1),
                "tuned": {"variant": ent["variant"], "tops": round(info["useful_ops"] / (ms_t * 1e-3) / 1e12, 1),
                          "ms_per_launch": round(ms_t, 4), "kernel": plan_t.info()["kernel_name"],
                          "tuner_ms": ent["ms"]},
                "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F16_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tops / PEAK_F16_TFLOPS, 4)}})
    samples["c4"]["lines"]["f16"] = len(out) - 1
    del C
    # the same shape in FP8: W quantised once (resident weights), X quantised
    # every step; per-row fp32 scales and per-32-block E8M0 scales; codes in
    # the receiver-blocked layout the quantiser writes directly (the planar
    # codes' product is timed beside it)
    for dt, block, name, key in ((tcbf.F8_E4M3, 0, "fp8-e4m3 per-row scales", "f8_e4m3"),
                                 (tcbf.MXF8_E4M3, 32, "mxfp8-e4m3 per-32-block scales", "mxf8_e4m3")):
        BL = tcbf.BLOCKED
        Wq, Ws = tcbf.quantize_e4m3(A, k_major=True, layout=tcbf.PLANAR, block=block, out_layout=BL)
        Xq, Xs = tcbf.quantize_e4m3(B, k_major=False, layout=tcbf.PLANAR, block=block, out_layout=BL)
        plan = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], dt, a_layout=BL, b_layout=BL)
        info = plan.info()
        C = plan.empty_output()
        ms_q = time_launches(lambda: tcbf.quantize_e4m3(B, k_major=False, layout=tcbf.PLANAR, block=block,
                                                        out=Xq, scales=Xs, out_layout=BL), st4, 1)
        Wp, Wps = tcbf.quantize_e4m3(A, k_major=True, layout=tcbf.PLANAR, block=block)
        Xp, Xps = tcbf.quantize_e4m3(B, k_major=False, layout=tcbf.PLANAR, block=block)
        plan_p = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], dt)
        # the autotuner's choice (128 x 128 tiles with two or three stages, or
        # the 256 x 128 ping-pong kernel), timed beside the default plan
        ent = tune.tune(1, cfg["M"], cfg["N"], cfg["K"], dt, operand_layout=BL, reps=10, warmup=3)
        plan_t = tcbf.Plan(1, cfg["M"], cfg["N"], cfg["K"], dt, a_layout=BL, b_layout=BL, variant=ent["variant"])
        runs = [lambda: plan.execute(Wq, Xq, C, Ws, Xs), lambda: plan_p.execute(Wp, Xp, C, Wps, Xps)]
        if ent["variant"] != info["variant"]:
            runs.append(lambda: plan_t.execute(Wq, Xq, C, Ws, Xs))
        ts = time_interleaved(runs, st4, 3)
        ms, ms_p = ts[0], ts[1]
        ms_t = ts[2] if len(ts) > 2 else ms
        del Wp, Wps, Xp, Xps
        tops = info["useful_ops"] / (ms * 1e-3) / 1e12
        out.append({"workload": "ultrasound-%s: batch=1 M=32768 K=8192 N=256" % name, "kernel": info["kernel_name"],
                    "value": round(tops, 1), "unit": "TeraOps/s", "ms_per_launch": round(ms, 4), "dtype": "e4m3",
                    "layout": "W and X codes receiver-blocked (as quantised)",
                    "planar_codes_tops": round(info["useful_ops"] / (ms_p * 1e-3) / 1e12, 1),
                    "x_quantise_ms": round(ms_q, 4),
                    "step_with_x_quantise_tops": round(info["useful_ops"] / ((ms + ms_q) * 1e-3) / 1e12, 1),
                    "variant": info["variant"],
                    "tuned": {"variant": ent["variant"], "tops": round(info["useful_ops"] / (ms_t * 1e-3) / 1e12, 1),
                              "ms_per_launch": round(ms_t, 4), "kernel": plan_t.info()["kernel_name"],
                              "tuner_ms": ent["ms"]},
                    "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F8_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(tops / PEAK_F8_TFLOPS, 4)}})
        plan.execute(Wq, Xq, C, Ws, Xs)
        samples["c4"]["outs"][key] = C[0][:, beams_d].cpu().numpy()
        samples["c4"]["lines"][key] = len(out) - 1
        del Wq, Ws, Xq, Xs, C
    del A, B
    torch.cuda.empty_cache()
    # grouped persistent launch: uneven job shapes in one launch, against one
    # launch per job; served-stream sizes (each job fills the GPU alone) and
    # small jobs (each leaves most CUs idle alone)
    ws = torch.empty(tcbf.GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:0")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(7)
    for label, count, ranges in (("16 jobs, M~U[128,4096] N~U[256,8192] K~U[64,2048]", 16, {}),
                                 ("32 small jobs, M~U[128,512] N~U[256,1024] K~U[64,512]", 32,
                                  dict(m_range=(128, 512), n_range=(256, 1024), k_range=(64, 512)))):
        shapes = wl.mixed_shapes(0, count, **ranges)
        probs = []
        for (M, N, K) in shapes:
            Wg = torch.randn((1, 2, M, K), device="cuda:0", generator=g).half()
            Xg = torch.randint(-127, 128, (1, 2, K, N), device="cuda:0", generator=g).half()
            probs.append((Wg, Xg, torch.empty((1, 2, M, N), device="cuda:0")))
        plans = [tcbf.Plan(1, M, N, K, tcbf.F16) for (M, N, K) in shapes]
        ops = sum(8.0 * M * N * K for (M, N, K) in shapes)
        ms_g = time_launches(lambda: tcbf.group_execute(probs, workspace=ws), st, 1)

        def each():
            for pl, (Wg, Xg, Cg) in zip(plans, probs):
                pl.execute(Wg, Xg, Cg)
        ms_s = time_launches(each, st, 1)
        # the same launch with receiver-blocked weights (repacked once)
        probs_b = [(tcbf.block_weights(Wg), Xg, Cg) for (Wg, Xg, Cg) in probs]
        ms_gb = time_launches(lambda: tcbf.group_execute(probs_b, workspace=ws, layout=tcbf.BLOCKED), st, 1)
        # per-problem variants chosen by the autotuner timing the grouped
        # launch itself (candidate lists: defaults, each problem's own tuned
        # plan, ping-pong tiles, 128 x 128 tiles), against the library's
        # default variants, both weight layouts
        full = [(1, M, N, K) for (M, N, K) in shapes]
        ent = tune.tune_group(full, lambda v: time_launches(
            lambda: tcbf.group_execute(probs, workspace=ws, variants=v), st, 1), reps=5, warmup=2)
        entb = tune.tune_group(full, lambda v: time_launches(
            lambda: tcbf.group_execute(probs_b, workspace=ws, layout=tcbf.BLOCKED, variants=v), st, 1),
            operand_layout=tcbf.BLOCKED, reps=5, warmup=2)
        tv, tvb = ent["variants"], entb["variants"]
        ms_d, ms_t, ms_db, ms_tb = time_interleaved(
            [lambda: tcbf.group_execute(probs, workspace=ws),
             lambda: tcbf.group_execute(probs, workspace=ws, variants=tv),
             lambda: tcbf.group_execute(probs_b, workspace=ws, layout=tcbf.BLOCKED),
             lambda: tcbf.group_execute(probs_b, workspace=ws, layout=tcbf.BLOCKED, variants=tvb)], st, 1)
        # the grouped call prepared once (table built at construction), and
        # the grouped call and the separate launches replayed from HIP graphs
        gc = tcbf.GroupCall(probs, workspace=ws)
        ms_gp = time_launches(gc, st, 1)
        ms_gg = time_graph(lambda: tcbf.group_execute(probs, workspace=ws))
        ms_sg = time_graph(each)
        dflt = [tcbf.Plan(1, M, N, K, tcbf.F16).info()["variant"] for (M, N, K) in shapes]
        dflt_b = [tcbf.Plan(1, M, N, K, tcbf.F16, a_layout=tcbf.BLOCKED).info()["variant"] for (M, N, K) in shapes]
        del probs_b
        # value: the prepared call (what a loop over the same buffers runs);
        # group_execute, which checks the tuples and builds the table on
        # every call, beside it
        tops = ops / (ms_gp * 1e-3) / 1e12
        out.append({"workload": "grouped fp16: " + label,
                    "kernel": "cgemm_f16_group_kernel + cgemm_f16_pp_group_kernel", "value": round(tops, 1),
                    "unit": "TeraOps/s", "ms_per_launch": round(ms_gp, 4),
                    "group_execute_tops": round(ops / (ms_g * 1e-3) / 1e12, 1),
                    "group_execute_ms": round(ms_g, 4),
                    "blocked_weights_tops": round(ops / (ms_gb * 1e-3) / 1e12, 1),
                    "separate_launches_tops": round(ops / (ms_s * 1e-3) / 1e12, 1),
                    "separate_launches_ms": round(ms_s, 4), "dtype": "f16",
                    "prepared_call": {"ms_per_call": round(ms_gp, 4),
                                      "tops": round(ops / (ms_gp * 1e-3) / 1e12, 1),
                                      "note": "GroupCall: the problem table built once, each call passes it"},
                    "graph_replay": {"ms_per_call": round(ms_gg, 4), "tops": round(ops / (ms_gg * 1e-3) / 1e12, 1),
                                     "separate_launches_ms": round(ms_sg, 4),
                                     "separate_launches_tops": round(ops / (ms_sg * 1e-3) / 1e12, 1),
                                     "note": "the calls captured in a HIP graph and replayed: device time "
                                             "without the host's per-call enqueue"},
                    "tuned": {"planar": {"default_tops": round(ops / (ms_d * 1e-3) / 1e12, 1),
                                         "tuned_tops": round(ops / (ms_t * 1e-3) / 1e12, 1),
                                         "policy": ent["policy"], "tuner_ms": ent["ms"],
                                         "default_variants": dflt, "tuned_variants": tv},
                              "blocked": {"default_tops": round(ops / (ms_db * 1e-3) / 1e12, 1),
                                          "tuned_tops": round(ops / (ms_tb * 1e-3) / 1e12, 1),
                                          "policy": entb["policy"], "tuner_ms": entb["ms"],
                                          "default_variants": dflt_b, "tuned_variants": tvb},
                              "note": "default and tuned timed in alternating rounds after tuning"},
                    "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F16_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(tops / PEAK_F16_TFLOPS, 4)}})
        del probs, plans
    # the same small-job mix in FP8 (per-row scales), codes made on the GPU
    shapes = wl.mixed_shapes(0, 32, m_range=(128, 512), n_range=(256, 1024), k_range=(64, 512))
    probs, plans = [], []
    for (M, N, K) in shapes:
        Wg = torch.randn((1, 2, M, K), device="cuda:0", generator=g).half()
        Xg = torch.randint(-127, 128, (1, 2, K, N), device="cuda:0", generator=g).half()
        Wq, Ws = tcbf.quantize_e4m3(Wg, k_major=True, block=0)
        Xq, Xs = tcbf.quantize_e4m3(Xg, k_major=False, block=0)
        probs.append((Wq, Xq, torch.empty((1, 2, M, N), device="cuda:0"), Ws, Xs))
        plans.append(tcbf.Plan(1, M, N, K, tcbf.F8_E4M3))
    ops = sum(8.0 * M * N * K for (M, N, K) in shapes)
    ms_g = time_launches(lambda: tcbf.group_execute(probs, workspace=ws, dtype=tcbf.F8_E4M3), st, 1)

    def each8():
        for pl, (Wq, Xq, Cg, Ws, Xs) in zip(plans, probs):
            pl.execute(Wq, Xq, Cg, Ws, Xs)
    ms_s = time_launches(each8, st, 1)
    gc = tcbf.GroupCall(probs, workspace=ws, dtype=tcbf.F8_E4M3)
    ms_gp = time_launches(gc, st, 1)
    ms_gg = time_graph(lambda: tcbf.group_execute(probs, workspace=ws, dtype=tcbf.F8_E4M3))
    ms_sg = time_graph(each8)
    tops = ops / (ms_gp * 1e-3) / 1e12
    out.append({"workload": "grouped fp8 per-row: 32 small jobs, M~U[128,512] N~U[256,1024] K~U[64,512]",
                "kernel": "cgemm_f8_group_kernel", "value": round(tops, 1), "unit": "TeraOps/s",
                "ms_per_launch": round(ms_gp, 4), "group_execute_tops": round(ops / (ms_g * 1e-3) / 1e12, 1),
                "group_execute_ms": round(ms_g, 4), "separate_launches_tops": round(ops / (ms_s * 1e-3) / 1e12, 1),
                "separate_launches_ms": round(ms_s, 4), "dtype": "e4m3",
                "prepared_call": {"ms_per_call": round(ms_gp, 4), "tops": round(ops / (ms_gp * 1e-3) / 1e12, 1)},
                "graph_replay": {"ms_per_call": round(ms_gg, 4), "tops": round(ops / (ms_gg * 1e-3) / 1e12, 1),
                                 "separate_launches_ms": round(ms_sg, 4),
                                 "separate_launches_tops": round(ops / (ms_sg * 1e-3) / 1e12, 1)},
                "roofline": {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_F8_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tops / PEAK_F8_TFLOPS, 4)}})
    del probs, plans
    torch.cuda.empty_cache()
    if serving:
        out.append(bench_serving())
    return out


def bench_lofar_k64(steps):
    """The LOFAR beamformer shape with 64 stations (256 x 1024 x 1024 x 64,
    fp16, blocked weights): memory-bound (60 ops per byte), scored against HBM
    bandwidth."""
    import torch
    import paper_2505_03269_amd as tcbf
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    batch, M, N, K = 256, 1024, 1024, 64
    plan = tcbf.Plan(batch, M, N, K, tcbf.F16, a_layout=tcbf.BLOCKED)
    info = plan.info()
    A = tcbf.block_weights(torch.randn((batch, 2, M, K), device="cuda:0", generator=g).half())
    B = torch.randint(-127, 128, plan.shape_b(), device="cuda:0", generator=g).half()
    C = plan.empty_output()
    ms = time_launches(lambda: plan.execute(A, B, C), max(steps, 20), 3)
    gbs = info["algorithmic_bytes"] / (ms * 1e-3) / 1e9
    del A, B, C
    torch.cuda.empty_cache()
    return {"workload": "lofar-stations fp16: batch=256 M=1024 K=64 N=1024", "kernel": info["kernel_name"],
            "value": round(gbs, 1), "unit": "GB/s", "ms_per_launch": round(ms, 4),
            "tops": round(info["useful_ops"] / (ms * 1e-3) / 1e12, 1), "dtype": "f16",
            "layout": "W receiver-blocked, X planar",
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4),
                         "algorithmic_bytes": info["algorithmic_bytes"]}}


def bench_serving(warmup=1000, measured=10000):
    """Served mixed stream: 16 resident weight sets per dtype (fp16, FP8
    per-row, 1-bit), jobs uniform over them, N ~ U[256, 8192]; a closed-loop
    run gives the sustained capacity, then Poisson arrivals at 80% and 50% of
    it.  Latency is completion seen by the host minus arrival."""
    from paper_2505_03269_amd import serve
    srv = serve.Server(seed=0)
    srv.run(srv.make_jobs(warmup, None, seed=100))
    closed = srv.run(srv.make_jobs(measured, None, seed=200))
    cap = measured / closed["makespan_s"]
    runs, overlap = {}, {}
    for load in (0.8, 0.5):
        runs[load] = srv.run(srv.make_jobs(measured, load * cap, seed=300 + int(load * 10)))
        overlap[load] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in srv.device_overlap().items()}
    r = runs[0.8]
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}  # noqa: E731
    # the same server with the autotuner's per-weight-set fp16 variants:
    # closed-loop capacity and the 80% run at the default runs' arrival rate
    t0 = time.perf_counter()
    srv.tune_weights()
    tune_s = time.perf_counter() - t0
    srv.run(srv.make_jobs(warmup // 4, None, seed=101))
    closed_t = srv.run(srv.make_jobs(measured, None, seed=200))
    open_t = srv.run(srv.make_jobs(measured, 0.8 * cap, seed=308))
    srv.use_tuned = False
    variants = sorted(set(srv.f16_variants.values()))
    return {"workload": "served mixed stream: fp16/fp8/1-bit jobs, 16 resident weight sets per dtype, "
                        "M~U[128,4096] K~U[64,2048] N~U[256,8192], Poisson arrivals at 80% of capacity",
            "kernel": "cgemm_f16_group_kernel + cgemm_f16_pp_group_kernel + cgemm_f8_group_kernel + "
                      "cgemm_1bit_group_kernel",
            "value": round(r["tops"], 1), "unit": "TeraOps/s", "p50_ms": round(r["p50_ms"], 3),
            "p99_ms": round(r["p99_ms"], 3), "capacity_jobs_per_s": round(cap, 1),
            "closed_loop": rnd(closed), "load_0.8": rnd(runs[0.8]), "load_0.5": rnd(runs[0.5]),
            "device_overlap_0.8": overlap[0.8], "device_overlap_0.5": overlap[0.5],
            "device_overlap_note": "batches on different streams in progress at the same device time "
                                   "(timing events around each batch on its own stream)",
            "tuned": {"closed_loop_tops": round(closed_t["tops"], 1),
                      "capacity_jobs_per_s": round(measured / closed_t["makespan_s"], 1),
                      "load_0.8_tops": round(open_t["tops"], 1), "load_0.8_p50_ms": round(open_t["p50_ms"], 3),
                      "load_0.8_p99_ms": round(open_t["p99_ms"], 3), "variants_used": variants,
                      "tuning_s": round(tune_s, 2),
                      "note": "fp16 variants tuned per weight set at N in {256..8192}; same job streams"},
            "completed": r["completed"], "rejected": r["rejected"], "failed": r["failed"],
            "warmup_jobs": warmup, "measured_jobs": measured, "streams": len(srv.streams),
            "budget_bytes": srv.budget}


def sweep(steps):
    """The paper's measurement shapes, synthetic data, one JSON line each:
    the LOFAR beamformer sweep (256 x 1024 beams x 1024 samples, 8..512
    stations, Sec. V-B) and the roofline shapes (Sec. IV-B)."""
    import torch
    import paper_2505_03269_amd as tcbf
    shapes = [("lofar-stations", tcbf.F16, 256, 1024, 1024, k) for k in
              (8, 16, 24, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 448, 512)]
    shapes += [("roofline-f16-small", tcbf.F16, 256, 1024, 1024, 64), ("roofline-f16-big", tcbf.F16, 1, 8192, 8192, 8192),
               ("roofline-int1-small", tcbf.INT1, 256, 1024, 1024, 256)]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    copy_gbs = measure_copy()["gbs"]
    for name, dt, batch, M, N, K in shapes:
        # fp16: receiver-blocked weights (repacked once), planar timed beside
        lay = tcbf.BLOCKED if dt == tcbf.F16 else tcbf.PLANAR
        plan = tcbf.Plan(batch, M, N, K, dt, a_layout=lay)
        info = plan.info()
        ms_p = None
        if dt == tcbf.INT1:
            A = torch.randint(-2**31, 2**31 - 1, plan.shape_a(), dtype=torch.int32, device="cuda:0", generator=g)
            B = torch.randint(-2**31, 2**31 - 1, plan.shape_b(), dtype=torch.int32, device="cuda:0", generator=g)
            peak = PEAK_I8_TOPS
            C = plan.empty_output()
            ms = time_launches(lambda: plan.execute(A, B, C), steps, 2)
        else:
            Ap = torch.randn((batch, 2, M, K), device="cuda:0", generator=g).half()
            A = tcbf.block_weights(Ap)
            B = torch.randint(-127, 128, plan.shape_b(), device="cuda:0", generator=g).half()
            peak = PEAK_F16_TFLOPS
            C = plan.empty_output()
            plan_p = tcbf.Plan(batch, M, N, K, dt)
            ms, ms_p = time_interleaved([lambda: plan.execute(A, B, C), lambda: plan_p.execute(Ap, B, C)],
                                        steps, 2)
            del Ap
            # the same launches over rotating copies of the inputs (at least
            # 1.2 GB in all), so that no launch finds its inputs still in the
            # 256 MB last-level cache from the launch before
            in_bytes = (A.numel() + B.numel()) * 2
            sets = int(min(16, max(2, -(-1.2e9 // in_bytes))))
            As = [A] + [A.clone() for _ in range(sets - 1)]
            Bs = [B] + [B.clone() for _ in range(sets - 1)]
            rot = [0]

            def cold():
                i = rot[0] % sets
                rot[0] += 1
                plan.execute(As[i], Bs[i], C)
            ms_c = time_launches(cold, max(steps, 2 * sets), sets)
            del As, Bs
        tops = info["useful_ops"] / (ms * 1e-3) / 1e12
        gbs = info["algorithmic_bytes"] / (ms * 1e-3) / 1e9
        ai = info["useful_ops"] / info["algorithmic_bytes"]
        ridge = peak * 1e3 / PEAK_HBM_GBS
        bound = "mfma" if ai >= ridge else "hbm"
        frac = tops / peak if bound == "mfma" else gbs / PEAK_HBM_GBS
        rec = {"sweep": name, "batch": batch, "M": M, "N": N, "K": K, "dtype": "f16" if dt == tcbf.F16 else "int1",
               "kernel": info["kernel_name"], "variant": info["variant"], "ms": round(ms, 4),
               "tops": round(tops, 1), "gbs_algorithmic": round(gbs, 1), "ops_per_byte": round(ai, 1),
               "bound": bound, "frac_of_bound": round(frac, 4)}
        if ms_p is not None:
            gbs_c = info["algorithmic_bytes"] / (ms_c * 1e-3) / 1e9
            rec.update({"weights": "blocked", "planar_weights_tops": round(info["useful_ops"] / (ms_p * 1e-3) / 1e12, 1),
                        "input_mb": round(in_bytes / 1e6, 1),
                        "cold_inputs": {"ms": round(ms_c, 4), "tops": round(info["useful_ops"] / (ms_c * 1e-3) / 1e12, 1),
                                        "gbs_algorithmic": round(gbs_c, 1), "input_sets": sets,
                                        "frac_of_measured_copy_rate": round(gbs_c / copy_gbs, 4)},
                        "measured_copy_gbs": copy_gbs,
                        "roofline_ms": round(max(info["algorithmic_bytes"] / (PEAK_HBM_GBS * 1e6),
                                                 info["useful_ops"] / (peak * 1e9)), 4)})
        print(json.dumps(rec), flush=True)
        del A, B, C
        torch.cuda.empty_cache()


def sweep_int1_big(slices=16):
    """The paper's large 1-bit roofline shape, 1 x 32768 x 8192 x 524288
    (Sec. IV-B): about 1.1e18 useful ops, timed as consecutive launches over
    slices of the beams (the same tiles and K loop as one launch; one launch
    of the whole shape would exceed 32-bit byte offsets of the weights), with
    one progress line per slice."""
    import torch
    import paper_2505_03269_amd as tcbf
    M, N, K = 32768, 8192, 524288
    ms_rows = M // slices
    g = torch.Generator(device="cuda:0")
    g.manual_seed(13)
    plan = tcbf.Plan(1, ms_rows, N, K, tcbf.INT1)
    info = plan.info()
    B = torch.randint(-2**31, 2**31 - 1, plan.shape_b(), dtype=torch.int32, device="cuda:0", generator=g)
    A = torch.randint(-2**31, 2**31 - 1, plan.shape_a(), dtype=torch.int32, device="cuda:0", generator=g)
    C = plan.empty_output()
    plan.execute(A, B, C)  # warm-up
    torch.cuda.synchronize()
    total_ms = 0.0
    for i in range(slices):
        A.random_(-2**31, 2**31 - 1, generator=g)  # a new beam slice of weights
        total_ms += time_launches(lambda: plan.execute(A, B, C), 1, 0)
        log("int1-big slice %d/%d: %.1f ms so far" % (i + 1, slices, total_ms))
    ops = 8.0 * M * N * K
    tops = ops / (total_ms * 1e-3) / 1e12
    abytes = 2 * (M + N) * (K // 32) * 4 + 8 * M * N
    rec = {"sweep": "roofline-int1-big", "batch": 1, "M": M, "N": N, "K": K, "dtype": "int1",
           "kernel": info["kernel_name"], "variant": info["variant"], "ms": round(total_ms, 1),
           "tops": round(tops, 1), "ops_per_byte": round(ops / abytes, 1), "bound": "mfma",
           "peak": PEAK_F4_TFLOPS if info["variant"] == 3 else PEAK_I8_TOPS,
           "frac_of_bound": round(tops / (PEAK_F4_TFLOPS if info["variant"] == 3 else PEAK_I8_TOPS), 4),
           "timed_as": "%d launches of %d beams each (sum of HIP-event times)" % (slices, ms_rows)}
    print(json.dumps(rec), flush=True)
    del A, B, C
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the served-stream line (for kernel traces)")
    ap.add_argument("--sweep", action="store_true",
                    help="print one JSON line per paper measurement shape (LOFAR station sweep, roofline shapes)")
    ap.add_argument("--int1-big", action="store_true",
                    help="time the large 1-bit roofline shape 1 x 32768 x 8192 x 524288 (about 4 minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the beamforming product shards over channels with no "
              "exchange, and this benchmark runs and reports a single MI355X (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
    if args.sweep:
        sweep(args.steps)
        return
    if args.int1_big:
        sweep_int1_big()
        return

    W, X, info, ms, tops, spread, planar, blocking, C_head = bench_c2(args.steps, args.warmup)
    log("c2: %.4f ms/launch, %.1f TeraOps/s" % (ms, tops))
    ach_flops = tops  # useful ops are the MFMA flops (8 per complex MAC)
    traffic = recorded_traffic(info["kernel_name"])
    if traffic is not None:
        traffic = round(traffic)
    roofline = {"bound": "mfma", "achieved": round(ach_flops, 1), "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach_flops / PEAK_F16_TFLOPS, 4), "traffic": traffic,
                "algorithmic_bytes": info["algorithmic_bytes"],
                "hbm_gbs_at_algorithmic_bytes": round(info["algorithmic_bytes"] / (ms * 1e-3) / 1e9, 1)}
    probes = None if args.no_secondary else peak_probes()
    if probes is not None:
        roofline["measured_peak"] = probes["f16"]["uniform"]["tops"]
        roofline["frac_of_measured_peak"] = round(ach_flops / probes["f16"]["uniform"]["tops"], 4)
        roofline["measured_peak_random_operands"] = probes["f16"]["random"]["tops"]
        roofline["random_operand_ceiling_frac"] = round(probes["f16"]["random"]["tops"] / PEAK_F16_TFLOPS, 4)
    # the goal set for this shape: 70% of the published fp16 dense peak; with
    # random operands the part's clock drops under power, which caps any
    # kernel near random_operand_ceiling_frac before memory traffic
    roofline["target_frac"] = TARGET_FRAC_F16
    roofline["target_met"] = bool(roofline["frac"] >= TARGET_FRAC_F16)
    samples = {}
    il_line = None if args.no_secondary else bench_c2_interleaved(W, X, args.steps)
    bf_line = None if args.no_secondary else bench_c2_bf16(W, X, args.steps, samples)
    secondary = [] if args.no_secondary else bench_secondary(
        args.steps, samples, serving=not args.no_serving, copy_gbs=probes["hbm_copy"]["gbs"],
        valu_peak=probes["valu_xor_popc"]["uniform"]["tops"])
    cpu = accuracy = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, X, C_head)
        accuracy = cpu.pop("accuracy")
        log("cpu baseline: %s" % {k: v for k, v in cpu.items() if k != "sample"})
        if "c1" in samples:
            secondary[0]["cpu_baseline"] = cpu_leg_c1(samples["c1"])
        if "c3" in samples:
            c3 = samples["c3"]
            secondary[c3["line"]]["cpu_baseline"] = cpu_leg_c3(c3["W0"], c3["X0"], c3["C0"], c3["K"])
        if "c4" in samples:
            c4 = samples["c4"]
            leg = cpu_leg_c4(c4["Ws"], c4["X"], c4["ms"], c4["outs"])
            acc = leg.pop("accuracy")
            secondary[c4["lines"]["f16"]]["cpu_baseline"] = leg
            for key, i in c4["lines"].items():
                if key in acc:
                    secondary[i]["accuracy"] = acc[key]
        if "bf16" in samples and bf_line is not None:
            bf_line["accuracy"] = cpu_leg_bf16(samples["bf16"])
    del W, X, C_head
    if bf_line is not None:
        secondary.insert(0, bf_line)  # after the CPU legs, which address lines by index
    if il_line is not None:
        secondary.insert(0, il_line)
    line = {
        "metric": METRIC, "value": round(tops, 2), "unit": "TeraOps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic (seeded phasor weights from random 2-D antenna geometry, 8-bit complex Gaussian data)",
        "config": {"workload": "radio-astro-fp16", "batch": 256, "M": 1024, "K": 576, "N": 4096,
                   "layout": "W receiver-blocked (repacked once), X planar, out planar",
                   "tile": [info["tile_m"], info["tile_n"], info["tile_k"]],
                   "kernel": info["kernel_name"], "workgroups": info["workgroups"]},
        "pct_of_fp16_peak": round(100.0 * tops / PEAK_F16_TFLOPS, 2),
        "launch_spread": spread,
        "weights_planar": planar,
        "weight_blocking": blocking,
        "roofline": roofline,
        "peak_probe": probes,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
