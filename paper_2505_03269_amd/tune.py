"""Autotuner: choose the fastest kernel variant for one problem shape by timing
every valid candidate on the device, and remember the choice in a JSON cache.

The paper tunes its kernel's compile-time parameters per GPU and shape with an
external tuner and ships the best points (Sec. IV-A, Table 3).  Here the
candidate configurations are the variants compiled into the library; the
sweep starts from the variant closest to Table 3's MI300X/MI300A float16 point
(128 x 128 complex outputs per workgroup, 64-row wave tiles), then tries the
rest.  Timing uses HIP events on the stream the library launches on, over
inputs resident on the device; the cache key is the device architecture, the
dtype, the exact problem shape and layouts, and the kernel set (a hash of the
built library and the candidate lists).

Only timing and bookkeeping happen here; every product runs in the library.
"""
import hashlib
import json
import os

from . import F16, F8_E4M3, INT1, LIB_PATH, MXF8_E4M3, PLANAR, Plan, TcbfError


def _layouts(dtype, operand_layout):
    """(a_layout, b_layout) of a plan: the operand layout applies to W (and,
    for FP8, to X as well; a blocked fp16 plan keeps X planar)."""
    fp8 = dtype in (F8_E4M3, MXF8_E4M3)
    return operand_layout, (operand_layout if fp8 else PLANAR)

# candidate variants per dtype, seed first
CANDIDATES = {
    F16: [2, 9, 8, 6, 3, 4, 5, 7, 1],   # 2: Table 3's MI300X point (128 x 128 tile, 2 x 2 waves of 64 x 64)
    F8_E4M3: [1, 3, 2],   # 3: the 256 x 128 ping-pong persistent kernel
    MXF8_E4M3: [1, 3, 2],
    INT1: [1, 3, 2],
}


_KERNEL_SET = None


def kernel_set_id():
    """Identity of the kernel set a cached choice refers to: a hash of the
    built library and of the candidate lists.  A rebuilt library with other
    kernels behind the same variant numbers, or a changed candidate list,
    gets new cache keys (so it is tuned again instead of reusing a choice
    made among other kernels)."""
    global _KERNEL_SET
    if _KERNEL_SET is None:
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        h.update(json.dumps({str(k): v for k, v in CANDIDATES.items()}, sort_keys=True).encode())
        _KERNEL_SET = h.hexdigest()[:12]
    return _KERNEL_SET


def cache_key(arch, dtype, batch, M, N, K, c_layout=PLANAR, a_shared=False, operand_layout=PLANAR, kernel_set=None):
    key = "%s|dtype%d|%dx%dx%dx%d|c%d|s%d" % (arch, int(dtype), batch, M, N, K, int(c_layout), int(bool(a_shared)))
    if operand_layout != PLANAR:
        key += "|op%d" % int(operand_layout)
    return key + "|ks" + (kernel_set if kernel_set is not None else kernel_set_id())


def load_cache(path):
    if path is None or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(path, cache):
    if path is None:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def valid_candidates(batch, M, N, K, dtype, c_layout=PLANAR, a_shared=False, device=0, operand_layout=PLANAR):
    """Variants the library accepts for this problem (plan creation succeeds)."""
    out = []
    al, bl = _layouts(dtype, operand_layout)
    for v in CANDIDATES[dtype]:
        try:
            Plan(batch, M, N, K, dtype, a_layout=al, b_layout=bl, c_layout=c_layout, a_shared=a_shared, variant=v,
                 device=device)
        except TcbfError:
            continue
        out.append(v)
    return out


def _device_inputs(plan):
    import torch
    dev = "cuda:%d" % plan.device
    g = torch.Generator(device=dev)
    g.manual_seed(1234)
    ta, tb, _ = plan._dtypes()
    if plan.dtype == INT1:
        A = torch.randint(-2**31, 2**31 - 1, plan.shape_a(), dtype=torch.int32, device=dev, generator=g)
        B = torch.randint(-2**31, 2**31 - 1, plan.shape_b(), dtype=torch.int32, device=dev, generator=g)
        kw = (plan.K + 31) // 32
        if plan.K % 32:
            mask = (1 << (plan.K % 32)) - 1
            A[..., kw - 1] &= mask
            B[..., kw - 1] &= mask
        return A, B, None, None
    if plan.dtype in (F8_E4M3, MXF8_E4M3):
        A = torch.randint(0, 0x7F, plan.shape_a(), dtype=torch.uint8, device=dev, generator=g)
        B = torch.randint(0, 0x7F, plan.shape_b(), dtype=torch.uint8, device=dev, generator=g)
        if plan.dtype == F8_E4M3:
            sa = torch.ones(plan.shape_a_scale(), dtype=torch.float32, device=dev)
            sb = torch.ones(plan.shape_b_scale(), dtype=torch.float32, device=dev)
        else:
            sa = torch.full(plan.shape_a_scale(), 127, dtype=torch.uint8, device=dev)
            sb = torch.full(plan.shape_b_scale(), 127, dtype=torch.uint8, device=dev)
        return A, B, sa, sb
    A = torch.randn(plan.shape_a(), device=dev, generator=g).to(ta)
    B = torch.randn(plan.shape_b(), device=dev, generator=g).to(tb)
    return A, B, None, None


def measure(plan, reps=10, warmup=2, inputs=None):
    """Mean milliseconds per launch of `plan` (HIP events on the current stream)."""
    import torch
    A, B, sa, sb = inputs if inputs is not None else _device_inputs(plan)
    C = plan.empty_output()
    run = (lambda: plan.execute(A, B, C, sa, sb)) if sa is not None else (lambda: plan.execute(A, B, C))
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        run()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def tune(batch, M, N, K, dtype=F16, c_layout=PLANAR, a_shared=False, cache_path=None, reps=10, warmup=2,
         device=0, arch=None, measure_fn=None, force=False, operand_layout=PLANAR):
    """Time every valid variant (seed first) and return
    {"variant": best, "ms": {variant: ms}}; cached under cache_path.
    operand_layout=BLOCKED tunes the receiver-blocked operand form."""
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    key = cache_key(arch, dtype, batch, M, N, K, c_layout, a_shared, operand_layout)
    cache = load_cache(cache_path)
    if key in cache and not force:
        return cache[key]
    cands = valid_candidates(batch, M, N, K, dtype, c_layout, a_shared, device, operand_layout)
    al, bl = _layouts(dtype, operand_layout)
    if not cands:
        raise TcbfError(2, "no kernel variant accepts this problem")
    timings = {}
    inputs = None
    for v in cands:
        plan = Plan(batch, M, N, K, dtype, a_layout=al, b_layout=bl, c_layout=c_layout, a_shared=a_shared,
                    variant=v, device=device)
        if measure_fn is not None:
            ms = measure_fn(plan)
        else:
            if inputs is None:
                inputs = _device_inputs(plan)
            ms = measure(plan, reps, warmup, inputs)
        timings[str(v)] = round(float(ms), 5)
    best = min(cands, key=lambda v: timings[str(v)])
    entry = {"variant": best, "ms": timings, "seed": cands[0]}
    cache = load_cache(cache_path)  # re-read: another process may have added keys
    cache[key] = entry
    save_cache(cache_path, cache)
    return entry


def tuned_plan(batch, M, N, K, dtype=F16, c_layout=PLANAR, a_shared=False, cache_path=None, device=0,
               operand_layout=PLANAR, **kw):
    """A Plan with the cached (or freshly tuned) variant for this shape."""
    entry = tune(batch, M, N, K, dtype, c_layout, a_shared, cache_path=cache_path, device=device,
                 operand_layout=operand_layout, **kw)
    al, bl = _layouts(dtype, operand_layout)
    return Plan(batch, M, N, K, dtype, a_layout=al, b_layout=bl, c_layout=c_layout, a_shared=a_shared,
                variant=entry["variant"], device=device)


def group_variant(entry):
    """The variant a grouped launch runs for a problem whose single-plan
    tuning gave `entry`: the tuned variant, or, where that is the generic
    kernel (which has no grouped form), the fastest variant that has one."""
    if entry["variant"] != 1:
        return entry["variant"]
    rest = [(ms, int(v)) for v, ms in entry["ms"].items() if int(v) != 1]
    if not rest:
        raise TcbfError(2, "no grouped kernel accepts this problem")
    return min(rest)[1]


def group_variants(shapes, dtype=F16, c_layout=PLANAR, operand_layout=PLANAR, cache_path=None, device=0, **kw):
    """Per-problem variants for a grouped launch of problems with the given
    (batch, M, N, K[, a_shared]) shapes: each fp16 problem takes the variant
    its own tuned plan runs (cached per shape, see tune()); FP8 and 1-bit
    problems take 0 (their grouped kernels have one tile shape)."""
    out = []
    memo = {}
    for s in shapes:
        batch, M, N, K = s[:4]
        a_shared = bool(s[4]) if len(s) > 4 else False
        if dtype != F16:
            out.append(0)
            continue
        key = (batch, M, N, K, a_shared)
        if key not in memo:
            memo[key] = group_variant(tune(batch, M, N, K, dtype, c_layout, a_shared, cache_path=cache_path,
                                           device=device, operand_layout=operand_layout, **kw))
        out.append(memo[key])
    return out


def group_cache_key(arch, dtype, shapes, c_layout=PLANAR, operand_layout=PLANAR, kernel_set=None):
    """Key of a grouped launch's tuned variants: the problems' shapes in
    order (a problem's position picks its entry in the variant list)."""
    sig = ",".join("%dx%dx%dx%d%s" % (s[0], s[1], s[2], s[3], "s" if len(s) > 4 and s[4] else "") for s in shapes)
    return "%s|dtype%d|group[%s]|c%d|op%d|ks%s" % (arch, int(dtype), sig, int(c_layout), int(operand_layout),
                                                kernel_set if kernel_set is not None else kernel_set_id())


def _accepts(s, variant, dtype, c_layout, operand_layout, device):
    al, bl = _layouts(dtype, operand_layout)
    try:
        Plan(s[0], s[1], s[2], s[3], dtype, a_layout=al, b_layout=bl, c_layout=c_layout,
             a_shared=bool(s[4]) if len(s) > 4 else False, variant=variant, device=device)
    except TcbfError:
        return False
    return True


def group_policies(shapes, dtype=F16, c_layout=PLANAR, operand_layout=PLANAR, device=0, cache_path=None, **kw):
    """Candidate per-problem variant lists for a grouped fp16 launch:
    "default" (every problem's default plan), "per_problem" (each problem's
    own tuned plan, see group_variants), "ping_pong" (the 256 x 128
    persistent tile wherever a problem takes it, else variant 2) and
    "small_tiles" (the 128 x 128 tile, variant 2, for every problem)."""
    pp = [9 if _accepts(s, 9, dtype, c_layout, operand_layout, device) else 2 for s in shapes]
    return {"default": [0] * len(shapes),
            "per_problem": group_variants(shapes, dtype, c_layout, operand_layout, cache_path, device, **kw),
            "ping_pong": pp,
            "small_tiles": [2] * len(shapes)}


def tune_group(shapes, measure_fn, dtype=F16, c_layout=PLANAR, operand_layout=PLANAR, cache_path=None, device=0,
               arch=None, force=False, **kw):
    """Choose the per-problem variants of a grouped fp16 launch by timing the
    launch itself: every candidate list of group_policies() is timed with
    measure_fn(variants) -> ms (the caller's grouped launch on its own
    buffers) and the fastest is kept, cached under the group's shapes.
    Returns {"variants": [...], "policy": name, "ms": {name: ms}}.  FP8 and
    1-bit groups have one tile shape: every variant is 0."""
    if dtype != F16:
        return {"variants": [0] * len(shapes), "policy": "default", "ms": {}}
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    key = group_cache_key(arch, dtype, shapes, c_layout, operand_layout)
    cache = load_cache(cache_path)
    if key in cache and not force:
        return cache[key]
    cands = group_policies(shapes, dtype, c_layout, operand_layout, device, cache_path, **kw)
    timings, seen = {}, {}
    for name, variants in cands.items():
        t = tuple(variants)
        if t in seen:   # the same lists under two names: timed once
            timings[name] = timings[seen[t]]
            continue
        seen[t] = name
        timings[name] = round(float(measure_fn(list(variants))), 5)
    best = min(cands, key=lambda n: timings[n])
    entry = {"variants": list(cands[best]), "policy": best, "ms": timings}
    cache = load_cache(cache_path)
    cache[key] = entry
    save_cache(cache_path, cache)
    return entry
