"""The C-ABI library loads, exports every symbol include/tcbf.h declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2505_03269_amd as tcbf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcbf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcbf_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared_functions() == sorted(tcbf.EXPORTS)


def test_library_exports_every_symbol():
    L = tcbf.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", tcbf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for name in _declared_functions():
        assert name in exported, name


def test_library_is_built_for_gfx950():
    data = open(tcbf.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_status_strings_and_version():
    assert tcbf.status_string(0) == "TCBF_SUCCESS"
    assert tcbf.status_string(1) == "TCBF_ERROR_INVALID_VALUE"
    assert tcbf.status_string(4) == "TCBF_ERROR_DEVICE"
    assert tcbf.status_string(99) == "TCBF_UNKNOWN_STATUS"
    assert tcbf.lib().tcbf_version() == 4


def _plan_status(**kw):
    d = dict(struct_size=ctypes.sizeof(tcbf.PlanDesc), device=0, batch=2, M=8, N=8, K=8, dtype=tcbf.F16,
             a_layout=0, b_layout=0, c_layout=0, a_shared=0, variant=0)
    d.update(kw)
    desc = tcbf.PlanDesc(**d)
    h = ctypes.c_void_p()
    st = tcbf.lib().tcbf_plan(ctypes.byref(desc), ctypes.byref(h))
    if st == 0:
        tcbf.lib().tcbf_plan_destroy(h)
    else:
        assert not h.value
    return st


@pytest.mark.parametrize("bad", [
    dict(struct_size=4), dict(batch=0), dict(M=0), dict(N=-1), dict(K=0), dict(dtype=7),
    dict(a_layout=3), dict(b_layout=-1), dict(c_layout=5), dict(variant=-1), dict(variant=10),
    # the receiver-blocked layout: fp16 weights only, fast kernel with 32 receivers per stage
    dict(b_layout=tcbf.BLOCKED), dict(c_layout=tcbf.BLOCKED), dict(dtype=tcbf.INT1, a_layout=tcbf.BLOCKED),
    dict(dtype=tcbf.F8_E4M3, a_layout=tcbf.BLOCKED), dict(dtype=tcbf.MXF8_E4M3, a_layout=tcbf.BLOCKED),
    dict(dtype=tcbf.F8_E4M3, b_layout=tcbf.BLOCKED), dict(dtype=tcbf.INT1, b_layout=tcbf.BLOCKED),
    dict(dtype=tcbf.F8_E4M3, a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED, N=6),
    dict(a_layout=tcbf.BLOCKED, b_layout=tcbf.INTERLEAVED, N=12), dict(a_layout=tcbf.BLOCKED, N=12),
    dict(a_layout=tcbf.BLOCKED, b_layout=tcbf.INTERLEAVED, variant=2),
    dict(a_layout=tcbf.BLOCKED, variant=1), dict(a_layout=tcbf.BLOCKED, variant=3),
    dict(a_layout=tcbf.BLOCKED, variant=4), dict(a_layout=tcbf.BLOCKED, variant=7),
    dict(dtype=tcbf.INT1, a_layout=tcbf.INTERLEAVED), dict(dtype=tcbf.INT1, b_layout=tcbf.INTERLEAVED),
    dict(dtype=tcbf.INT1, variant=7),
    dict(dtype=tcbf.F8_E4M3, a_layout=tcbf.INTERLEAVED), dict(dtype=tcbf.MXF8_E4M3, b_layout=tcbf.INTERLEAVED),
    dict(dtype=tcbf.F8_E4M3, N=6), dict(dtype=tcbf.MXF8_E4M3, N=1), dict(dtype=tcbf.F8_E4M3, variant=4),
    # FP8 ping-pong with per-block scales: every 8-stage scale group spans two stages or more
    dict(dtype=tcbf.MXF8_E4M3, variant=3, K=576), dict(dtype=tcbf.MXF8_E4M3, variant=3, K=1),
    dict(dtype=tcbf.MXF8_E4M3, a_layout=tcbf.BLOCKED, b_layout=tcbf.BLOCKED, variant=3, K=2049),
    dict(dtype=5),
    # bfloat16: variants 1, 2 and 9 only (9 with planar X), not in grouped launches
    dict(dtype=tcbf.BF16, variant=3), dict(dtype=tcbf.BF16, variant=6), dict(dtype=tcbf.BF16, variant=8),
    dict(dtype=tcbf.BF16, b_layout=tcbf.INTERLEAVED, variant=9), dict(dtype=tcbf.BF16, a_layout=tcbf.BLOCKED, variant=1),
    # receiver-contiguous X and strided W (descriptor fields of version 4)
    dict(reserved=1), dict(b_k_contiguous=2), dict(a_batch_stride=-8), dict(a_shared=1, a_batch_stride=1024),
    dict(a_batch_stride=8), dict(a_batch_stride=132), dict(b_k_contiguous=1, variant=2),
    dict(b_k_contiguous=1, variant=9), dict(b_k_contiguous=1, b_layout=tcbf.BLOCKED),
    dict(dtype=tcbf.INT1, a_batch_stride=12), dict(dtype=tcbf.F8_E4M3, a_batch_stride=8 * 32),
    dict(a_layout=tcbf.BLOCKED, a_batch_stride=2 * 8 * 8),
])
def test_bad_descriptors_rejected_without_device(bad):
    assert _plan_status(**bad) == 1


def test_version4_fields_accepted_and_short_descriptor_ignores_them():
    """Valid strides and receiver-contiguous X pass validation (the plan then
    needs a device); a descriptor whose struct_size ends before the version-4
    fields is read without them."""
    for ok in (dict(a_batch_stride=136), dict(a_batch_stride=1 << 20), dict(b_k_contiguous=1),
               dict(b_k_contiguous=1, b_layout=tcbf.INTERLEAVED, variant=1),
               dict(dtype=tcbf.INT1, a_batch_stride=16), dict(dtype=tcbf.F8_E4M3, a_batch_stride=2 * 8 * 32),
               dict(dtype=tcbf.F8_E4M3, b_k_contiguous=1), dict(a_layout=tcbf.BLOCKED, a_batch_stride=2 * 8 * 32)):
        assert _plan_status(**ok) in (0, 4), ok
    v3 = tcbf.PlanDesc.b_k_contiguous.offset
    assert v3 == 64 and ctypes.sizeof(tcbf.PlanDesc) == 80
    assert _plan_status(struct_size=v3, reserved=7, b_k_contiguous=9, a_batch_stride=-1) in (0, 4)
    assert _plan_status(struct_size=v3 - 4) == 1


def test_oversized_rejected():
    assert _plan_status(M=1 << 20, K=1 << 12) == 2
    # blocked weights are padded to whole 32-receiver blocks: 2*M*32*ceil(K/32) elements
    assert _plan_status(a_layout=tcbf.BLOCKED, M=1 << 15, K=(1 << 15) - 31) == 2
    assert _plan_status(dtype=tcbf.INT1, K=(1 << 26) + 1) == 2
    assert _plan_status(dtype=tcbf.F8_E4M3, M=1 << 14, K=1 << 16) == 2   # 2*M*Kp bytes
    assert _plan_status(dtype=tcbf.MXF8_E4M3, M=1 << 14, N=1 << 14) == 2  # 8*M*N bytes


def test_null_arguments():
    L = tcbf.lib()
    h = ctypes.c_void_p()
    assert L.tcbf_plan(None, ctypes.byref(h)) == 1
    assert L.tcbf_execute(None, None, None, None, None, None, None) == 1
    assert L.tcbf_plan_query(None, None) == 1
    assert L.tcbf_plan_destroy(None) == 0
    assert L.tcbf_pack1bit(None, 0, 0, 1, 1, 1, 1, None, None) == 1
    assert L.tcbf_quantize_e4m3(None, 0, 0, 1, 1, 1, 1, 0, 0, None, None, None) == 1
    assert L.tcbf_block_weights(None, 0, 1, 1, 1, None, None) == 1


def test_block_weights_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(256)
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    assert L.tcbf_block_weights(p, tcbf.BLOCKED, 1, 1, 1, p, None) == 1   # blocked source
    assert L.tcbf_block_weights(p, -1, 1, 1, 1, p, None) == 1            # bad layout
    assert L.tcbf_block_weights(p, 0, 0, 1, 1, p, None) == 1             # batch 0
    assert L.tcbf_block_weights(p, 0, 1, 0, 1, p, None) == 1             # M 0
    assert L.tcbf_block_weights(p, 0, 1, 1, 0, p, None) == 1             # K 0
    q = ctypes.c_void_p(addr + 8)
    assert L.tcbf_block_weights(p, 0, 1, 1, 1, q, None) == 1             # misaligned dst
    assert L.tcbf_block_weights(p, 0, 1 << 40, 1 << 20, 1 << 10, p, None) == 2   # too large


def test_f8_codes_shape():
    assert tcbf.f8_codes_shape(2, 10, 100) == (2, 2, 10, 128)
    assert tcbf.f8_codes_shape(2, 10, 100, tcbf.BLOCKED) == (2, 2, 2, 10, 64)
    assert tcbf.f8_codes_shape(1, 3, 8192, tcbf.BLOCKED) == (1, 2, 128, 3, 64)
    assert tcbf.f8_codes_shape(1, 3, 33, tcbf.BLOCKED) == (1, 2, 1, 3, 64)


def test_blocked_shape():
    assert tcbf.blocked_shape(3, 100, 1) == (3, 2, 1, 100, 32)
    assert tcbf.blocked_shape(1, 8, 64) == (1, 2, 2, 8, 32)
    assert tcbf.blocked_shape(2, 8, 65) == (2, 2, 3, 8, 32)


def test_pack_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(256)
    # 16-byte aligned host pointers pass the pointer checks; every call below
    # fails on a size/enum/alignment check before anything is launched
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    assert L.tcbf_pack1bit(p, 9, 0, 1, 1, 1, 1, p, None) == 1       # bad source type
    assert L.tcbf_pack1bit(p, 0, 3, 1, 1, 1, 1, p, None) == 1       # bad layout
    assert L.tcbf_pack1bit(p, 0, 0, 0, 1, 1, 1, p, None) == 1       # batch 0
    assert L.tcbf_pack1bit(p, 0, 0, 1, 1, 0, 1, p, None) == 1       # K 0
    q = ctypes.c_void_p(addr + 4)
    assert L.tcbf_pack1bit(q, 0, 0, 1, 1, 1, 1, p, None) == 1       # misaligned


def test_quantize_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(256)
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    assert L.tcbf_quantize_e4m3(p, 9, 0, 1, 1, 1, 1, 0, 0, p, p, None) == 1     # bad source type
    assert L.tcbf_quantize_e4m3(p, 1, 2, 1, 1, 1, 1, 0, 0, p, p, None) == 1     # bad layout
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 0, 1, p, p, None) == 1     # interleaved output
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 0, 5, p, p, None) == 1     # bad output layout
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 16, 0, p, p, None) == 1    # bad block
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 0, 1, 1, 0, 0, p, p, None) == 1     # rows 0
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 0, 0, p, None, None) == 1  # no scales
    q = ctypes.c_void_p(addr + 4)
    assert L.tcbf_quantize_e4m3(p, 1, 0, 1, 1, 1, 1, 32, 2, p, q, None) == 1    # misaligned scales


def test_steering_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(256)
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    q = ctypes.c_void_p(addr + 4)
    assert L.tcbf_steering_weights(None, p, p, 3e8, 1, 1, 1, 1, 0, p, None) == 1   # NULL positions
    assert L.tcbf_steering_weights(p, p, p, 3e8, 1, 1, 1, 0, 0, p, None) == 1      # int8 output
    assert L.tcbf_steering_weights(p, p, p, 0.0, 1, 1, 1, 1, 0, p, None) == 1      # wave speed 0
    assert L.tcbf_steering_weights(p, p, p, float("nan"), 1, 1, 1, 1, 0, p, None) == 1
    assert L.tcbf_steering_weights(p, p, p, 3e8, 1, 0, 1, 1, 0, p, None) == 1      # M 0
    assert L.tcbf_steering_weights(q, p, p, 3e8, 1, 1, 1, 1, 0, p, None) == 1      # misaligned positions
    assert L.tcbf_steering_weights(p, p, p, 3e8, 1, 1, 1, 2, 2, p, None) == 1      # blocked fp32
    assert L.tcbf_steering_weights(p, p, p, 3e8, 1, 1, 1, 1, 1, p, None) == 1      # interleaved out
    assert L.tcbf_steering_weights(p, p, p, 3e8, 1, 1, 1, 1, 0, ctypes.c_void_p(addr + 8), None) == 1


def test_peak_probe_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(2048)
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    need = 256 * 4 + 32
    assert L.tcbf_peak_probe(5, 1, 1, 0, 0, p, need, None, None) == 1                       # unknown kind
    assert L.tcbf_peak_probe(-1, 1, 1, 0, 0, p, need, None, None) == 1
    assert L.tcbf_peak_probe(0, 1, 1, 0, 2, p, need, None, None) == 1                       # unknown operand mode
    assert L.tcbf_peak_probe(0, 0, 1, 0, 0, p, need, None, None) == 1                       # no blocks
    assert L.tcbf_peak_probe(0, 1, 0, 0, 0, p, need, None, None) == 1                       # no iterations
    assert L.tcbf_peak_probe(0, 1, 1, 0, 0, None, need, None, None) == 1                    # no sink
    assert L.tcbf_peak_probe(0, 1, 1, 0, 0, ctypes.c_void_p(addr + 4), need, None, None) == 1  # misaligned
    assert L.tcbf_peak_probe(0, 1, 1, 0, 0, p, need - 1, None, None) == 1                   # sink too small
    assert L.tcbf_peak_probe(0, 1, 1 << 41, 0, 0, p, need, None, None) == 2                 # too many rounds


def test_group_argument_checks():
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(1024)
    addr = (ctypes.addressof(buf) + 15) & ~15
    p = ctypes.c_void_p(addr)
    good = tcbf.GroupProblem(addr, addr, addr, 1, 8, 8, 8, 0, 0, None, None)
    one = (tcbf.GroupProblem * 1)(good)
    assert L.tcbf_group_execute(0, tcbf.F16, 0, None, 1, p, None) == 1                 # no problems
    assert L.tcbf_group_execute(0, tcbf.F16, 0, one, 0, p, None) == 1                  # count 0
    assert L.tcbf_group_execute(0, tcbf.F16, 0, one, tcbf.GROUP_MAX + 1, p, None) == 1
    assert L.tcbf_group_execute(0, 9, 0, one, 1, p, None) == 1                         # unknown dtype
    assert L.tcbf_group_execute(0, tcbf.BF16, 0, one, 1, p, None) == 1                 # no grouped bfloat16
    int1 = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=8, a_shared=0, layout=0)
    for bad, want in ((dict(a_scale=addr), 1), (dict(K=(1 << 26) + 1), 2), (dict(M=1 << 16, N=1 << 15), 2)):
        d = dict(int1)
        d.update(bad)
        arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
        assert L.tcbf_group_execute(0, tcbf.INT1, 0, arr, 1, p, None) == want, bad
    assert L.tcbf_group_execute(0, tcbf.F16, 0, one, 1, ctypes.c_void_p(addr + 4), None) == 1
    # per-problem variants: fast variants only (not the generic kernel), blocked
    # weights only with the variants that read them, 0 for FP8 and 1-bit
    for bad in (dict(variant=1), dict(variant=10), dict(variant=-1), dict(reserved=1),
                dict(layout=2, variant=3)):
        d = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=8, a_shared=0, layout=0)
        d.update(bad)
        arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
        assert L.tcbf_group_execute(0, tcbf.F16, 0, arr, 1, p, None) == 1, bad
    d = dict(int1, variant=3)
    arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
    assert L.tcbf_group_execute(0, tcbf.INT1, 0, arr, 1, p, None) == 1
    for bad in (dict(K=12), dict(N=4), dict(batch=0), dict(layout=1), dict(layout=3), dict(A=addr + 2),
                dict(a_scale=addr), dict(layout=2, N=4)):
        d = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=8, a_shared=0, layout=0)
        d.update(bad)
        arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
        assert L.tcbf_group_execute(0, tcbf.F16, 0, arr, 1, p, None) == 1, bad
    # blocked layouts: not for 1-bit; one layout per launch
    d = dict(int1)
    d.update(layout=2)
    arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
    assert L.tcbf_group_execute(0, tcbf.INT1, 0, arr, 1, p, None) == 1
    a = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=8, a_shared=0, layout=0)
    b = dict(a, layout=2)
    two = (tcbf.GroupProblem * 2)(tcbf.GroupProblem(**a), tcbf.GroupProblem(**b))
    assert L.tcbf_group_execute(0, tcbf.F16, 0, two, 2, p, None) == 1
    # FP8: scales required and aligned, N a multiple of 4, the plan's size limits
    for dt in (tcbf.F8_E4M3, tcbf.MXF8_E4M3):
        for bad, want in ((dict(), 1), (dict(a_scale=addr), 1), (dict(a_scale=addr, b_scale=addr + 4), 1),
                          (dict(a_scale=addr, b_scale=addr, N=6), 1),
                          (dict(a_scale=addr, b_scale=addr, M=1 << 14, K=1 << 16), 2)):
            d = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=40, a_shared=0, layout=0)
            d.update(bad)
            arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
            assert L.tcbf_group_execute(0, dt, 0, arr, 1, p, None) == want, (dt, bad)


def test_group_noalloc_argument_checks():
    """The allocation-free grouped launch makes the same argument checks as
    the workspace launch, before it looks for a device."""
    L = tcbf.lib()
    buf = ctypes.create_string_buffer(1024)
    addr = (ctypes.addressof(buf) + 15) & ~15
    good = tcbf.GroupProblem(addr, addr, addr, 1, 8, 8, 8, 0, 0, None, None)
    one = (tcbf.GroupProblem * 1)(good)
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 0, None, 1, None) == 1                 # no problems
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 0, one, 0, None) == 1                  # count 0
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 0, one, tcbf.GROUP_MAX + 1, None) == 1
    assert L.tcbf_group_execute_noalloc(0, 9, 0, one, 1, None) == 1                         # unknown dtype
    assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 4, one, 1, None) == 1                  # unknown layout
    for bad in (dict(K=12), dict(N=4), dict(batch=0), dict(A=addr + 2), dict(a_scale=addr)):
        d = dict(A=addr, B=addr, C=addr, batch=1, M=8, N=8, K=8, a_shared=0, layout=0)
        d.update(bad)
        arr = (tcbf.GroupProblem * 1)(tcbf.GroupProblem(**d))
        assert L.tcbf_group_execute_noalloc(0, tcbf.F16, 0, arr, 1, None) == 1, bad


def test_valid_descriptor_without_gpu_reports_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _plan_status() == 4
    with pytest.raises(tcbf.TcbfError):
        tcbf.Plan(1, 4, 4, 4)


def test_no_undefined_internal_symbols():
    """Every kernel the library launches has its host stub defined."""
    out = subprocess.run(["nm", "-D", "--undefined-only", tcbf.LIB_PATH], capture_output=True, text=True).stdout
    missing = [l.split()[-1] for l in out.splitlines() if "tcbf" in l]
    assert not missing, missing


def test_built_library_matches_the_sources():
    """The library was built from the sources in this tree (build writes their
    identity beside it): a stale libtcbf.so would test and measure old code."""
    from paper_2505_03269_amd import build as libbuild
    assert os.path.exists(libbuild.SOURCES_ID), "libtcbf.so has no source identity: rebuild it"
    assert open(libbuild.SOURCES_ID).read().strip() == libbuild.sources_id(), \
        "libtcbf.so was built from other sources: rebuild it (python -m paper_2505_03269_amd.build)"
