"""Lint of the library's gfx950 machine code (compiled here, no GPU needed).

Store-data hazard: a vector-memory store of more than 8 bytes reads its data
registers after it issues; the instruction right after it must not overwrite
them, or the store may write the new value.  The compiler inserts the needed
wait state for stores whose scalar offset is an immediate but not for stores
with a register scalar offset, and a kernel here once stored garbage that way.
The kernels keep every buffer-store offset in the per-lane register; this test
checks the generated code of every source for the pattern itself.

Scratch memory: no kernel on a default path may use private (scratch)
memory.  A kernel whose register arrays the compiler could not keep in
registers (a lambda left out of line, so arrays it captures by reference
escape to memory, or a pointer select the compiler turns into a table of
generic LDS pointers) runs up to an order of magnitude slower with identical
results, which no parity test notices; the kernel descriptors in the generated
code say it directly.  Known users, all off the default paths: the fast-kernel
variants with more than two stage buffers in their epilogue staging (3, 4, 6,
7) and the split ring (8), whose staged-row selects become a scratch table of
LDS pointers.
"""
import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2505_03269_amd import build as libbuild

CSRC = os.path.join(os.path.dirname(libbuild.__file__), "csrc")
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

STORE = re.compile(r"^(buffer_store_dwordx[34]|buffer_store_b(?:96|128))\s+(v\[\d+:\d+\])")
FLAT_STORE = re.compile(r"^((?:global|flat)_store_dwordx[34]|(?:global|flat)_store_b(?:96|128))\s+\S+,\s*(v\[\d+:\d+\])")


def _regs(tok):
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _instructions(asm):
    out = []
    for line in asm.splitlines():
        t = line.split(";")[0].strip()
        if not t or t.startswith(".") or t.endswith(":"):
            continue
        out.append(t)
    return out


def store_data_hazards(asm):
    ins = _instructions(asm)
    found = []
    for i, t in enumerate(ins[:-1]):
        m = STORE.match(t) or FLAT_STORE.match(t)
        if not m:
            continue
        data = _regs(m.group(2))
        nxt = ins[i + 1]
        if nxt.startswith("v_"):
            dst = nxt.split()[1].rstrip(",")
            if _regs(dst) & data:
                found.append((t, nxt))
    return found


def test_detector_flags_the_pattern():
    asm = ("\tbuffer_store_dwordx4 v[4:7], v16, s[16:19], s11 offen\n"
           "\tv_or_b32_e32 v4, s2, v14\n"
           "\tbuffer_store_dwordx4 v[8:11], v17, s[16:19], 0 offen\n"
           "\tv_add_u32_e32 v95, v1, v85\n"
           "\tv_or_b32_e32 v8, s2, v96\n")
    assert store_data_hazards(asm) == [("buffer_store_dwordx4 v[4:7], v16, s[16:19], s11 offen",
                                        "v_or_b32_e32 v4, s2, v14")]


def scratch_users(asm):
    """Kernels whose descriptor asks for private (scratch) memory."""
    out = []
    name = None
    for line in asm.splitlines():
        m = re.match(r"\s*\.amdhsa_kernel\s+(\S+)", line)
        if m:
            name = m.group(1)
        m = re.match(r"\s*\.amdhsa_private_segment_fixed_size\s+(\d+)", line)
        if m and name is not None and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


def test_scratch_detector():
    asm = ("\t.amdhsa_kernel _Z1av\n\t\t.amdhsa_private_segment_fixed_size 0\n\t.end_amdhsa_kernel\n"
           "\t.amdhsa_kernel _Z1bv\n\t\t.amdhsa_private_segment_fixed_size 768\n\t.end_amdhsa_kernel\n")
    assert scratch_users(asm) == [("_Z1bv", 768)]


_ASM = {}


def _generated(src):
    if src not in _ASM:
        tmp = tempfile.mkdtemp(prefix="tcbf_isa_")
        try:
            out = os.path.join(tmp, src + ".s")
            cmd = [libbuild.HIPCC] + libbuild.FLAGS + ["--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            _ASM[src] = open(out).read()
        finally:
            shutil.rmtree(tmp, ignore_errors=True)
    return _ASM[src]


def _all_generated():
    with ThreadPoolExecutor(max_workers=4) as ex:
        return list(zip(SOURCES, ex.map(_generated, SOURCES)))


# kernels allowed to use scratch (see the module note): mangled-name fragments
KNOWN_SCRATCH = ("cgemm_f16_fast_kernelILi2ELi16E", "cgemm_f16_fast_kernelILi4E", "cgemm_f16_split_kernel")


@pytest.mark.skipif(not os.path.exists(libbuild.HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_no_kernel_uses_scratch():
    problems = []
    for src, asm in _all_generated():
        problems += ["%s: %s uses %d bytes of scratch" % (src, k, n) for k, n in scratch_users(asm)
                     if not any(f in k for f in KNOWN_SCRATCH)]
    assert not problems, "\n".join(problems)


@pytest.mark.skipif(not os.path.exists(libbuild.HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_no_store_data_hazard_in_generated_code():
    results = _all_generated()
    problems = []
    for src, asm in results:
        problems += ["%s: %s  ->  %s" % (src, a, b) for a, b in store_data_hazards(asm)]
    assert not problems, "\n".join(problems)
