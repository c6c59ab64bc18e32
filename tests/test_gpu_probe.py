"""Peak probe (tcbf_peak_probe): with unit operands every accumulator element
ends at a closed-form count, which shows that every instruction of every
round ran; the VALU kind is checked against its xor/popcount sum computed
here; the clock marks are ordered; random operands give finite, repeatable
results that differ from lane to lane."""
import os

import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2505_03269_amd as tcbf  # noqa: E402

# products added per accumulator element by one instruction (unit operands)
PER_INSTR = {tcbf.PROBE_F16: 16, tcbf.PROBE_I8: 32, tcbf.PROBE_F8: 64, tcbf.PROBE_F4: 64}
FLOPS = {tcbf.PROBE_F16: 2 * 32 * 32 * 16, tcbf.PROBE_I8: 2 * 32 * 32 * 32, tcbf.PROBE_F8: 2 * 32 * 32 * 64,
         tcbf.PROBE_F4: 2 * 32 * 32 * 64}


@pytest.mark.parametrize("kind", [tcbf.PROBE_F16, tcbf.PROBE_I8, tcbf.PROBE_F8, tcbf.PROBE_F4])
def test_matrix_probe_counts(kind):
    blocks, iters = 6, 301
    log("probe kind %d" % kind)
    ops, vals, marks = tcbf.peak_probe(kind, blocks, iters)
    torch.cuda.synchronize()
    v = vals.cpu().numpy()
    expect = 4 * PER_INSTR[kind] * iters          # four chains summed
    got = v.astype(np.int64) if kind == tcbf.PROBE_I8 else v.view(np.float32)
    assert np.all(got == expect), (kind, np.unique(got)[:5])
    assert ops == blocks * 4 * iters * 4 * FLOPS[kind]
    m = marks.cpu().numpy()
    assert np.all(m[:, 2] >= m[:, 0]) and np.all(m[:, 3] >= m[:, 1])


def test_valu_probe_popcounts():
    blocks, iters = 3, 200
    bits = tcbf.PROBE_UNIT_OPERAND[tcbf.PROBE_VALU_XOR_POPC]
    ops, vals, marks = tcbf.peak_probe(tcbf.PROBE_VALU_XOR_POPC, blocks, iters)
    torch.cuda.synchronize()
    v = vals.cpu().numpy().view(np.uint32).reshape(blocks, 256)
    t = np.arange(256, dtype=np.uint64)
    b = (np.arange(iters, dtype=np.uint64) * 0x9E3779B9) & 0xFFFFFFFF
    total = np.zeros(256, np.int64)
    for j in range(8):
        w = (bits ^ (0x01010101 * j)) ^ t                      # [256]
        x = (w[:, None] ^ b[None, :]).astype(np.uint32)        # [256, iters]
        total += np.unpackbits(x.view(np.uint8), axis=1).reshape(256, -1).sum(axis=1).astype(np.int64)
    assert np.array_equal(v, np.broadcast_to(total.astype(np.uint32), v.shape))
    assert ops == blocks * 4 * iters * 8 * 64 * 64


@pytest.mark.parametrize("kind", [tcbf.PROBE_F16, tcbf.PROBE_I8, tcbf.PROBE_F8, tcbf.PROBE_F4,
                                  tcbf.PROBE_VALU_XOR_POPC])
def test_random_operands_repeatable(kind):
    runs = []
    for _ in range(2):
        ops, vals, marks = tcbf.peak_probe(kind, 4, 50, operand_bits=1234, random=True)
        torch.cuda.synchronize()
        runs.append(vals.cpu().numpy().copy())
    assert np.array_equal(runs[0], runs[1])
    if kind in (tcbf.PROBE_F16, tcbf.PROBE_F8, tcbf.PROBE_F4):
        assert np.all(np.isfinite(runs[0].view(np.float32)))
    assert len(np.unique(runs[0])) > 64


def test_probe_rejects_small_sink():
    sink = torch.empty(100, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ValueError):
        tcbf.peak_probe(tcbf.PROBE_F16, 1, 1, sink=sink)


def test_library_on_the_device_matches_the_sources():
    """The library these GPU tests load was built from the sources beside it."""
    from paper_2505_03269_amd import build as libbuild
    assert os.path.exists(libbuild.SOURCES_ID) and \
        open(libbuild.SOURCES_ID).read().strip() == libbuild.sources_id(), "stale libtcbf.so: rebuild it"
