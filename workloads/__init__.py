"""Seeded synthetic inputs for the beamforming product B[c] = W[c] X[c].

This module only draws inputs; it holds none of the method's arithmetic.  The
GPU tests, the benchmark and the CPU oracle all take their inputs from here, so
both sides see identical data.

Every array is generated on the host with numpy from
``SeedSequence([cfg_id, tensor_id, channel])`` (tensor_id 0 = W, 1 = X), so any
channel can be regenerated alone.  Layouts returned here are the library's
planar layouts:

  W planar [2, M, K] per channel (re plane, im plane; K contiguous), fp16
  X planar [2, K, N] per channel (N contiguous), fp16
  1-bit:   W words [2, M, ceil(K/32)], X words [2, N, ceil(K/32)], uint32

Workload recipes (synthetic stand-ins; no instrument data is used):
  C1  plain FP16: 4 ch, M=128, K=64, N=512; W unit phasors, phase U[0, 2pi)
      in FP64 rounded to fp16; X complex Gaussian sigma=32 per component,
      rounded half-even and clipped to [-127, 127] (8-bit range), stored fp16.
  C2  radio-astronomy FP16: 256 ch, M=1024 beams, K=576 receivers, N=4096
      samples.  Antenna (x, y) uniform in a 1000 m disk, beam direction cosines
      (l, m) uniform in a disk of radius 0.05; channel c at
      f_c = 150 MHz + (c - 127.5) * 195312.5 Hz; phase
      phi = 2 pi frac(f_c (x l + y m) / c0) in FP64; w = exp(+i phi) rounded to
      fp16.  X as in C1.
  C3  1-bit: 64 ch, M=2048, K=8192, N=8192; every sign bit i.i.d. Bernoulli(1/2)
      drawn directly as uint32 words (pad bits past K cleared).
  C4  ultrasound FP16: 1 ch, M=32768 voxels, K=8192, N=256 frames; W re, im
      ~ N(0, 1) (Rayleigh(1) magnitude, uniform phase) rounded to fp16; X re,
      im ~ N(0, 512^2) rounded and clipped to [-2048, 2047] (12-bit range).
  C5  served mixed stream: job shapes M ~ U[128, 4096], K ~ U[64, 2048],
      N ~ U[256, 8192] (integers; rounded up to multiples of 8 where a kernel
      needs it), see mixed_shapes().
"""
import numpy as np

C0 = 299792458.0  # speed of light, m/s

# The workloads by name; seed_id is the first component of every seed drawn
# for that workload (see rng).
WORKLOADS = {
    "plain-fp16-4ch": dict(seed_id=1, batch=4, M=128, K=64, N=512, dtype="f16"),
    "radio-astro-fp16": dict(seed_id=2, batch=256, M=1024, K=576, N=4096, dtype="f16"),
    "one-bit": dict(seed_id=3, batch=64, M=2048, K=8192, N=8192, dtype="int1"),
    "ultrasound-fp16": dict(seed_id=4, batch=1, M=32768, K=8192, N=256, dtype="f16"),
}


def rng(cfg_id, tensor_id, channel=0):
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(tensor_id), int(channel)]))


def _to_f16_planes(re, im):
    out = np.empty((2,) + re.shape, np.float16)
    out[0] = re
    out[1] = im
    return out


def quantised_gaussian(g, shape, sigma, lo, hi):
    """Complex Gaussian, each component rounded half-even and clipped."""
    re = np.clip(np.rint(g.normal(0.0, sigma, shape)), lo, hi)
    im = np.clip(np.rint(g.normal(0.0, sigma, shape)), lo, hi)
    return _to_f16_planes(re, im)


def unit_phasors(g, shape):
    phi = g.uniform(0.0, 2.0 * np.pi, shape)
    return _to_f16_planes(np.cos(phi), np.sin(phi))


# ---- C1 -------------------------------------------------------------------

def c1_channel(c, M=128, K=64, N=512, cfg_id=1):
    W = unit_phasors(rng(cfg_id, 0, c), (M, K))
    X = quantised_gaussian(rng(cfg_id, 1, c), (K, N), 32.0, -127, 127)
    return W, X


# ---- C2 -------------------------------------------------------------------

def c2_geometry(K=576, M=1024, cfg_id=2):
    """Antenna positions (m) and beam direction cosines, fixed for all channels."""
    g = rng(cfg_id, 2, 0)
    r = 1000.0 * np.sqrt(g.uniform(0.0, 1.0, K))
    t = g.uniform(0.0, 2.0 * np.pi, K)
    ax, ay = r * np.cos(t), r * np.sin(t)
    rb = 0.05 * np.sqrt(g.uniform(0.0, 1.0, M))
    tb = g.uniform(0.0, 2.0 * np.pi, M)
    bl, bm = rb * np.cos(tb), rb * np.sin(tb)
    return ax, ay, bl, bm


def c2_frequency(c, nchan=256):
    return 150.0e6 + (c - (nchan - 1) / 2.0) * 195312.5


def c2_weights(c, geometry, nchan=256):
    ax, ay, bl, bm = geometry
    f = c2_frequency(c, nchan)
    cycles = f * (np.outer(bl, ax) + np.outer(bm, ay)) / C0  # [M, K], FP64
    phi = 2.0 * np.pi * (cycles - np.floor(cycles))
    return _to_f16_planes(np.cos(phi), np.sin(phi))


def c2_channel(c, geometry=None, M=1024, K=576, N=4096, nchan=256, cfg_id=2):
    if geometry is None:
        geometry = c2_geometry(K, M, cfg_id)
    W = c2_weights(c, geometry, nchan)
    X = quantised_gaussian(rng(cfg_id, 1, c), (K, N), 32.0, -127, 127)
    return W, X


# ---- C3 -------------------------------------------------------------------

def random_words(g, rows, K):
    kw = (K + 31) // 32
    w = g.integers(0, 2**32, size=(2, rows, kw), dtype=np.uint64).astype(np.uint32)
    tail = K - 32 * (kw - 1)
    if tail < 32:
        w[..., -1] &= np.uint32((1 << tail) - 1)
    return w


def c3_channel(c, M=2048, K=8192, N=8192, cfg_id=3):
    Wp = random_words(rng(cfg_id, 0, c), M, K)
    Xp = random_words(rng(cfg_id, 1, c), N, K)
    return Wp, Xp


# ---- C4 -------------------------------------------------------------------

def c4_channel(c=0, M=32768, K=8192, N=256, cfg_id=4):
    g = rng(cfg_id, 0, c)
    W = _to_f16_planes(g.normal(0.0, 1.0, (M, K)), g.normal(0.0, 1.0, (M, K)))
    X = quantised_gaussian(rng(cfg_id, 1, c), (K, N), 512.0, -2048, 2047)
    return W, X


# ---- generic cases for tests -------------------------------------------------

def random_f16_case(seed, batch, M, N, K, shared_w=False, scale_w=1.0, scale_x=32.0):
    """Generic planar fp16 case: W [batch|1, 2, M, K], X [batch, 2, K, N]."""
    g = np.random.default_rng(np.random.SeedSequence([1000, int(seed), batch, M, N, K]))
    nw = 1 if shared_w else batch
    W = np.empty((nw, 2, M, K), np.float16)
    X = np.empty((batch, 2, K, N), np.float16)
    W[...] = g.normal(0.0, scale_w, W.shape)
    X[...] = np.clip(np.rint(g.normal(0.0, scale_x, X.shape)), -127, 127)
    return W, X


def random_bits_case(seed, batch, M, N, K, shared_w=False):
    g = np.random.default_rng(np.random.SeedSequence([2000, int(seed), batch, M, N, K]))
    nw = 1 if shared_w else batch
    Wp = np.stack([random_words(g, M, K) for _ in range(nw)])
    Xp = np.stack([random_words(g, N, K) for _ in range(batch)])
    return Wp, Xp


def planar_to_complex(P):
    """[..., 2, r, c] planar (any float dtype) -> complex128 [..., r, c]."""
    P = np.asarray(P)
    return P[..., 0, :, :].astype(np.float64) + 1j * P[..., 1, :, :].astype(np.float64)


# ---- whole configurations ------------------------------------------------------

def _parallel(fn, n, threads):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(fn, range(n)))


def generate_c2(batch=256, threads=8):
    """Radio-astronomy inputs: W [batch, 2, 1024, 576], X [batch, 2, 576, 4096] fp16."""
    cfg = WORKLOADS["radio-astro-fp16"]
    M, K, N = cfg["M"], cfg["K"], cfg["N"]
    geo = c2_geometry(K, M)
    W = np.empty((batch, 2, M, K), np.float16)
    X = np.empty((batch, 2, K, N), np.float16)

    def one(c):
        W[c], X[c] = c2_channel(c, geo, M, K, N)
    _parallel(one, batch, threads)
    return W, X


def generate_c3(batch=64, threads=8):
    """One-bit inputs: packed W [batch, 2, 2048, 256], X [batch, 2, 8192, 256]."""
    cfg = WORKLOADS["one-bit"]
    M, K, N = cfg["M"], cfg["K"], cfg["N"]
    kw = (K + 31) // 32
    W = np.empty((batch, 2, M, kw), np.uint32)
    X = np.empty((batch, 2, N, kw), np.uint32)

    def one(c):
        W[c], X[c] = c3_channel(c, M, K, N)
    _parallel(one, batch, threads)
    return W, X


# ---- C5 shapes -------------------------------------------------------------

def mixed_shapes(seed, count, align=8, m_range=(128, 4096), n_range=(256, 8192), k_range=(64, 2048)):
    """`count` job shapes (M, N, K) drawn uniformly from the given ranges
    (default: the served-stream distribution), each rounded up to a multiple
    of `align`."""
    g = rng(5, 3, seed)
    up = lambda v: int(-(-int(v) // align) * align)  # noqa: E731
    M = g.integers(m_range[0], m_range[1] + 1, count)
    K = g.integers(k_range[0], k_range[1] + 1, count)
    N = g.integers(n_range[0], n_range[1] + 1, count)
    return [(up(m), up(n), up(k)) for m, n, k in zip(M, N, K)]
