"""CPU oracle for the batched complex beamforming product B[c] = W[c] X[c].

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the library never does.  It shares no
code with the GPU library.  The arithmetic lives in ``oracle.c`` (plain C,
FP64 / int64 loops over the definition); this module only marshals numpy
arrays into it.

Array conventions (numpy, C order):
  W  [batch, M, K]  complex (beams x receivers), or [M, K] when shared
  X  [batch, K, N]  complex (receivers x samples)
  B  [batch, M, N]  complex
FP16 inputs are widened to float64 with numpy before the call; that widening is
exact.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # build on first use if nothing is built
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_cgemm_f64.argtypes = [_i64, _i64, _i64, _i64, _int] + [_p] * 6
    lib.oracle_cgemm_f64_entries.argtypes = [_i64, _i64, _i64, _i64, _int] + [_p] * 4 + [_i64] + [_p] * 5
    lib.oracle_abs_dot_entries.argtypes = [_i64, _i64, _i64, _int] + [_p] * 4 + [_i64] + [_p] * 4
    lib.oracle_pack1bit.argtypes = [_i64, _i64, _i64, _p, _p]
    lib.oracle_unpack1bit.argtypes = [_i64, _i64, _i64, _p, _p]
    lib.oracle_cgemm_1bit_def.argtypes = [_i64, _i64, _i64, _i64, _int] + [_p] * 6
    lib.oracle_cgemm_1bit_popc.argtypes = [_i64, _i64, _i64, _i64, _i64, _int] + [_p] * 6
    lib.oracle_cgemm_1bit_popc_entries.argtypes = [_i64, _i64, _i64, _i64, _int] + [_p] * 4 + [_i64] + [_p] * 5
    lib.oracle_dot1bit_xor.argtypes = [_i64, _p, _p]
    lib.oracle_dot1bit_xor.restype = _i64
    lib.oracle_dot1bit_and.argtypes = [_i64, _p, _p]
    lib.oracle_dot1bit_and.restype = _i64
    lib.oracle_e4m3_decode.argtypes = [_i64, _p, _p]
    lib.oracle_quantize_e4m3_rows.argtypes = [_i64, _i64, _p, _p, _p, _p, _p]
    lib.oracle_quantize_e4m3_blocks.argtypes = [_i64, _i64, _p, _p, _p, _p, _p]
    lib.oracle_steering_weights.argtypes = [_i64, _i64, _i64, _p, _p, _p, ctypes.c_double, _p, _p]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = _int
    _lib = lib
    return lib


def num_threads():
    """Threads the oracle's parallel loops use."""
    return int(_load().oracle_num_threads())


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _split(z):
    z = np.asarray(z)
    if np.iscomplexobj(z):
        return _c(z.real, np.float64), _c(z.imag, np.float64)
    return _c(z, np.float64), np.zeros(z.shape, np.float64)


def _shapes(W, X):
    X = np.asarray(X)
    W = np.asarray(W)
    if X.ndim != 3:
        raise ValueError("X must be [batch, K, N]")
    batch, K, N = X.shape
    if W.ndim == 2:
        shared = 1
        M = W.shape[0]
        if W.shape[1] != K:
            raise ValueError("W/X K mismatch")
    elif W.ndim == 3:
        shared = 0
        if W.shape[0] != batch or W.shape[2] != K:
            raise ValueError("W/X shape mismatch")
        M = W.shape[1]
    else:
        raise ValueError("W must be [batch, M, K] or [M, K]")
    return batch, M, N, K, shared


# --------------------------------------------------------------------------
# floating-point mode
# --------------------------------------------------------------------------

def cgemm(W, X):
    """B[c] = W[c] X[c] in FP64 (complex128 result).  W, X: complex arrays
    (any float/complex dtype; converted exactly to float64)."""
    lib = _load()
    batch, M, N, K, shared = _shapes(W, X)
    wr, wi = _split(W)
    xr, xi = _split(X)
    br = np.empty((batch, M, N), np.float64)
    bi = np.empty((batch, M, N), np.float64)
    lib.oracle_cgemm_f64(batch, M, N, K, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                         _ptr(br), _ptr(bi))
    return br + 1j * bi


def cgemm_entries(W, X, cs, ms, ns):
    """Selected entries B[cs[s], ms[s], ns[s]] in FP64 (complex128 vector)."""
    lib = _load()
    batch, M, N, K, shared = _shapes(W, X)
    wr, wi = _split(W)
    xr, xi = _split(X)
    cs, ms, ns = (_c(v, np.int64) for v in (cs, ms, ns))
    _check_idx(cs, ms, ns, batch, M, N)
    cnt = cs.size
    o_r = np.empty(cnt, np.float64)
    o_i = np.empty(cnt, np.float64)
    lib.oracle_cgemm_f64_entries(batch, M, N, K, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                                 cnt, _ptr(cs), _ptr(ms), _ptr(ns), _ptr(o_r), _ptr(o_i))
    return o_r + 1j * o_i


def abs_dot_entries(W, X, cs, ms, ns):
    """sum_k |W[c,m,k]| |X[c,k,n]| for the selected entries (error-bound scale)."""
    lib = _load()
    batch, M, N, K, shared = _shapes(W, X)
    wr, wi = _split(W)
    xr, xi = _split(X)
    cs, ms, ns = (_c(v, np.int64) for v in (cs, ms, ns))
    _check_idx(cs, ms, ns, batch, M, N)
    out = np.empty(cs.size, np.float64)
    lib.oracle_abs_dot_entries(M, N, K, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                               cs.size, _ptr(cs), _ptr(ms), _ptr(ns), _ptr(out))
    return out


def _check_idx(cs, ms, ns, batch, M, N):
    if not (cs.shape == ms.shape == ns.shape):
        raise ValueError("index vectors differ in length")
    for v, hi in ((cs, batch), (ms, M), (ns, N)):
        if v.size and (v.min() < 0 or v.max() >= hi):
            raise ValueError("entry index out of range")


# --------------------------------------------------------------------------
# 1-bit mode
# --------------------------------------------------------------------------

def words_per_row(K):
    return (int(K) + 31) // 32


def pack1bit(vals, K=None):
    """Pack [..., K] real values to [..., ceil(K/32)] uint32 words: bit k%32 of
    word k//32 is 1 when the value's sign bit is clear (+1), else 0 (-1)."""
    v = np.asarray(vals)
    K = v.shape[-1] if K is None else K
    rows = int(np.prod(v.shape[:-1])) if v.ndim > 1 else 1
    flat = _c(v.reshape(rows, K), np.float64)
    kw = words_per_row(K)
    out = np.empty((rows, kw), np.uint32)
    _load().oracle_pack1bit(rows, K, kw, _ptr(flat), _ptr(out))
    return out.reshape(v.shape[:-1] + (kw,))


def unpack1bit(words, K):
    """[..., kw] uint32 -> [..., K] int8 of +1/-1 (Fig. 1 mapping, LSB first)."""
    w = _c(words, np.uint32)
    kw = w.shape[-1]
    if kw * 32 < K:
        raise ValueError("too few words for K")
    rows = int(np.prod(w.shape[:-1])) if w.ndim > 1 else 1
    out = np.empty((rows, K), np.int8)
    _load().oracle_unpack1bit(rows, K, kw, _ptr(w.reshape(rows, kw)), _ptr(out))
    return out.reshape(w.shape[:-1] + (K,))


def cgemm_1bit_def(Wr, Wi, Xr, Xi):
    """Definition form on +-1 int8 planes: W [batch,M,K] (or [M,K]), X [batch,K,N].
    Returns (Re, Im) int64 [batch, M, N]."""
    lib = _load()
    batch, M, N, K, shared = _shapes(Wr, Xr)
    wr, wi, xr, xi = (_c(a, np.int8) for a in (Wr, Wi, Xr, Xi))
    br = np.empty((batch, M, N), np.int64)
    bi = np.empty((batch, M, N), np.int64)
    lib.oracle_cgemm_1bit_def(batch, M, N, K, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                              _ptr(br), _ptr(bi))
    return br, bi


def _shapes_packed(Wr, Xr):
    Wr = np.asarray(Wr)
    Xr = np.asarray(Xr)
    if Xr.ndim != 3:
        raise ValueError("packed X must be [batch, N, kw]")
    batch, N, kw = Xr.shape
    if Wr.ndim == 2:
        shared, M = 1, Wr.shape[0]
        if Wr.shape[1] != kw:
            raise ValueError("packed W/X word count mismatch")
    elif Wr.ndim == 3:
        shared, M = 0, Wr.shape[1]
        if Wr.shape[0] != batch or Wr.shape[2] != kw:
            raise ValueError("packed W/X shape mismatch")
    else:
        raise ValueError("packed W must be [batch, M, kw] or [M, kw]")
    return batch, M, N, kw, shared


def cgemm_1bit_popc(Wr, Wi, Xr, Xi, K):
    """The paper's XOR/popcount form on packed words.  W planes [batch,M,kw]
    (or [M,kw]); X planes [batch,N,kw] (packed along K).  Returns int64 (Re, Im)."""
    lib = _load()
    batch, M, N, kw, shared = _shapes_packed(Wr, Xr)
    if not (0 < K <= 32 * kw):
        raise ValueError("K out of range for the word count")
    wr, wi, xr, xi = (_c(a, np.uint32) for a in (Wr, Wi, Xr, Xi))
    br = np.empty((batch, M, N), np.int64)
    bi = np.empty((batch, M, N), np.int64)
    lib.oracle_cgemm_1bit_popc(batch, M, N, K, kw, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                               _ptr(br), _ptr(bi))
    return br, bi


def cgemm_1bit_popc_entries(Wr, Wi, Xr, Xi, K, cs, ms, ns):
    lib = _load()
    batch, M, N, kw, shared = _shapes_packed(Wr, Xr)
    wr, wi, xr, xi = (_c(a, np.uint32) for a in (Wr, Wi, Xr, Xi))
    cs, ms, ns = (_c(v, np.int64) for v in (cs, ms, ns))
    _check_idx(cs, ms, ns, batch, M, N)
    o_r = np.empty(cs.size, np.int64)
    o_i = np.empty(cs.size, np.int64)
    lib.oracle_cgemm_1bit_popc_entries(M, N, K, kw, shared, _ptr(wr), _ptr(wi), _ptr(xr), _ptr(xi),
                                       cs.size, _ptr(cs), _ptr(ms), _ptr(ns), _ptr(o_r), _ptr(o_i))
    return o_r, o_i


def dot1bit_xor(a_words, b_words, L):
    a = _c(a_words, np.uint32)
    b = _c(b_words, np.uint32)
    return int(_load().oracle_dot1bit_xor(L, _ptr(a), _ptr(b)))


def dot1bit_and(a_words, b_words, L):
    a = _c(a_words, np.uint32)
    b = _c(b_words, np.uint32)
    return int(_load().oracle_dot1bit_and(L, _ptr(a), _ptr(b)))


# --------------------------------------------------------------------------
# FP8 (e4m3) mode
# --------------------------------------------------------------------------

def e4m3_decode(codes):
    """uint8 e4m3 codes -> exact float64 values (NaN for the NaN codes)."""
    c = _c(codes, np.uint8)
    out = np.empty(c.shape, np.float64)
    _load().oracle_e4m3_decode(c.size, _ptr(c), _ptr(out))
    return out


def quantize_e4m3_rows(re, im):
    """Per-row quantisation of [rows, cols] planes (values converted to fp32).
    Returns (q_re, q_im) uint8 codes and fp32 scales [rows]."""
    r = _c(re, np.float32)
    i = _c(im, np.float32)
    if r.shape != i.shape or r.ndim != 2:
        raise ValueError("re, im must be equal-shape [rows, cols]")
    rows, cols = r.shape
    qr = np.empty((rows, cols), np.uint8)
    qi = np.empty((rows, cols), np.uint8)
    sc = np.empty(rows, np.float32)
    _load().oracle_quantize_e4m3_rows(rows, cols, _ptr(r), _ptr(i), _ptr(qr), _ptr(qi), _ptr(sc))
    return qr, qi, sc


def quantize_e4m3_blocks(re, im):
    """Per-32-block quantisation of [rows, cols] planes (values converted to
    fp32).  Returns (q_re, q_im) uint8 codes and uint8 E8M0 scale codes
    [rows, ceil(cols / 32)] (scale 2^(code - 127))."""
    r = _c(re, np.float32)
    i = _c(im, np.float32)
    if r.shape != i.shape or r.ndim != 2:
        raise ValueError("re, im must be equal-shape [rows, cols]")
    rows, cols = r.shape
    qr = np.empty((rows, cols), np.uint8)
    qi = np.empty((rows, cols), np.uint8)
    codes = np.empty((rows, (cols + 31) // 32), np.uint8)
    _load().oracle_quantize_e4m3_blocks(rows, cols, _ptr(r), _ptr(i), _ptr(qr), _ptr(qi), _ptr(codes))
    return qr, qi, codes


def e8m0_decode(codes):
    """E8M0 scale codes -> float64 powers of two 2^(code - 127) (NaN for 255)."""
    c = np.asarray(codes, np.int64)
    out = np.ldexp(1.0, c - 127)
    return np.where(c == 255, np.nan, out)


# --------------------------------------------------------------------------
# steering weights (Sec. II delays, Eq. 3 weights)
# --------------------------------------------------------------------------

def steering_weights(positions, directions, freqs, wave_speed):
    """positions [K, 3] m, directions [M, 3] (direction cosines), freqs [batch] Hz
    -> complex128 weights [batch, M, K], w = exp(+2 pi i frac(f s / c))."""
    p = _c(positions, np.float64)
    d = _c(directions, np.float64)
    f = _c(np.atleast_1d(freqs), np.float64)
    if p.ndim != 2 or p.shape[1] != 3 or d.ndim != 2 or d.shape[1] != 3:
        raise ValueError("positions [K, 3] and directions [M, 3]")
    K, M, batch = p.shape[0], d.shape[0], f.size
    re = np.empty((batch, M, K), np.float64)
    im = np.empty((batch, M, K), np.float64)
    _load().oracle_steering_weights(batch, M, K, _ptr(p), _ptr(d), _ptr(f), float(wave_speed), _ptr(re), _ptr(im))
    return re + 1j * im
