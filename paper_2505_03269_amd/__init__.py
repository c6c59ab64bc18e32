"""tcbf -- batched complex beamforming product B[c] = W[c] X[c] on MI355X.

Thin ctypes binding over the C ABI in ``include/tcbf.h`` (``libtcbf.so``).
This module only marshals arguments: every step of the computation runs in
the library's HIP kernels.  torch tensors are accepted for device memory and
streams; the current torch stream is passed to the library.

If the shared library is missing, importing works but every call raises
``TcbfError``; there is no fallback implementation.
"""
import ctypes
import os

__all__ = [
    "F16", "INT1", "F8_E4M3", "MXF8_E4M3", "BF16", "PLANAR", "INTERLEAVED", "BLOCKED", "SRC_I8", "SRC_F16", "SRC_F32",
    "TcbfError", "Plan", "block_weights", "blocked_shape", "f8_codes_shape", "pack1bit", "quantize_e4m3", "steering_weights", "group_execute", "group_execute_noalloc", "GroupCall", "peak_probe", "f8_kp", "mx_scale_pitch", "mx_scales_to_rows",
    "mx_scales_from_rows", "lib",
    "status_string", "EXPORTS", "GROUP_MAX", "GROUP_WORKSPACE_BYTES", "GROUP_SCRATCH_BYTES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcbf.so")

F16, INT1, F8_E4M3, MXF8_E4M3, BF16 = 0, 1, 2, 3, 4
PLANAR, INTERLEAVED, BLOCKED = 0, 1, 2
SRC_I8, SRC_F16, SRC_F32 = 0, 1, 2

# every symbol include/tcbf.h declares
EXPORTS = ("tcbf_plan", "tcbf_execute", "tcbf_block_weights", "tcbf_pack1bit", "tcbf_quantize_e4m3", "tcbf_steering_weights",
           "tcbf_peak_probe", "tcbf_group_execute", "tcbf_group_execute_noalloc", "tcbf_plan_query", "tcbf_plan_destroy", "tcbf_status_string",
           "tcbf_version")
GROUP_MAX = 32
GROUP_WORKSPACE_BYTES = 256
GROUP_SCRATCH_BYTES = 256
# peak-probe kinds, and the operand pattern of each whose products are all 1
PROBE_F16, PROBE_I8, PROBE_F8, PROBE_F4, PROBE_VALU_XOR_POPC = 0, 1, 2, 3, 4
PROBE_UNIT_OPERAND = {PROBE_F16: 0x3C00, PROBE_I8: 0x01010101, PROBE_F8: 0x38383838, PROBE_F4: 0x22222222,
                      PROBE_VALU_XOR_POPC: 0x5A5A5A5A}

_STATUS = {0: "TCBF_SUCCESS", 1: "TCBF_ERROR_INVALID_VALUE", 2: "TCBF_ERROR_NOT_SUPPORTED",
           3: "TCBF_ERROR_OUT_OF_MEMORY", 4: "TCBF_ERROR_DEVICE", 5: "TCBF_ERROR_INTERNAL"}


class TcbfError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s%s" % (_STATUS.get(status, "status %d" % status), (": " + what) if what else ""))


class PlanDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("M", ctypes.c_int64), ("N", ctypes.c_int64),
                ("K", ctypes.c_int64), ("dtype", ctypes.c_int32), ("a_layout", ctypes.c_int32),
                ("b_layout", ctypes.c_int32), ("c_layout", ctypes.c_int32),
                ("a_shared", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("b_k_contiguous", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("a_batch_stride", ctypes.c_int64)]


class GroupProblem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("batch", ctypes.c_int64), ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("a_shared", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("a_scale", ctypes.c_void_p), ("b_scale", ctypes.c_void_p),
                ("variant", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("variant", ctypes.c_int32),
                ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("workgroups", ctypes.c_int64),
                ("useful_ops", ctypes.c_double), ("algorithmic_bytes", ctypes.c_double),
                ("kernel_name", ctypes.c_char * 64)]


_lib = None


def lib():
    """Load libtcbf.so (raises TcbfError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TcbfError(4, "libtcbf.so not built (run python -m paper_2505_03269_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.tcbf_plan.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    L.tcbf_plan.restype = i32
    L.tcbf_execute.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.tcbf_execute.restype = i32
    L.tcbf_block_weights.argtypes = [vp, i32, i64, i64, i64, vp, vp]
    L.tcbf_block_weights.restype = i32
    L.tcbf_pack1bit.argtypes = [vp, i32, i32, i64, i64, i64, i32, vp, vp]
    L.tcbf_pack1bit.restype = i32
    L.tcbf_quantize_e4m3.argtypes = [vp, i32, i32, i64, i64, i64, i32, i32, i32, vp, vp, vp]
    L.tcbf_quantize_e4m3.restype = i32
    L.tcbf_steering_weights.argtypes = [vp, vp, vp, ctypes.c_double, i64, i64, i64, i32, i32, vp, vp]
    L.tcbf_steering_weights.restype = i32
    L.tcbf_peak_probe.argtypes = [i32, i64, i64, ctypes.c_uint32, i32, vp, i64, ctypes.POINTER(ctypes.c_double), vp]
    L.tcbf_peak_probe.restype = i32
    L.tcbf_group_execute.argtypes = [i32, i32, i32, ctypes.POINTER(GroupProblem), i32, vp, vp]
    L.tcbf_group_execute.restype = i32
    L.tcbf_group_execute_noalloc.argtypes = [i32, i32, i32, ctypes.POINTER(GroupProblem), i32, vp]
    L.tcbf_group_execute_noalloc.restype = i32
    L.tcbf_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.tcbf_plan_query.restype = i32
    L.tcbf_plan_destroy.argtypes = [vp]
    L.tcbf_plan_destroy.restype = i32
    L.tcbf_status_string.argtypes = [i32]
    L.tcbf_status_string.restype = ctypes.c_char_p
    L.tcbf_version.argtypes = []
    L.tcbf_version.restype = i32
    _lib = L
    return L


def f8_kp(K):
    """Row pitch (bytes) of the FP8 operand form: 32 * ceil(K / 32)."""
    return (int(K) + 31) // 32 * 32


def mx_scale_pitch(K):
    """Row pitch (bytes) of per-block E8M0 scales: the Kp / 32 block codes
    padded to a multiple of 16 (16 * ceil(Kp / 512))."""
    return (f8_kp(K) // 32 + 15) // 16 * 16


def mx_scales_to_rows(scales, K):
    """Per-block scale codes in the library's grouped layout [..., Ks/16, rows,
    16] -> [..., rows, Kp/32] (row-major blocks; works on numpy arrays and
    tensors)."""
    g = scales.shape[-3]
    rows = scales.shape[-2]
    lead = tuple(scales.shape[:-3])
    t = scales.swapaxes(-3, -2) if hasattr(scales, "swapaxes") else scales.transpose(-3, -2)
    return t.reshape(lead + (rows, 16 * g))[..., :f8_kp(K) // 32]


def mx_scales_from_rows(codes, K, pad=0):
    """Row-major per-block codes [..., rows, Kp/32] (numpy) -> the grouped
    layout [..., Ks/16, rows, 16], padding codes set to `pad`."""
    import numpy as np
    ks = mx_scale_pitch(K)
    rows = codes.shape[-2]
    lead = tuple(codes.shape[:-2])
    full = np.full(lead + (rows, ks), pad, np.uint8)
    full[..., :codes.shape[-1]] = codes
    return np.ascontiguousarray(full.reshape(lead + (rows, ks // 16, 16)).swapaxes(-3, -2))


def _scale_shape(dtype, nb, rows, K):
    """Scales of `rows` rows in an FP8 mode: fp32 [nb, rows] per row, or E8M0
    codes in groups of 16 blocks [nb, Ks/16, rows, 16] per block."""
    return (nb, rows) if dtype == F8_E4M3 else (nb, mx_scale_pitch(K) // 16, rows, 16)


def _is_f8(dtype):
    return dtype in (F8_E4M3, MXF8_E4M3)


def status_string(status):
    return lib().tcbf_status_string(status).decode()


def _check(status, what=""):
    if status != 0:
        raise TcbfError(status, what)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, name, batch_stride=0):
    """Device pointer of a contiguous tensor; with batch_stride > 0, of a
    tensor whose entries along dim 0 are contiguous and batch_stride
    elements apart (a view into a larger buffer)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if batch_stride:
        if t.dim() < 2 or not t[0].is_contiguous() or (t.shape[0] > 1 and t.stride(0) != batch_stride):
            raise ValueError("%s must have contiguous entries %d elements apart" % (name, batch_stride))
    elif not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A validated problem (tcbf_plan).  Shapes follow include/tcbf.h."""

    def __init__(self, batch, M, N, K, dtype=F16, a_layout=PLANAR, b_layout=PLANAR,
                 c_layout=PLANAR, a_shared=False, variant=0, device=0, b_k_contiguous=False, a_batch_stride=0):
        """b_k_contiguous: fp16 X receiver-contiguous ([batch, 2, N, K] planar,
        [batch, N, K, 2] interleaved).  a_batch_stride: elements of W's
        storage type between consecutive batch entries of W (0: packed); W is
        then passed as a view with that stride along dim 0."""
        d = PlanDesc(ctypes.sizeof(PlanDesc), int(device), int(batch), int(M), int(N), int(K),
                     int(dtype), int(a_layout), int(b_layout), int(c_layout), int(bool(a_shared)),
                     int(variant), int(bool(b_k_contiguous)), 0, int(a_batch_stride))
        h = ctypes.c_void_p()
        self._h = None
        _check(lib().tcbf_plan(ctypes.byref(d), ctypes.byref(h)), "tcbf_plan")
        self._h = h
        self.desc = d
        self.batch, self.M, self.N, self.K = int(batch), int(M), int(N), int(K)
        self.dtype, self.a_layout, self.b_layout, self.c_layout = dtype, a_layout, b_layout, c_layout
        self.a_shared = bool(a_shared)
        self.device = int(device)
        self.b_k_contiguous = bool(b_k_contiguous) and dtype in (F16, BF16)
        self.a_batch_stride = int(a_batch_stride)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.tcbf_plan_destroy(self._h)
            self._h = None

    def info(self):
        i = PlanInfo()
        i.struct_size = ctypes.sizeof(PlanInfo)
        _check(lib().tcbf_plan_query(self._h, ctypes.byref(i)), "tcbf_plan_query")
        return {"variant": i.variant, "tile_m": i.tile_m, "tile_n": i.tile_n, "tile_k": i.tile_k,
                "threads": i.threads, "workgroups": i.workgroups, "useful_ops": i.useful_ops,
                "algorithmic_bytes": i.algorithmic_bytes, "kernel_name": i.kernel_name.decode()}

    # -- expected tensor shapes (element type, shape) ------------------------
    def shape_a(self):
        nb = 1 if self.a_shared else self.batch
        if self.dtype == INT1:
            return (nb, 2, self.M, (self.K + 31) // 32)
        if _is_f8(self.dtype):
            return f8_codes_shape(nb, self.M, self.K, self.a_layout)
        if self.a_layout == BLOCKED:
            return blocked_shape(nb, self.M, self.K)
        return (nb, 2, self.M, self.K) if self.a_layout == PLANAR else (nb, self.M, self.K, 2)

    def shape_b(self):
        if self.dtype == INT1:
            return (self.batch, 2, self.N, (self.K + 31) // 32)
        if _is_f8(self.dtype):
            return f8_codes_shape(self.batch, self.N, self.K, self.b_layout)
        if self.b_k_contiguous:
            return (self.batch, 2, self.N, self.K) if self.b_layout == PLANAR else (self.batch, self.N, self.K, 2)
        return (self.batch, 2, self.K, self.N) if self.b_layout == PLANAR else (self.batch, self.K, self.N, 2)

    def shape_a_scale(self):
        """FP8 modes: W scales ([nb, M] fp32 per row; per block uint8 codes in
        groups of 16, [nb, Ks/16, M, 16])."""
        return _scale_shape(self.dtype, 1 if self.a_shared else self.batch, self.M, self.K)

    def shape_b_scale(self):
        return _scale_shape(self.dtype, self.batch, self.N, self.K)

    def shape_c(self):
        return (self.batch, 2, self.M, self.N) if self.c_layout == PLANAR else (self.batch, self.M, self.N, 2)

    def _dtypes(self):
        import torch
        if self.dtype == INT1:
            return torch.int32, torch.int32, torch.int32  # packed words viewed as int32
        if _is_f8(self.dtype):
            return torch.uint8, torch.uint8, torch.float32  # e4m3 codes
        if self.dtype == BF16:
            return torch.bfloat16, torch.bfloat16, torch.float32
        return torch.float16, torch.float16, torch.float32

    def empty_output(self):
        import torch
        return torch.empty(self.shape_c(), dtype=self._dtypes()[2], device="cuda:%d" % self.device)

    def execute(self, A, B, C, a_scale=None, b_scale=None, stream=None):
        """Enqueue C = A . B (W, X, output) on the current torch stream.

        FP8 modes also take the W and X scales (as quantize_e4m3 returns them).
        """
        import torch
        ta, tb, tc = self._dtypes()
        checks = [(A, ta, self.shape_a(), "A"), (B, tb, self.shape_b(), "B"), (C, tc, self.shape_c(), "C")]
        if _is_f8(self.dtype):
            if a_scale is None or b_scale is None:
                raise ValueError("FP8 plans need a_scale and b_scale")
            st = torch.float32 if self.dtype == F8_E4M3 else torch.uint8
            checks += [(a_scale, st, self.shape_a_scale(), "a_scale"), (b_scale, st, self.shape_b_scale(), "b_scale")]
        elif a_scale is not None or b_scale is not None:
            raise ValueError("scales are only taken by FP8 plans")
        for t, dt, shp, nm in checks:
            if t.dtype != dt and not (self.dtype == INT1 and t.dtype == torch.uint32 and nm != "C"):
                raise ValueError("%s must be %s, got %s" % (nm, dt, t.dtype))
            if tuple(t.shape) != tuple(shp):
                raise ValueError("%s must have shape %s, got %s" % (nm, shp, tuple(t.shape)))
        pa, pb, pc = _dev_ptr(A, "A", self.a_batch_stride), _dev_ptr(B, "B"), _dev_ptr(C, "C")
        psa = _dev_ptr(a_scale, "a_scale") if a_scale is not None else None
        psb = _dev_ptr(b_scale, "b_scale") if b_scale is not None else None
        _check(lib().tcbf_execute(self._h, pa, pb, pc, psa, psb, _stream_handle(stream)), "tcbf_execute")
        return C


def blocked_shape(batch, M, K):
    """Shape of fp16 weights in the receiver-blocked layout: [batch, 2, ceil(K/32), M, 32]."""
    return (int(batch), 2, (int(K) + 31) // 32, int(M), 32)


def block_weights(W, layout=PLANAR, out=None, stream=None):
    """Repack 16-bit weights (fp16 or bfloat16; planar [batch, 2, M, K] or
    interleaved [batch, M, K, 2]) into the receiver-blocked layout
    (tcbf_block_weights, which moves 16-bit values without reading them);
    returns (or fills) [batch, 2, ceil(K/32), M, 32] of W's dtype, zero past K."""
    import torch
    if W.dtype not in (torch.float16, torch.bfloat16) or W.dim() != 4:
        raise ValueError("W must be a 4-d float16 or bfloat16 tensor")
    if layout == PLANAR:
        if W.shape[1] != 2:
            raise ValueError("planar W needs a plane axis of 2")
        batch, M, K = W.shape[0], W.shape[2], W.shape[3]
    elif layout == INTERLEAVED:
        if W.shape[3] != 2:
            raise ValueError("interleaved W needs a trailing axis of 2")
        batch, M, K = W.shape[0], W.shape[1], W.shape[2]
    else:
        raise ValueError("source layout must be PLANAR or INTERLEAVED")
    shape = blocked_shape(batch, M, K)
    if out is None:
        out = torch.empty(shape, dtype=W.dtype, device=W.device)
    if tuple(out.shape) != shape or out.dtype != W.dtype:
        raise ValueError("out must be %s %s" % (W.dtype, shape))
    _check(lib().tcbf_block_weights(_dev_ptr(W, "W"), int(layout), int(batch), int(M), int(K),
                                    _dev_ptr(out, "out"), _stream_handle(stream)), "tcbf_block_weights")
    return out


def pack1bit(src, K=None, k_major=True, layout=PLANAR, out=None, stream=None):
    """Sign-pack a device tensor (int8 / float16 / float32).

    k_major=True : planar [batch, 2, rows, K] or interleaved [batch, rows, K, 2]
    k_major=False: planar [batch, 2, K, rows] or interleaved [batch, K, rows, 2]
    Returns (or fills) int32 words [batch, 2, rows, ceil(K/32)].
    """
    import torch
    types = {torch.int8: SRC_I8, torch.float16: SRC_F16, torch.float32: SRC_F32}
    if src.dtype not in types:
        raise ValueError("unsupported source dtype %s" % src.dtype)
    if src.dim() != 4:
        raise ValueError("source must be 4-d")
    if layout == PLANAR:
        if src.shape[1] != 2:
            raise ValueError("planar source needs a plane axis of 2")
        batch = src.shape[0]
        rows, kk = (src.shape[2], src.shape[3]) if k_major else (src.shape[3], src.shape[2])
    else:
        if src.shape[3] != 2:
            raise ValueError("interleaved source needs a trailing axis of 2")
        batch = src.shape[0]
        rows, kk = (src.shape[1], src.shape[2]) if k_major else (src.shape[2], src.shape[1])
    if K is not None and K != kk:
        raise ValueError("K does not match the source")
    kw = (kk + 31) // 32
    if out is None:
        out = torch.empty((batch, 2, rows, kw), dtype=torch.int32, device=src.device)
    if tuple(out.shape) != (batch, 2, rows, kw) or out.dtype not in (torch.int32, torch.uint32):
        raise ValueError("out must be int32 [batch, 2, rows, ceil(K/32)]")
    _check(lib().tcbf_pack1bit(_dev_ptr(src, "src"), types[src.dtype], int(layout), int(batch), int(rows),
                               int(kk), int(bool(k_major)), _dev_ptr(out, "out"), _stream_handle(stream)),
           "tcbf_pack1bit")
    return out


def _source_geometry(src, k_major, layout):
    if src.dim() != 4:
        raise ValueError("source must be 4-d")
    if layout == PLANAR:
        if src.shape[1] != 2:
            raise ValueError("planar source needs a plane axis of 2")
        rows, kk = (src.shape[2], src.shape[3]) if k_major else (src.shape[3], src.shape[2])
    else:
        if src.shape[3] != 2:
            raise ValueError("interleaved source needs a trailing axis of 2")
        rows, kk = (src.shape[1], src.shape[2]) if k_major else (src.shape[2], src.shape[1])
    return src.shape[0], rows, kk


def f8_codes_shape(batch, rows, K, out_layout=PLANAR):
    """Shape of e4m3 codes: planar [batch, 2, rows, Kp] or receiver-blocked
    [batch, 2, ceil(Kp/64), rows, 64], Kp = 32 * ceil(K/32)."""
    kp = f8_kp(K)
    if out_layout == BLOCKED:
        return (int(batch), 2, (kp + 63) // 64, int(rows), 64)
    return (int(batch), 2, int(rows), kp)


def quantize_e4m3(src, k_major=True, layout=PLANAR, block=0, out=None, scales=None, stream=None,
                  out_layout=PLANAR):
    """Quantise a device tensor (int8 / float16 / float32) to the FP8 operand form.

    Source orientation as for pack1bit.  Returns (codes, scales): uint8 codes
    (f8_codes_shape: [batch, 2, rows, Kp], or receiver-blocked
    [batch, 2, ceil(Kp/64), rows, 64] with out_layout=BLOCKED) and fp32 scales
    [batch, rows] (block=0) or uint8 E8M0
    codes in groups of 16 blocks [batch, Ks/16, rows, 16] (block=32; Ks =
    mx_scale_pitch(K); block j of row r at [j // 16, r, j % 16]; codes past
    Kp/32 not written).  mx_scales_to_rows turns them into [batch, rows, Kp/32].
    """
    import torch
    types = {torch.int8: SRC_I8, torch.float16: SRC_F16, torch.float32: SRC_F32}
    if src.dtype not in types:
        raise ValueError("unsupported source dtype %s" % src.dtype)
    batch, rows, kk = _source_geometry(src, k_major, layout)
    if out_layout not in (PLANAR, BLOCKED):
        raise ValueError("out_layout must be PLANAR or BLOCKED")
    cshape = f8_codes_shape(batch, rows, kk, out_layout)
    if out is None:
        out = torch.empty(cshape, dtype=torch.uint8, device=src.device)
    if scales is None:
        if block == 0:
            scales = torch.empty((batch, rows), dtype=torch.float32, device=src.device)
        else:
            scales = torch.empty((batch, mx_scale_pitch(kk) // 16, rows, 16), dtype=torch.uint8, device=src.device)
    if tuple(out.shape) != cshape or out.dtype != torch.uint8:
        raise ValueError("out must be uint8 %s" % (cshape,))
    want = (((batch, rows), torch.float32) if block == 0
            else ((batch, mx_scale_pitch(kk) // 16, rows, 16), torch.uint8))
    if tuple(scales.shape) != want[0] or scales.dtype != want[1]:
        raise ValueError("scales must be %s %s" % (want[1], want[0]))
    _check(lib().tcbf_quantize_e4m3(_dev_ptr(src, "src"), types[src.dtype], int(layout), int(batch), int(rows),
                                    int(kk), int(bool(k_major)), int(block), int(out_layout), _dev_ptr(out, "out"),
                                    _dev_ptr(scales, "scales"), _stream_handle(stream)),
           "tcbf_quantize_e4m3")
    return out, scales


def steering_weights(positions, directions, frequencies, wave_speed, dtype=None, out=None, stream=None,
                     out_layout=PLANAR):
    """Steering weights on the device: positions [K, 3], directions [M, 3],
    frequencies [batch] (float64 device tensors) -> planar [batch, 2, M, K]
    float16 (default) or float32 weights, w = exp(+2 pi i frac(f s / c));
    out_layout=BLOCKED: float16 in the receiver-blocked layout (blocked_shape)."""
    import torch
    dtype = torch.float16 if dtype is None else dtype
    types = {torch.float16: SRC_F16, torch.float32: SRC_F32}
    if dtype not in types:
        raise ValueError("dtype must be float16 or float32")
    for t, nm in ((positions, "positions"), (directions, "directions"), (frequencies, "frequencies")):
        if t.dtype != torch.float64:
            raise ValueError("%s must be float64" % nm)
    if positions.dim() != 2 or positions.shape[1] != 3 or directions.dim() != 2 or directions.shape[1] != 3:
        raise ValueError("positions [K, 3] and directions [M, 3]")
    K, M, batch = positions.shape[0], directions.shape[0], frequencies.numel()
    if out_layout not in (PLANAR, BLOCKED) or (out_layout == BLOCKED and dtype != torch.float16):
        raise ValueError("out_layout must be PLANAR, or BLOCKED with float16 weights")
    shape = blocked_shape(batch, M, K) if out_layout == BLOCKED else (batch, 2, M, K)
    if out is None:
        out = torch.empty(shape, dtype=dtype, device=positions.device)
    if tuple(out.shape) != tuple(shape) or out.dtype != dtype:
        raise ValueError("out must be %s %s" % (dtype, tuple(shape)))
    _check(lib().tcbf_steering_weights(_dev_ptr(positions, "positions"), _dev_ptr(directions, "directions"),
                                       _dev_ptr(frequencies, "frequencies"), float(wave_speed), int(batch), int(M),
                                       int(K), types[dtype], int(out_layout), _dev_ptr(out, "out"),
                                       _stream_handle(stream)),
           "tcbf_steering_weights")
    return out


def peak_probe(kind, blocks, iterations, operand_bits=None, random=False, sink=None, stream=None):
    """Enqueue one peak-probe launch (measurement tool).  `random`: pseudo-random
    operands alternating every instruction (seeded by operand_bits) instead of
    uniform ones.  Returns (ops, values,
    marks): the launch's useful operations, the uint32 [blocks * 256]
    per-thread results and the uint64 [blocks, 4] clock marks (shader-clock
    counter and 100 MHz counter before and after each workgroup's loop).
    The caller times the launch on the stream."""
    import torch
    if kind not in PROBE_UNIT_OPERAND:
        raise ValueError("unknown probe kind %r" % (kind,))
    bits = PROBE_UNIT_OPERAND[kind] if operand_bits is None else int(operand_bits)
    nbytes = int(blocks) * 256 * 4 + int(blocks) * 32
    if sink is None:
        sink = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    if sink.dtype != torch.uint8 or sink.numel() < nbytes:
        raise ValueError("sink must be uint8 with at least %d bytes" % nbytes)
    ops = ctypes.c_double(0.0)
    _check(lib().tcbf_peak_probe(int(kind), int(blocks), int(iterations), bits & 0xFFFFFFFF, int(bool(random)),
                                 _dev_ptr(sink, "sink"), int(sink.numel()), ctypes.byref(ops), _stream_handle(stream)),
           "tcbf_peak_probe")
    values = sink[:int(blocks) * 256 * 4].view(torch.int32)
    marks = sink[int(blocks) * 256 * 4:nbytes].view(torch.int64).view(int(blocks), 4)
    return ops.value, values, marks


def group_execute(problems, c_layout=PLANAR, workspace=None, device=0, stream=None, dtype=F16, layout=PLANAR,
                  variants=None):
    """One grouped persistent launch over up to GROUP_MAX problems of one dtype.

    dtype F16: problems are (W, X, C) or (W, X, C, a_shared) device tensors
    with W float16 [batch|1, 2, M, K] (layout=BLOCKED: blocked_shape(batch|1,
    M, K), from block_weights), X float16 [batch, 2, K, N].
    dtype F8_E4M3 / MXF8_E4M3: (W, X, C, a_scale, b_scale) or
    (W, X, C, a_scale, b_scale, a_shared) with e4m3 codes W uint8
    [batch|1, 2, M, Kp], X uint8 [batch, 2, N, Kp] and the scales of that
    mode (see Plan.shape_a_scale / shape_b_scale); layout=BLOCKED: blocked
    codes (f8_codes_shape) and the true K after the scales,
    (W, X, C, a_scale, b_scale, K[, a_shared]).
    dtype INT1: (W, X, C, K) or (W, X, C, K, a_shared) with packed sign words
    W int32 [batch|1, 2, M, kw], X int32 [batch, 2, N, kw] and the true K.
    C: float32 (int32 for INT1) [batch, 2, M, N] (planar) or [batch, M, N, 2]
    (interleaved).
    workspace: uint8 device tensor of GROUP_WORKSPACE_BYTES (allocated here
    if None; pass one to stay allocation-free).
    variants: fp16 only, one kernel variant per problem (0 = the plan's
    default; e.g. the autotuner's choice, tune.tune_group); problems with
    256-beam-tile variants (6, 7, 9) run in a grouped ping-pong launch, the
    rest in the grouped 128 x 128 launch.
    """
    import torch
    arr = _group_table(problems, c_layout, dtype, layout, variants)
    if workspace is None:
        workspace = torch.empty(GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:%d" % device)
    if workspace.numel() * workspace.element_size() < GROUP_WORKSPACE_BYTES:
        raise ValueError("workspace too small")
    _check(lib().tcbf_group_execute(int(device), int(dtype), int(c_layout), arr, len(problems),
                                    _dev_ptr(workspace, "workspace"), _stream_handle(stream)),
           "tcbf_group_execute")
    return [pr[2] for pr in problems]


class GroupCall:
    """A grouped launch prepared once and issued many times: the problem
    tuples are checked and the C problem table built at construction (the
    same arguments as group_execute), so each call only passes the table, the
    workspace and the stream to tcbf_group_execute.  For a serving or
    streaming loop that runs the same buffers again and again; the tensors
    are kept alive by the object."""

    def __init__(self, problems, c_layout=PLANAR, workspace=None, device=0, dtype=F16, layout=PLANAR,
                 variants=None):
        import torch
        self._arr = _group_table(problems, c_layout, dtype, layout, variants)
        if workspace is None:
            workspace = torch.empty(GROUP_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda:%d" % device)
        if workspace.numel() * workspace.element_size() < GROUP_WORKSPACE_BYTES:
            raise ValueError("workspace too small")
        self._ws = workspace
        self._ws_ptr = _dev_ptr(workspace, "workspace")
        self._problems = list(problems)
        self._args = (int(device), int(dtype), int(c_layout))
        self._fn = lib().tcbf_group_execute

    def __call__(self, stream=None):
        d, t, c = self._args
        _check(self._fn(d, t, c, self._arr, len(self._problems), self._ws_ptr, _stream_handle(stream)),
               "tcbf_group_execute")
        return [pr[2] for pr in self._problems]


def group_execute_noalloc(problems, c_layout=PLANAR, device=0, stream=None, dtype=F16, layout=PLANAR,
                          variants=None):
    """The grouped launch of group_execute (same problem tuples and results)
    through the allocation-free entry point: its tile counter lives in the
    library's per-GPU scratch array, so launches of this call that overlap in
    time on one GPU race (use group_execute with one workspace per stream)."""
    arr = _group_table(problems, c_layout, dtype, layout, variants)
    _check(lib().tcbf_group_execute_noalloc(int(device), int(dtype), int(c_layout), arr, len(problems),
                                            _stream_handle(stream)),
           "tcbf_group_execute_noalloc")
    return [pr[2] for pr in problems]


def _group_table(problems, c_layout, dtype, layout, variants=None):
    """Check the problem tuples of a grouped launch and build its C table."""
    import torch
    if variants is not None and len(variants) != len(problems):
        raise ValueError("one variant per problem")
    if not 1 <= len(problems) <= GROUP_MAX:
        raise ValueError("1..%d problems per launch" % GROUP_MAX)
    f8 = _is_f8(dtype)
    if dtype not in (F16, INT1) and not f8:
        raise ValueError("grouped launches take F16, F8_E4M3, MXF8_E4M3 or INT1")
    if layout not in (PLANAR, BLOCKED) or (layout == BLOCKED and dtype == INT1):
        raise ValueError("layout must be PLANAR, or BLOCKED for fp16 and FP8")
    blocked = layout == BLOCKED
    arr = (GroupProblem * len(problems))()
    for i, pr in enumerate(problems):
        W, X, C = pr[0], pr[1], pr[2]
        # fields before the optional a_shared
        nfix = (6 if blocked else 5) if f8 else 4 if dtype == INT1 else 3
        shared = bool(pr[nfix]) if len(pr) > nfix else False
        nb = lambda b: 1 if shared else b  # noqa: E731
        elem = torch.uint8 if f8 else torch.int32 if dtype == INT1 else torch.float16
        cdt = torch.int32 if dtype == INT1 else torch.float32
        if W.dtype != elem or X.dtype != elem or C.dtype != cdt:
            raise ValueError("problem %d: W, X %s and C %s expected" % (i, elem, cdt))
        if W.dim() not in (4, 5) or X.dim() not in (4, 5) or W.shape[1] != 2 or X.shape[1] != 2:
            raise ValueError("problem %d: W [b, 2, ...] and X [b, 2, ...] expected" % i)
        if dtype == INT1:
            if len(pr) < 4:
                raise ValueError("problem %d: 1-bit problems are (W, X, C, K[, a_shared])" % i)
            batch, N, kw = X.shape[0], X.shape[2], X.shape[3]
            K = int(pr[3])
            if not 0 < K <= 32 * kw or (K + 31) // 32 != kw:
                raise ValueError("problem %d: K does not match the word count" % i)
            M = W.shape[2]
            want_w = (nb(batch), 2, M, kw)
        elif f8 and blocked:
            if len(pr) < 6:
                raise ValueError("problem %d: blocked FP8 problems are (W, X, C, a_scale, b_scale, K[, a_shared])" % i)
            K = int(pr[5])
            batch, N, M = X.shape[0], X.shape[3], W.shape[3]
            if tuple(X.shape) != f8_codes_shape(batch, N, K, BLOCKED):
                raise ValueError("problem %d: X must be %s" % (i, f8_codes_shape(batch, N, K, BLOCKED)))
            want_w = f8_codes_shape(nb(batch), M, K, BLOCKED)
        elif f8:
            batch, N, K = X.shape[0], X.shape[2], X.shape[3]
            if K % 32:
                raise ValueError("problem %d: FP8 rows must be Kp = 32 * ceil(K / 32) bytes" % i)
            M = W.shape[2]
            want_w = (nb(batch), 2, M, K)
        else:
            batch, K, N = X.shape[0], X.shape[2], X.shape[3]
            M = W.shape[3] if blocked else W.shape[2]
            want_w = blocked_shape(nb(batch), M, K) if blocked else (nb(batch), 2, M, K)
        if tuple(W.shape) != tuple(want_w):
            raise ValueError("problem %d: W must have shape %s to match X" % (i, tuple(want_w)))
        want = (batch, 2, M, N) if c_layout == PLANAR else (batch, M, N, 2)
        if tuple(C.shape) != want:
            raise ValueError("problem %d: C must have shape %s" % (i, want))
        sa = sb = None
        if f8:
            st = torch.float32 if dtype == F8_E4M3 else torch.uint8
            for t, shape, nm in ((pr[3], _scale_shape(dtype, nb(batch), M, K), "a_scale"),
                                 (pr[4], _scale_shape(dtype, batch, N, K), "b_scale")):
                if t.dtype != st or tuple(t.shape) != tuple(shape):
                    raise ValueError("problem %d: %s must be %s %s" % (i, nm, st, tuple(shape)))
            sa, sb = _dev_ptr(pr[3], "a_scale").value, _dev_ptr(pr[4], "b_scale").value
        arr[i] = GroupProblem(_dev_ptr(W, "W").value, _dev_ptr(X, "X").value, _dev_ptr(C, "C").value,
                              batch, M, N, K, int(shared), int(layout), sa, sb,
                              0 if variants is None else int(variants[i]), 0)
    return arr
