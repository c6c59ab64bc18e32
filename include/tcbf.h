/*
 * tcbf.h -- batched complex beamforming product on AMD MI355X (gfx950).
 *
 * The library computes, for every channel (or frame) c of a batch,
 *
 *     B[c] = W[c] . X[c]          W: M x K,  X: K x N,  B: M x N, all complex
 *
 * i.e. Eq. (3) of the Tensor-Core Beamformer paper (each beam output is the
 * weighted sum of the K receiver signals) evaluated for N samples at once,
 * which Sec. II maps to a matrix product with M = beams, N = samples and
 * K = receivers.  There is no conjugation.  The input precisions are those of
 * Sec. III, 16-bit float and 1-bit (sign only, Sec. III-D), plus 8-bit float
 * (OCP FP8 e4m3), which Sec. VI names as a future option, with per-row or
 * per-32-receiver-block scales.
 *
 * Every entry point is a plain C function over plain pointers and sizes.
 * Device pointers are HIP device (or managed) allocations; `stream` is a
 * hipStream_t passed as void* (NULL = the default stream).  No entry point
 * throws, aborts or allocates device memory in the execution calls.
 *
 * Ownership: the caller owns every buffer.  The library never frees, retains
 * or caches a user pointer after a call returns.  A plan owns only host
 * memory and is released with tcbf_plan_destroy.
 *
 * Errors: invalid sizes, NULL or misaligned pointers and unsupported
 * combinations are rejected synchronously, before anything is enqueued, with
 * TCBF_ERROR_INVALID_VALUE or TCBF_ERROR_NOT_SUPPORTED.  A failed launch returns
 * TCBF_ERROR_DEVICE.  Faults while a kernel runs surface at the caller's next
 * synchronisation with the stream, as with any HIP launch.
 */
#ifndef TCBF_H
#define TCBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TCBF_VERSION 4

typedef enum tcbf_status {
    TCBF_SUCCESS = 0,
    TCBF_ERROR_INVALID_VALUE = 1, /* bad size, pointer, alignment or enum value  */
    TCBF_ERROR_NOT_SUPPORTED = 2, /* valid request the library/device cannot run */
    TCBF_ERROR_OUT_OF_MEMORY = 3, /* host allocation for a plan failed           */
    TCBF_ERROR_DEVICE = 4,        /* HIP runtime error (no device, launch failed) */
    TCBF_ERROR_INTERNAL = 5
} tcbf_status;

/* Input precision of W and X (Sec. III: 16-bit float and 1-bit; Sec. VI: 8-bit float). */
typedef enum tcbf_dtype {
    TCBF_F16 = 0,       /* fp16 in, fp32 accumulate, fp32 complex out            */
    TCBF_INT1 = 1,      /* packed sign bits in, exact int32 complex out          */
    TCBF_F8_E4M3 = 2,   /* e4m3 in with one fp32 scale per row, fp32 out         */
    TCBF_MXF8_E4M3 = 3, /* e4m3 in with an E8M0 scale per 32-receiver block       */
    TCBF_BF16 = 4       /* bfloat16 in, fp32 accumulate, fp32 complex out; the
                           fp16 layouts (blocked W included), variants 1, 2 and
                           9 (9 with planar X), not in grouped launches          */
} tcbf_dtype;

/* Complex storage.  PLANAR keeps a real plane then an imaginary plane for each
 * batch entry; INTERLEAVED stores (re, im) pairs (the "usual interleaved
 * format" of Sec. VI).  BLOCKED is a planar weight layout tiled along the
 * receivers (Sec. III: the product kernel takes its inputs tiled in device
 * memory, prepared by a separate transpose kernel; Sec. V-A: for the model
 * matrix this is done once, before the data stream); see TCBF_F16 below and
 * tcbf_block_weights. */
typedef enum tcbf_layout {
    TCBF_PLANAR = 0,
    TCBF_INTERLEAVED = 1,
    TCBF_BLOCKED = 2
} tcbf_layout;

/* Element type of a source array for tcbf_pack1bit. */
typedef enum tcbf_src_type {
    TCBF_SRC_I8 = 0,
    TCBF_SRC_F16 = 1,
    TCBF_SRC_F32 = 2
} tcbf_src_type;

/*
 * Problem description.  Sizes are element counts (complex elements).
 *
 * TCBF_F16 buffer layouts (fp16 = IEEE binary16, fp32 = IEEE binary32):
 *   A = W   planar      [batch][2][M][K]   K contiguous
 *           interleaved [batch][M][K][2]
 *           blocked     [batch][2][Kb][M][32], Kb = ceil(K/32): receiver k of
 *                       beam m in block k/32, position k%32 (each block holds
 *                       all M beams x 32 receivers, 64 bytes per beam);
 *                       entries at k >= K must be zero (tcbf_block_weights
 *                       writes them so).  A layout only; needs b_layout
 *                       TCBF_PLANAR and N a multiple of 8 (any K); variants
 *                       0 (default), 2, 5, 6, 8, 9.  Results are bitwise
 *                       identical to the planar layout's.
 *   B = X   planar      [batch][2][K][N]   N contiguous
 *           interleaved [batch][K][N][2]
 *           with b_k_contiguous: planar [batch][2][N][K], interleaved
 *           [batch][N][K][2] (receivers contiguous for each sample, as
 *           sensor data often arrives); variant 1 only
 *   C = out planar      [batch][2][M][N]   fp32
 *           interleaved [batch][M][N][2]   fp32
 *
 * TCBF_INT1 buffer layouts (packed as tcbf_pack1bit writes them; kw = ceil(K/32)):
 *   A = W   [batch][2][M][kw]  uint32, sample k in bit k%32 of word k/32
 *   B = X   [batch][2][N][kw]  uint32, packed along K for each sample n
 *   C = out planar [batch][2][M][N] or interleaved [batch][M][N][2], int32
 *   a_layout and b_layout must be TCBF_PLANAR (the packed form).  Bits past K
 *   in the last word must be 0 (tcbf_pack1bit guarantees it).
 *
 * TCBF_F8_E4M3 / TCBF_MXF8_E4M3 layouts (as tcbf_quantize_e4m3 writes them;
 * codes are OCP FP8 E4M3 bytes; Kp = 32 * ceil(K / 32)):
 *   A = W   planar  [batch][2][M][Kp]  receivers contiguous, bytes past K zero
 *           blocked [batch][2][Kb][M][64], Kb = ceil(Kp / 64): receiver k of
 *                   row m in block k/64, position k%64 (each block all M rows
 *                   x 64 receivers); bytes past Kp are never read
 *   B = X   planar  [batch][2][N][Kp]  packed along K for each sample n
 *           blocked [batch][2][Kb][N][64]
 *   C = out planar [batch][2][M][N] or interleaved [batch][M][N][2], fp32
 *   a_layout and b_layout both TCBF_PLANAR or both TCBF_BLOCKED (results
 *   bitwise identical; blocked reads whole cache lines per stage); N must be
 *   a multiple of 4.
 *   Scales (tcbf_execute's a_scale, b_scale):
 *     TCBF_F8_E4M3:   fp32 a_scale [batch][M] (or [M] when a_shared), fp32
 *                     b_scale [batch][N]; out = a_scale[m] * b_scale[n] *
 *                     sum_k decode(W[m][k]) * decode(X[n][k]) (complex)
 *     TCBF_MXF8_E4M3: uint8 E8M0 codes (2^(code-127), 255 not allowed)
 *                     in groups of 16 blocks: a_scale [batch][Ks/16][M][16]
 *                     (or [Ks/16][M][16]), b_scale [batch][Ks/16][N][16],
 *                     Ks = 16 * ceil(Kp / 512); block j of row r (scaling
 *                     receivers 32j..32j+31) is at [j / 16][r][j % 16];
 *                     codes of blocks j >= Kp/32 are padding the library
 *                     never uses
 *
 * a_shared != 0: W holds a single batch entry that every channel uses.
 * a_batch_stride > 0: batch entry c's W starts a_batch_stride elements of
 * W's storage type (fp16 values, e4m3 code bytes, packed uint32 words) after
 * entry c-1's; at least one entry's size in the layout above, and a multiple
 * of 16 bytes; 0 means entries packed back to back (or the single shared
 * entry).  FP8 scales stay per entry ([batch][M] or blocked groups) unless
 * a_shared.  The FP8 and 1-bit X operands are always receiver-contiguous
 * (codes or packed words); b_k_contiguous may be 0 or 1 for them.
 * C is always overwritten (the output starts from zero, as in Sec. III-B).
 */
typedef struct tcbf_plan_desc {
    uint32_t struct_size; /* sizeof(tcbf_plan_desc), for ABI growth            */
    int32_t device;       /* HIP device ordinal the plan executes on           */
    int64_t batch;        /* >= 1                                              */
    int64_t M;            /* beams, >= 1                                       */
    int64_t N;            /* samples, >= 1                                     */
    int64_t K;            /* receivers, >= 1                                   */
    int32_t dtype;        /* tcbf_dtype                                        */
    int32_t a_layout;     /* tcbf_layout of W                                  */
    int32_t b_layout;     /* tcbf_layout of X                                  */
    int32_t c_layout;     /* tcbf_layout of the output                         */
    int32_t a_shared;     /* nonzero: one W for all batch entries              */
    int32_t variant;      /* 0 = automatic kernel choice; >0 forces a variant  */
    /* Fields below are read when struct_size covers them (TCBF_VERSION >= 4);
     * a shorter descriptor means b_k_contiguous = 0, a_batch_stride = 0. */
    int32_t b_k_contiguous; /* nonzero: fp16 X receiver-contiguous (see above) */
    int32_t reserved;       /* must be 0                                       */
    int64_t a_batch_stride; /* W elements between batch entries; 0 = packed    */
} tcbf_plan_desc;
/* Variants.  TCBF_F16: 1 register-staged kernel for any layout and alignment;
 * 2..9 the direct-to-LDS kernels (planar or blocked W, planar X, N a
 * multiple of 8, K a multiple of 8 for planar W): 2 128 x 128 tile, 32
 * receivers per stage, two-deep ring; 3 / 4 16 receivers, four / five deep;
 * 5 32 receivers, three deep; 6 / 7 a 256 x 128 tile (512 threads); 8 separate
 * rings for W (two deep) and X (three deep); 9 a persistent 256 x 128 tile
 * whose two wave groups alternate matrix and data phases (one workgroup per
 * CU).  The default is 9 for problems with at least as many 256 x 128 tiles
 * as the device has CUs and K > 32 (2 or more stages of 32 receivers per
 * tile), else 2.  TCBF_F8_E4M3 / TCBF_MXF8_E4M3: 1 (default)
 * 128 x 128 tile, two-deep ring, 2 three-deep, 3 the persistent 256 x 128
 * ping-pong tile (TCBF_MXF8_E4M3 only where ceil(Kp / 64) % 8 != 1).  TCBF_INT1: 1 int8 matrix instructions on
 * +-1 expanded to {0, 1}, 2 XOR + popcount on the vector ALU, 3 e2m1 (4-bit
 * float) matrix instructions on the +-1 values, for K <= 2^23 with
 * ceil(K/32) a multiple of 4 (default where it applies, else 1).  Every
 * variant of a dtype gives bitwise identical results.  A variant that does
 * not accept the problem makes tcbf_plan fail with TCBF_ERROR_INVALID_VALUE. */

typedef struct tcbf_plan_s *tcbf_plan_t;

/* What a plan chose; filled by tcbf_plan_query. */
typedef struct tcbf_plan_info {
    uint32_t struct_size;
    int32_t variant;           /* kernel variant id actually used             */
    int32_t tile_m, tile_n;    /* complex outputs per workgroup                */
    int32_t tile_k;            /* K per main-loop stage                        */
    int32_t threads;           /* threads per workgroup                        */
    int64_t workgroups;        /* workgroups per launch                        */
    double useful_ops;         /* 8*M*N*K*batch (Sec. IV-A op count)           */
    double algorithmic_bytes;  /* each input read once, output written once    */
    char kernel_name[64];      /* name of the main kernel (for profilers)      */
} tcbf_plan_info;

/*
 * tcbf_plan -- validate a problem and choose the kernel configuration
 * (Sec. III-C/IV-A: tile sizes are picked automatically for the device and
 * shapes).  Host-only; enqueues nothing.
 * Returns INVALID_VALUE for a NULL argument, a struct_size smaller than the
 * version-1 struct, non-positive sizes, unknown enum values or layouts the
 * dtype does not accept; NOT_SUPPORTED when `device` is not a gfx950 device
 * (or sizes exceed the kernels' 32-bit index limits); DEVICE when the HIP
 * runtime cannot report the device.  On success *plan owns host memory only.
 */
tcbf_status tcbf_plan(const tcbf_plan_desc *desc, tcbf_plan_t *plan);

/*
 * tcbf_execute -- enqueue B = W . X on `stream` (Sec. III-B: four real
 * products per complex product, Im(X) negated in registers; Sec. III-D for
 * TCBF_INT1).  A, B, C are device pointers in the plan's layouts, each 16-byte
 * aligned; C must not overlap A or B.  a_scale and b_scale are device
 * pointers to the FP8 scales described above (16-byte aligned) and must be
 * NULL for TCBF_F16 and TCBF_INT1.  Asynchronous, allocation-free and
 * graph-capturable.  The device that is current on the calling thread must be
 * the plan's device.
 */
tcbf_status tcbf_execute(tcbf_plan_t plan, const void *A, const void *B, void *C,
                         const void *a_scale, const void *b_scale, void *stream);

/*
 * tcbf_block_weights -- repack 16-bit weights (fp16 or bfloat16: values are
 * moved, never interpreted) into the TCBF_BLOCKED layout
 * (Sec. III: the library's transpose kernel tiles the inputs in device memory;
 * here, the receiver axis of W in blocks of 32).
 *   src (device): W, planar [batch][2][M][K] (src_layout TCBF_PLANAR) or
 *                 interleaved [batch][M][K][2] (TCBF_INTERLEAVED).
 *   dst (device): [batch][2][ceil(K/32)][M][32]; receivers k >= K are
 *                 written as +0 (bits 0, in both formats).  Values are copied
 *                 bit for bit.
 * src and dst must be 16-byte aligned device pointers that do not overlap.
 * Asynchronous on `stream`, allocation-free.  TCBF_ERROR_INVALID_VALUE for
 * NULL or misaligned pointers, sizes below 1 or a src_layout other than
 * TCBF_PLANAR / TCBF_INTERLEAVED; TCBF_ERROR_NOT_SUPPORTED for sizes whose
 * launch would exceed 2^31 - 1 workgroups.
 */
tcbf_status tcbf_block_weights(const void *src, int32_t src_layout, int64_t batch, int64_t M,
                               int64_t K, void *dst, void *stream);

/*
 * tcbf_pack1bit -- sign-pack complex data for TCBF_INT1 (Sec. III kernels
 * paragraph: 32 consecutive 1-bit samples per 32-bit word; Sec. III-D and
 * Fig. 1: per component bit 1 = +1, bit 0 = -1).
 *   sign rule: integers: bit = (x >= 0); floats: bit = sign bit clear, so +0
 *   gives +1 and -0 gives -1.
 *   src (device), element type src_type, complex layout src_layout:
 *     src_k_major != 0:  planar [batch][2][rows][K]   or interleaved [batch][rows][K][2]
 *     src_k_major == 0:  planar [batch][2][K][rows]   or interleaved [batch][K][rows][2]
 *   (W is K-major with rows = M; X as beamformer data [K][N] is not, rows = N.)
 *   dst (device): [batch][2][rows][ceil(K/32)] uint32, LSB first, pad bits 0.
 * src and dst must be 16-byte aligned device pointers that do not overlap.
 */
tcbf_status tcbf_pack1bit(const void *src, int32_t src_type, int32_t src_layout,
                          int64_t batch, int64_t rows, int64_t K, int32_t src_k_major,
                          uint32_t *dst, void *stream);

/*
 * tcbf_quantize_e4m3 -- quantise complex data to the FP8 operand form.
 * The paper has no 8-bit kernel (Sec. VI names 8-bit floats as future work);
 * the rule is the library's.  Every value x of a row (both parts) or of a
 * 32-receiver block of a row is mapped to the nearest e4m3 code (ties to an
 * even mantissa, saturating at +-448, NaN to 0x7f) of:
 *   block == 0:  x * (448 / amax), scale = amax / 448 (both fp32; 1 and 1 when
 *                amax == 0), amax = max |x| over the row's re and im parts
 *   block == 32: ldexp(x, -e), scale code e + 127, e the smallest integer with
 *                amax <= 448 * 2^e over the block (clamped to [-127, 127],
 *                0 for an all-zero block)
 *   src (device), src_type, src_layout and src_k_major as for tcbf_pack1bit.
 *   dst (device), dst_layout TCBF_PLANAR: [batch][2][rows][Kp] bytes,
 *   Kp = 32 * ceil(K / 32), zero past K; TCBF_BLOCKED: [batch][2][Kb][rows][64],
 *   Kb = ceil(Kp / 64), receiver k of row r at [k / 64][r][k % 64], zero past
 *   K (the whole last block written).  scales (device): block 0: fp32 [batch][rows]; block 32: uint8
 *   [batch][Ks / 16][rows][16], Ks = 16 * ceil(Kp / 512), block j of row r
 *   at [j / 16][r][j % 16] (the padding codes j >= Kp / 32 are not written).
 * src, dst and scales must be 16-byte aligned device buffers that do not
 * overlap.  Enqueues several kernels on `stream`; allocation-free.
 */
tcbf_status tcbf_quantize_e4m3(const void *src, int32_t src_type, int32_t src_layout,
                               int64_t batch, int64_t rows, int64_t K, int32_t src_k_major,
                               int32_t block, int32_t dst_layout, uint8_t *dst, void *scales,
                               void *stream);

/*
 * tcbf_steering_weights -- the weights W of Eq. 3 from array geometry, with
 * the phase in FP64 on the device.  Sec. II's far-field delay (Eq. 2), for sensor k at
 * positions[k] = (x, y, z) metres and beam m along directions[m] = (l, m, n)
 * (direction cosines), is tau = (x l + y m + z n) / wave_speed; the weight
 * that re-aligns its phase at frequencies[c] is
 *     W[c][m][k] = exp(+i 2 pi frac(f tau)),   frac(v) = v - floor(v),
 * with s = x l + y m + z n summed left to right, cycles = (f s) / wave_speed,
 * every FP64 operation rounded on its own (nothing fused).  cos/sin of
 * 2 pi frac(cycles) come from the device math library: in FP64 for fp32
 * output (each value rounded once, to nearest); for fp16 output, after an
 * exact FP64 split of frac(cycles) into quarter turns and a remainder of at
 * most 1/8 turn, from the fp32 sincospi of the remainder (relative error
 * about 2^-21 before the rounding to fp16 nearest-even, so at most one fp16
 * ulp from the correctly rounded value and equal to it except near rounding
 * boundaries).
 *   positions (device) [K][3] double, directions (device) [M][3] double,
 *   frequencies (device) [batch] double, all 8-byte aligned;
 *   W (device, 16-byte aligned), element type out_type = TCBF_SRC_F16 or
 *   TCBF_SRC_F32, out_layout TCBF_PLANAR: [batch][2][M][K]; out_layout
 *   TCBF_BLOCKED (fp16 only): the receiver-blocked [batch][2][ceil(K/32)][M][32]
 *   with zeros past K, the same values as tcbf_block_weights of the planar
 *   output.  These are the TCBF_F16 operand layouts of W; FP8 weights follow
 *   with tcbf_quantize_e4m3.
 * Returns INVALID_VALUE for NULL or misaligned pointers, non-positive sizes,
 * a wave speed that is not positive and finite, another out_type, or another
 * out_layout (blocked with fp32 included).
 * Asynchronous on `stream`; allocation-free.
 */
tcbf_status tcbf_steering_weights(const double *positions, const double *directions,
                                  const double *frequencies, double wave_speed, int64_t batch,
                                  int64_t M, int64_t K, int32_t out_type, int32_t out_layout,
                                  void *W, void *stream);

/*
 * Grouped persistent launch (TCBF_F16, TCBF_F8_E4M3, TCBF_MXF8_E4M3,
 * TCBF_INT1): up to TCBF_GROUP_MAX independent problems of different shapes
 * -- channels, frames or jobs, each B = W . X in the layouts of `dtype`
 * (planar or receiver-blocked W and planar X for fp16; the row-major or
 * blocked e4m3 codes and the scales of that FP8 mode; the packed sign words
 * for 1-bit, int8-MFMA variant; the `layout` field, one per launch) -- run in
 * ONE launch.  The
 * problems' output tiles form one work list, longest receiver count first
 * (the paper's Sec. IV-C size sweep shows per-shape padding and tail effects;
 * one shared list keeps every CU busy across shape boundaries); persistent
 * workgroups (two per CU) take tiles from a device counter until the list is
 * empty.  fp16 problems whose variant (given, or the plan's default) has
 * 256-beam tiles (6, 7, 9) run instead in a grouped form of the ping-pong
 * kernel (one 512-thread workgroup per CU, a static tile list), so a call
 * makes at most two persistent launches, one after the other on `stream`.
 * The problem table travels in the launch's kernel arguments, so the call
 * can be captured in a HIP graph and replayed.
 *   problems: host array of `count` descriptors (1 <= count <= TCBF_GROUP_MAX);
 *     each needs batch, M, N, K >= 1, 16-byte aligned device pointers and
 *     the size limits of a plan of its dtype; fp16: N a multiple of 8 and
 *     K too with planar W, per-channel W and X below 2 GiB, a_scale =
 *     b_scale = NULL; every problem the same `layout`; FP8: N a
 *     multiple of 4, a_scale and b_scale as for tcbf_execute; 1-bit: K at
 *     most 2^26, a_scale = b_scale = NULL, int32 output.  Every
 *     problem's output equals its own plan's (default variant) bit for bit.
 *   workspace: device memory of TCBF_GROUP_WORKSPACE_BYTES, 16-byte aligned,
 *     used for the tile counter; calls that overlap in time (on different
 *     streams) need different workspaces.
 * The current device must be `device`.  Enqueues two kernels on `stream`
 * (counter reset, persistent product); allocation-free.
 */
#define TCBF_GROUP_MAX 32
#define TCBF_GROUP_WORKSPACE_BYTES 256

typedef struct tcbf_group_problem {
    const void *A;       /* W in the dtype's layout (shared: one batch entry) */
    const void *B;       /* X in the dtype's layout                           */
    void *C;             /* output (fp32; int32 for 1-bit), layout c_layout   */
    int64_t batch, M, N, K;
    int32_t a_shared;    /* nonzero: one W for all batch entries              */
    int32_t layout;      /* TCBF_PLANAR (0) or TCBF_BLOCKED: fp16 W blocked
                            (X planar), FP8 W and X codes blocked; 1-bit
                            planar only.  The same for every problem of one
                            launch.                                           */
    const void *a_scale; /* FP8 modes: W scales; fp16: NULL                   */
    const void *b_scale; /* FP8 modes: X scales; fp16: NULL                   */
    int32_t variant;     /* fp16: 0 = the plan's default for this problem, or
                            a fast variant 2..9 a plan of this problem takes
                            (e.g. the autotuner's choice); FP8, 1-bit: 0     */
    int32_t reserved;    /* 0                                                 */
} tcbf_group_problem;

tcbf_status tcbf_group_execute(int32_t device, int32_t dtype, int32_t c_layout,
                               const tcbf_group_problem *problems, int32_t count,
                               void *workspace, void *stream);

/*
 * Allocation-free grouped launch, for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same launch as
 * tcbf_group_execute, with the same arguments, checks and results, except
 * that the tile counter lives in a library-owned scratch array of
 * TCBF_GROUP_SCRATCH_BYTES per GPU (a static device array, held by every GPU
 * the library runs on until the process ends) instead of a workspace.  The
 * counter is reset by a kernel at the start of every launch.  All calls on
 * one GPU share that array: calls whose launches overlap in time on one GPU
 * (different streams, or different threads) race on the counter and give
 * wrong results; use tcbf_group_execute with one workspace per stream for
 * those.  Rejects count outside 1..TCBF_GROUP_MAX (the launch's size limit)
 * and a device index of 64 or more with an error; calls no allocating
 * routine.  The current device must be `device`.
 */
#define TCBF_GROUP_SCRATCH_BYTES 256

tcbf_status tcbf_group_execute_noalloc(int32_t device, int32_t dtype, int32_t c_layout,
                                       const tcbf_group_problem *problems, int32_t count,
                                       void *stream);

/*
 * Peak probe (measurement tool, not a step of the product): the throughput of
 * one matrix instruction (or of the VALU xor/popcount pair) on register
 * operands with no global-memory traffic, the measured ceiling the paper
 * places its kernels against (Sec. III-A, Table 1; Sec. IV-B).  Every wave
 * of `blocks` workgroups of 256 threads runs `iterations` rounds of 4
 * independent accumulations (VALU: 8 words per lane per round).  Operands:
 *   TCBF_PROBE_UNIFORM: every element has the bit pattern `operand_bits`
 *     (unit operands give closed-form accumulator values);
 *   TCBF_PROBE_RANDOM: two sets of pseudo-random elements per lane (seeded
 *     by operand_bits; fp16 and e4m3 in +-[0.5, 1)), alternated from one
 *     instruction to the next as real data changes them -- the chip's power
 *     draw and sustained clock depend on it.
 * Kinds:
 *   TCBF_PROBE_F16  v_mfma_f32_32x32x16_f16, element = operand_bits & 0xffff
 *   TCBF_PROBE_I8   v_mfma_i32_32x32x32_i8, four int8 per 32-bit word
 *   TCBF_PROBE_F8   scaled 32x32x64 f8f6f4 MFMA with e4m3 operands, scale 2^0
 *   TCBF_PROBE_F4   the same instruction with e2m1 operands
 *   TCBF_PROBE_VALU_XOR_POPC  per lane cnt += popcount(word ^ b), b changing
 *                   every round (32 bit-products, counted as 64 operations)
 *   sink (device, 16-byte aligned, sink_bytes >= blocks * 1056): first
 *     uint32 [blocks * 256], one accumulator value per thread (float bits for
 *     F16/F8/F4: the sum over the 4 chains of accumulator element
 *     thread % 16;
 *     int32 for I8; the VALU popcount total); then uint64 [blocks][4]: the
 *     shader-clock counter and the constant 100 MHz counter read by thread 0
 *     before and after its loop.
 *   ops (host, may be NULL): the useful operations of the launch (2 per
 *     multiply-add), to divide by the launch time the caller measures.
 * Enqueues one kernel on `stream` of the current device; allocation-free.
 */
enum tcbf_probe_operands { TCBF_PROBE_UNIFORM = 0, TCBF_PROBE_RANDOM = 1 };

enum tcbf_probe_kind {
    TCBF_PROBE_F16 = 0,
    TCBF_PROBE_I8 = 1,
    TCBF_PROBE_F8 = 2,
    TCBF_PROBE_F4 = 3,
    TCBF_PROBE_VALU_XOR_POPC = 4
};

tcbf_status tcbf_peak_probe(int32_t kind, int64_t blocks, int64_t iterations, uint32_t operand_bits,
                            int32_t operand_mode, void *sink, int64_t sink_bytes, double *ops, void *stream);

/* Report the plan's choice.  info->struct_size must be set by the caller. */
tcbf_status tcbf_plan_query(tcbf_plan_t plan, tcbf_plan_info *info);

/* Release a plan (NULL is accepted).  Must not race with tcbf_execute on it. */
tcbf_status tcbf_plan_destroy(tcbf_plan_t plan);

/* Static, human-readable name of a status code. */
const char *tcbf_status_string(tcbf_status status);

/* TCBF_VERSION of the built library. */
int32_t tcbf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TCBF_H */
