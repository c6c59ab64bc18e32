// FP16 batched complex product B[c] = W[c] . X[c] on gfx950 MFMA.
//
// Complex product as four real products with one imaginary part negated in
// registers (Sec. III-B): Re += Wr.Xr + (-Wi).Xi, Im += Wr.Xi + Wi.Xr, fp16 x
// fp16 products accumulated in fp32 by v_mfma_f32_32x32x16_f16.
//
// Tiling (both kernels): a workgroup of 256 threads (4 waves) owns 128 x 128
// complex outputs; each wave owns 64 x 64 = 2 x 2 MFMA tiles of 32 x 32, with a
// real and an imaginary fp32 accumulator each (128 registers).  Per K stage
// the workgroup brings the W tile (both planes) and the X tile (both planes)
// into LDS once, and all four real products of every wave read that single
// copy (Sec. III-C data reuse).  In the accumulators, lanes 0..31 of a wave
// hold 32 consecutive samples of one beam, so every output store instruction
// writes whole 128-byte row segments.  Two workgroups fit on a CU (64 KiB LDS,
// <= 256 VGPRs), so one drains its stores while the other multiplies.
// Workgroup ids are remapped so consecutive tiles of a channel stay on one
// XCD's L2.
//
// Two kernels share the exact same MFMA sequence (same 16-receiver steps in
// increasing order, same k assignment per lane, same operand order and
// accumulation order), so they produce bitwise-identical results:
//  * cgemm_f16_fast_kernel: planar (or receiver-blocked) W, planar X, K and N
//    multiples of 8 (any K with blocked W).  Global
//    tiles go straight into LDS with buffer_load ... lds (no registers, no
//    ALU work per stage) through a ring of NS stage buffers; out-of-range rows,
//    columns and the K tail read as zero through the buffer descriptor's range
//    check.  X stays N-contiguous in LDS and its MFMA fragments are read with
//    ds_read_b64_tr_b16, which transposes 4 x 16 blocks of 16-bit values
//    across each 16-lane group.  Stores use scalar row offsets, so the
//    epilogue spends no vector ALU work on addresses.
//  * cgemm_f16_kernel: any layout and alignment.  Tiles go through registers,
//    interleaved (re, im) data is split into planes and X is transposed while
//    being written to LDS.
#include <string.h>

#include <algorithm>

#include "tcbf_tile.h"

namespace tcbf {
namespace {

using namespace tile;
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef short short4v __attribute__((ext_vector_type(4)));
#define LDS_AS TCBF_LDS_AS

constexpr int BK = 32;                    // receivers per stage (generic kernel)
constexpr int PLANE_A = BM * BK;          // halves per W plane in a stage
constexpr int PLANE_B = BN * BK;          // halves per X plane in a stage
constexpr int STAGE = 2 * PLANE_A + 2 * PLANE_B;  // 16384 halves = 32 KiB

__device__ __forceinline__ half8 negate(half8 v) {
    u32x4 u = __builtin_bit_cast(u32x4, v);
    u ^= 0x80008000u;  // flip both fp16 sign bits: exact negation
    return __builtin_bit_cast(half8, u);
}

// The 32 x 32 x 16 matrix instruction on 16-bit operands held as raw 16-bit
// patterns: fp16 (BF = 0) or bfloat16 (BF = 1).  Loads, LDS staging and the
// sign flip of negate() are the same for both formats (bit 15 is the sign).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
template <int BF>
__device__ __forceinline__ f32x16 mfma16(const half8 &a, const half8 &b, const f32x16 &c) {
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// One 16-receiver step.  w*: W fragments (lane l: beam l%32, receivers
// 8*(l/32) + 0..7); x*: X fragments (lane l: sample l%32, same receivers).
// X is the matrix unit's first operand, so the result comes out transposed
// (samples along the accumulator's row index).
template <int BF = 0>
__device__ __forceinline__ void mma_step(Acc &a, const half8 (&wr)[2], const half8 (&wi)[2],
                                         const half8 (&xr)[2], const half8 (&xi)[2]) {
    half8 wn[2] = {negate(wi[0]), negate(wi[1])};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            a.re[i][j] = mfma16<BF>(xr[j], wr[i], a.re[i][j]);
            a.im[i][j] = mfma16<BF>(xi[j], wr[i], a.im[i][j]);
            a.re[i][j] = mfma16<BF>(xi[j], wn[i], a.re[i][j]);
            a.im[i][j] = mfma16<BF>(xr[j], wi[i], a.im[i][j]);
        }
}

// ===========================================================================
// Generic kernel: register-staged loads (any layout, any alignment).
// ===========================================================================

// Offset in halves of 16-byte chunk `ch` (0..3, i.e. k = 8ch..8ch+7) of row
// `row` inside a [rows][32] fp16 plane.  Two rows share a 128-byte line whose
// eight chunks are XOR-swizzled by the line index.
__device__ __forceinline__ int lds_off(int row, int ch) {
    int line = row >> 1;
    int slot = (((row & 1) << 2) | ch) ^ (line & 7);
    return line * 64 + slot * 8;
}

// Load 8 consecutive fp16 values (as raw bits), zero past `valid`.
__device__ __forceinline__ u32x4 load8(const uint16_t *p, int valid, bool vec) {
    if (vec && valid >= 8) return *reinterpret_cast<const u32x4 *>(p);
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (e < valid) ? (uint32_t)p[e] : 0u;
    u32x4 r;
    r.x = h[0] | (h[1] << 16);
    r.y = h[2] | (h[3] << 16);
    r.z = h[4] | (h[5] << 16);
    r.w = h[6] | (h[7] << 16);
    return r;
}

__device__ __forceinline__ uint32_t lo16(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
__device__ __forceinline__ uint32_t hi16(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }
__device__ __forceinline__ uint32_t el(const u32x4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// ---------------------------------------------------------------------------
// Global -> register loaders (one K stage).  Each thread owns 4 x 16 bytes.
// ---------------------------------------------------------------------------

// W planar [2][M][K]: chunk q -> plane q>>9, row (q>>2)&127, 8-k chunk q&3.
struct ALoaderPlanar {
    const uint16_t *p[4];
    int row_ok[4];
    int kofs[4];
    __device__ void init(const uint16_t *W, int64_t M, int64_t K, int64_t m0, int tid) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int q = tid + i * NT;
            int plane = q >> 9, row = (q >> 2) & (BM - 1), ch = q & 3;
            int64_t m = m0 + row;
            row_ok[i] = m < M;
            kofs[i] = ch * 8;
            p[i] = W + (int64_t)plane * M * K + (row_ok[i] ? m : 0) * K + ch * 8;
        }
    }
    __device__ void load(u32x4 (&r)[4], int64_t k0, int64_t K, bool vec) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int64_t left = K - k0 - kofs[i];
            int valid = row_ok[i] ? (int)(left < 8 ? (left < 0 ? 0 : left) : 8) : 0;
            r[i] = load8(p[i] + k0, valid, vec);
        }
    }
    __device__ static void store(uint16_t *st, int tid, const u32x4 (&r)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int q = tid + i * NT;
            int plane = q >> 9, row = (q >> 2) & (BM - 1), ch = q & 3;
            *reinterpret_cast<u32x4 *>(st + plane * PLANE_A + lds_off(row, ch)) = r[i];
        }
    }
};

// W interleaved [M][K][2]: item q (0..511) -> row q>>2, 8-k chunk q&3; two
// 16-byte loads of 4 complex values each.
struct ALoaderInter {
    const uint16_t *p[2];
    int row_ok[2];
    int kofs[2];
    __device__ void init(const uint16_t *W, int64_t M, int64_t K, int64_t m0, int tid) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int q = tid + i * NT;
            int row = q >> 2, ch = q & 3;
            int64_t m = m0 + row;
            row_ok[i] = m < M;
            kofs[i] = ch * 8;
            p[i] = W + ((row_ok[i] ? m : 0) * K + ch * 8) * 2;
        }
    }
    __device__ void load(u32x4 (&r)[4], int64_t k0, int64_t K, bool vec) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int64_t left = K - k0 - kofs[i];  // complex values left in the row
            int valid = row_ok[i] ? (int)(left < 8 ? (left < 0 ? 0 : left) : 8) : 0;
            r[2 * i] = load8(p[i] + 2 * k0, 2 * valid, vec);
            r[2 * i + 1] = load8(p[i] + 2 * k0 + 8, 2 * valid - 8, vec);
        }
    }
    __device__ static void store(uint16_t *st, int tid, const u32x4 (&r)[4]) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int q = tid + i * NT;
            int row = q >> 2, ch = q & 3;
            const u32x4 &a = r[2 * i], &b = r[2 * i + 1];
            u32x4 re, im;
            re.x = lo16(a.x, a.y); re.y = lo16(a.z, a.w); re.z = lo16(b.x, b.y); re.w = lo16(b.z, b.w);
            im.x = hi16(a.x, a.y); im.y = hi16(a.z, a.w); im.z = hi16(b.x, b.y); im.w = hi16(b.z, b.w);
            *reinterpret_cast<u32x4 *>(st + lds_off(row, ch)) = re;
            *reinterpret_cast<u32x4 *>(st + PLANE_A + lds_off(row, ch)) = im;
        }
    }
};

// X planar [2][K][N]: thread -> plane tid>>7, 8-n group (tid>>3)&15, 4-k group
// tid&7; loads 4 rows of 8 n, stores 8 columns of 4 k (transposed).
struct BLoaderPlanar {
    const uint16_t *p;
    int64_t N;
    int kofs;
    int n_left0;  // N - n for this thread's first column (may be <= 0)
    __device__ void init(const uint16_t *X, int64_t K, int64_t N_, int64_t n0, int tid) {
        N = N_;
        int plane = tid >> 7, ng = (tid >> 3) & 15, kg = tid & 7;
        int64_t n = n0 + ng * 8;
        kofs = kg * 4;
        n_left0 = (int)((N - n) > 8 ? 8 : (N - n));
        p = X + (int64_t)plane * K * N + (int64_t)kofs * N + (n < N ? n : 0);
    }
    __device__ void load(u32x4 (&r)[4], int64_t k0, int64_t K, bool vec) {
        const uint16_t *q = p + k0 * N;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int valid = (k0 + kofs + i < K) ? (n_left0 > 0 ? n_left0 : 0) : 0;
            r[i] = load8(q + i * N, valid, vec);
        }
    }
    __device__ static void store(uint16_t *st, int tid, const u32x4 (&r)[4]) {
        int plane = tid >> 7, ng = (tid >> 3) & 15, kg = tid & 7;
        uint16_t *base = st + 2 * PLANE_A + plane * PLANE_B;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int n = ng * 8 + e;
            uint32_t d0 = el(r[0], e >> 1), d1 = el(r[1], e >> 1);
            uint32_t d2 = el(r[2], e >> 1), d3 = el(r[3], e >> 1);
            u32x2 v;
            if (e & 1) { v.x = hi16(d0, d1); v.y = hi16(d2, d3); }
            else       { v.x = lo16(d0, d1); v.y = lo16(d2, d3); }
            *reinterpret_cast<u32x2 *>(base + lds_off(n, kg >> 1) + (kg & 1) * 4) = v;
        }
    }
};

// X interleaved [K][N][2]: thread -> 4-complex n group (tid>>3) (0..31), 4-k
// group tid&7; loads 4 rows x 4 complex, stores 4 columns x 4 k per plane.
struct BLoaderInter {
    const uint16_t *p;
    int64_t N;
    int kofs;
    int n_left0;
    __device__ void init(const uint16_t *X, int64_t K, int64_t N_, int64_t n0, int tid) {
        (void)K;
        N = N_;
        int ng = tid >> 3, kg = tid & 7;
        int64_t n = n0 + ng * 4;
        kofs = kg * 4;
        n_left0 = (int)((N - n) > 4 ? 4 : (N - n));
        p = X + ((int64_t)kofs * N + (n < N ? n : 0)) * 2;
    }
    __device__ void load(u32x4 (&r)[4], int64_t k0, int64_t K, bool vec) {
        const uint16_t *q = p + k0 * N * 2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int valid = (k0 + kofs + i < K) ? (n_left0 > 0 ? 2 * n_left0 : 0) : 0;
            r[i] = load8(q + i * N * 2, valid, vec);
        }
    }
    __device__ static void store(uint16_t *st, int tid, const u32x4 (&r)[4]) {
        int ng = tid >> 3, kg = tid & 7;
        uint16_t *base = st + 2 * PLANE_A;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int n = ng * 4 + e;
            // complex e of each row sits in dword e: re = low half, im = high half
            uint32_t d0 = el(r[0], e), d1 = el(r[1], e), d2 = el(r[2], e), d3 = el(r[3], e);
            u32x2 re, im;
            re.x = lo16(d0, d1); re.y = lo16(d2, d3);
            im.x = hi16(d0, d1); im.y = hi16(d2, d3);
            int off = lds_off(n, kg >> 1) + (kg & 1) * 4;
            *reinterpret_cast<u32x2 *>(base + off) = re;
            *reinterpret_cast<u32x2 *>(base + PLANE_B + off) = im;
        }
    }
};

// X receiver-contiguous, planar [2][N][K] or interleaved [N][K][2]: the
// same rows as W's (samples in place of beams), staged into the X region,
// which has W's row layout (the MFMA's B operand is read by sample rows).
static_assert(BM == BN && PLANE_A == PLANE_B, "X rows stage like W rows");
template <class L> struct BLoaderKMajor {
    L l;
    __device__ void init(const uint16_t *X, int64_t K, int64_t N, int64_t n0, int tid) { l.init(X, N, K, n0, tid); }
    __device__ void load(u32x4 (&r)[4], int64_t k0, int64_t K, bool vec) { l.load(r, k0, K, vec); }
    __device__ static void store(uint16_t *st, int tid, const u32x4 (&r)[4]) { L::store(st + 2 * PLANE_A, tid, r); }
};

template <int AIL> struct ASel { typedef ALoaderPlanar T; };
template <> struct ASel<1> { typedef ALoaderInter T; };
// BIL: 0 planar [2][K][N], 1 interleaved [K][N][2], 2 planar [2][N][K],
// 3 interleaved [N][K][2]
template <int BIL> struct BSel { typedef BLoaderPlanar T; };
template <> struct BSel<1> { typedef BLoaderInter T; };
template <> struct BSel<2> { typedef BLoaderKMajor<ALoaderPlanar> T; };
template <> struct BSel<3> { typedef BLoaderKMajor<ALoaderInter> T; };

__device__ __forceinline__ half8 lds_frag(const uint16_t *plane, int row, int ch) {
    return *reinterpret_cast<const half8 *>(plane + lds_off(row, ch));
}

// Store one lane's four consecutive samples (re[4], im[4]) of beam m starting
// at sample n, masked to the problem.
template <int CIL>
__device__ __forceinline__ void store4(float *C, int64_t c, int64_t M, int64_t N, int64_t m, int64_t n,
                                       const f32x4 &re, const f32x4 &im) {
    if (m >= M || n >= N) return;
    const bool whole = n + 4 <= N;
    if (CIL) {
        float *o = C + ((c * M + m) * N + n) * 2;
        if (whole && (((uintptr_t)o & 15) == 0)) {
            *reinterpret_cast<f32x4 *>(o) = (f32x4){re[0], im[0], re[1], im[1]};
            *reinterpret_cast<f32x4 *>(o + 4) = (f32x4){re[2], im[2], re[3], im[3]};
        } else {
            for (int e = 0; e < 4 && n + e < N; ++e) {
                o[2 * e] = re[e];
                o[2 * e + 1] = im[e];
            }
        }
    } else {
        float *o = C + (c * 2 * M + m) * N + n;
        float *oi = o + M * N;
        if (whole && (((uintptr_t)o & 15) == 0) && (((uintptr_t)oi & 15) == 0)) {
            *reinterpret_cast<f32x4 *>(o) = re;
            *reinterpret_cast<f32x4 *>(oi) = im;
        } else {
            for (int e = 0; e < 4 && n + e < N; ++e) {
                o[e] = re[e];
                oi[e] = im[e];
            }
        }
    }
}

template <int AIL, int BIL, int CIL, int BF = 0>
__global__ __launch_bounds__(NT, 2) void cgemm_f16_kernel(
    const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, float *__restrict__ C,
    int64_t M, int64_t N, int64_t K, int64_t a_stride, int tiles_m, int tiles_n, int64_t nblocks,
    int a_vec, int b_vec) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];

    const int tid = threadIdx.x;
    const int64_t t = xcd_remap(blockIdx.x, nblocks);
    const int64_t per_c = (int64_t)tiles_m * tiles_n;
    const int64_t c = t / per_c;
    const int rem = (int)(t - c * per_c);
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

    const uint16_t *Wc = A + c * a_stride;
    const uint16_t *Xc = B + c * 2 * K * N;

    typename ASel<AIL>::T al;
    typename BSel<BIL>::T bl;
    al.init(Wc, M, K, m0, tid);
    bl.init(Xc, K, N, n0, tid);

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    Acc acc;
    acc.zero();

    const int nk = (int)((K + BK - 1) / BK);
    u32x4 ra[4], rb[4];
    al.load(ra, 0, K, a_vec);
    bl.load(rb, 0, K, b_vec);
    ASel<AIL>::T::store(lds, tid, ra);
    BSel<BIL>::T::store(lds, tid, rb);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const uint16_t *st = lds + (kt & 1) * STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            al.load(ra, (int64_t)(kt + 1) * BK, K, a_vec);
            bl.load(rb, (int64_t)(kt + 1) * BK, K, b_vec);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int ch = 2 * s + hl;
            half8 wr[2], wi[2], xr[2], xi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                int row = wm * 64 + i * 32 + l32;
                wr[i] = lds_frag(st, row, ch);
                wi[i] = lds_frag(st + PLANE_A, row, ch);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                int col = wn * 64 + j * 32 + l32;
                xr[j] = lds_frag(st + 2 * PLANE_A, col, ch);
                xi[j] = lds_frag(st + 2 * PLANE_A + PLANE_B, col, ch);
            }
            mma_step<BF>(acc, wr, wi, xr, xi);
        }
        if (more) {
            uint16_t *nx = lds + ((kt + 1) & 1) * STAGE;
            ASel<AIL>::T::store(nx, tid, ra);
            BSel<BIL>::T::store(nx, tid, rb);
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t m = m0 + wm * 64 + i * 32 + l32;
                const int64_t n = n0 + wn * 64 + j * 32 + 8 * q + 4 * hl;
                store4<CIL>(C, c, M, N, m, n, quad(acc.re[i][j], q), quad(acc.im[i][j], q));
            }
}

// ===========================================================================
// Fast kernel: direct-to-LDS loads, transposing LDS reads, NS-deep ring.
// ===========================================================================
//
// The workgroup has 2*WM waves in a WM x 2 grid and owns TM = 64*WM beams x
// 128 samples.  LDS stage (bytes), for a stage of BK receivers:
//   W region [2 planes][TM beams][BK] fp16: rows of BK*2 bytes split in
//     16-byte chunks; chunk ch of beam m sits at ch ^ swzW(m);
//   X region [2 planes][BK][128 samples] fp16: rows of 256 bytes (16 chunks);
//     chunk ch of row k sits at ch ^ swzX(k).
// The swizzles keep the MFMA operand reads free of bank conflicts (the W
// reads in 16-lane phases, the transposing X reads in 32-lane phases).
template <int WM, int BK> struct FastGeo {
    static constexpr int TM = 64 * WM;                 // beams per workgroup
    static constexpr int NW = 2 * WM;                  // waves
    static constexpr int WCH = BK / 8;                 // chunks per W row
    static constexpr int WREG = 2 * TM * BK * 2;       // W region bytes
    static constexpr int XREG = 2 * BK * BN * 2;       // X region bytes
    static constexpr int STAGE = WREG + XREG;          // stage bytes
    // both use only beam bits 1..3, so beams 16 apart share a swizzle
    __device__ static int swzW(int m) {
        return BK == 32 ? (((m >> 1) ^ ((m >> 3) & 1)) & 3) : (((m >> 2) ^ (m >> 3)) & 1);
    }
    // receiver rows k..k+3 get chunk offsets 0, 4, 8, 12: the transposing
    // fragment read of 32 lanes (4 rows x 64 bytes) then touches every bank
    // once (measured: no LDS bank conflicts)
    __device__ static int swzX(int k) { return 4 * (k & 3); }
};

__device__ __forceinline__ half8 tr_frag(const char *lds_bytes, int off0, int off1) {
    short4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDS_AS short4v *)(lds_bytes + off0));
    short4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((LDS_AS short4v *)(lds_bytes + off1));
    typedef short short8v __attribute__((ext_vector_type(8)));
    short8v v = (short8v){lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    return __builtin_bit_cast(half8, v);
}

// The stage buffers of one workgroup.  Every buffer is its own __shared__
// object, so the compiler can tell the direct-to-LDS writes into one from the
// fragment reads of another; buffers past the ring depth are 4-byte stubs.
template <int WM, int BK, int NS> struct FastLds {
    typedef FastGeo<WM, BK> G;
    static constexpr int S2 = NS > 2 ? G::STAGE : 4, S3 = NS > 3 ? G::STAGE : 4, S4 = NS > 4 ? G::STAGE : 4,
                         S5 = NS > 5 ? G::STAGE : 4;
};
#define TCBF_FAST_LDS(WM, BK, NS)                                                                          \
    __shared__ __attribute__((aligned(1024))) char lds0[FastGeo<WM, BK>::STAGE];                           \
    __shared__ __attribute__((aligned(1024))) char lds1[FastGeo<WM, BK>::STAGE];                           \
    __shared__ __attribute__((aligned(NS > 2 ? 1024 : 4))) char lds2[FastLds<WM, BK, NS>::S2];             \
    __shared__ __attribute__((aligned(NS > 3 ? 1024 : 4))) char lds3[FastLds<WM, BK, NS>::S3];             \
    __shared__ __attribute__((aligned(NS > 4 ? 1024 : 4))) char lds4[FastLds<WM, BK, NS>::S4];             \
    __shared__ __attribute__((aligned(NS > 5 ? 1024 : 4))) char lds5[FastLds<WM, BK, NS>::S5];

// One output tile (64*WM beams x 128 samples of channel c at tile (tm, tn)):
// the whole K loop and the epilogue.  Entered and left with the stage buffers
// idle; the caller separates two tiles of one workgroup with a barrier.
// AB: W in the receiver-blocked layout (TCBF_BLOCKED: per plane, blocks of
// 32 receivers, each block all M beams x 32 receivers), so a stage's W tile
// is one contiguous run per plane and every load instruction reads whole
// cache lines; with planar W each beam row contributes a 64-byte piece.
template <int WM, int BK, int NS, int CIL, int AB, int BF = 0>
__device__ __forceinline__ void fast_tile(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                          float *__restrict__ C, int M, int N, int K, int64_t a_stride, int c,
                                          int tm, int tn, char *lds0, char *lds1, char *lds2, char *lds3,
                                          char *lds4, char *lds5) {
    typedef FastGeo<WM, BK> G;
    constexpr int TM = G::TM, NW = G::NW;
    static_assert(NS >= 2 && NS <= 6, "ring depth");
    static_assert(G::WREG % (NW * 1024) == 0 && G::XREG % (NW * 1024) == 0, "whole wave loads");
    // stage buffer i: a select chain, not an array -- an array of LDS
    // pointers that the compiler cannot index statically goes to scratch
    // memory as generic pointers, and every fragment read becomes a flat load
    auto bufs = [&](int i) __attribute__((always_inline)) -> char * {
        char *b = lds0;
        if (i == 1) b = lds1;
        if (i == 2) b = lds2;
        if (i == 3) b = lds3;
        if (i == 4) b = lds4;
        if (i == 5) b = lds5;
        return b;
    };

    const int tid = threadIdx.x;
    const int m0 = tm * TM, n0 = tn * BN;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    static_assert(!AB || BK == 32, "blocked W holds 32-receiver blocks");
    const int KW = AB ? (K + 31) / 32 * 32 : K;  // receivers per W row as stored (blocked: padded)
    const uint16_t *Wc = A + (int64_t)c * a_stride;
    const uint16_t *Xc = B + (int64_t)c * 2 * K * N;
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc((void *)Wc, 0, 4 * M * KW, RSRC_FLAGS);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, 0, 4 * K * N, RSRC_FLAGS);

    // The 16-byte chunks this lane moves into LDS per stage.  A wave load
    // writes 1 KiB in lane order, so LDS slot s (16 B) = piece*64 + lane with
    // the workgroup's pieces dealt to waves in consecutive runs.  Within a wave
    // the pieces differ only by whole rows (same plane, same swizzle), so one
    // per-lane offset plus a uniform row stride per piece addresses them all.
    constexpr int WPIECES = G::WREG / 1024, XPIECES = G::XREG / 1024;
    constexpr int WPW = WPIECES / NW, XPW = XPIECES / NW;  // pieces per wave
    constexpr int WROWS = 64 / G::WCH, XROWS = 64 / 16;  // rows per piece
    uint32_t va, vb;   // byte offsets of piece 0
    int ka, kb, am;    // receiver offset of the W chunk, X row of piece 0, W beam of piece 0
    {
        const int s = wave * WPW * 64 + lane;
        const int p = s / (TM * G::WCH), m = (s / G::WCH) % TM;
        const int ch = (s % G::WCH) ^ G::swzW(m);
        ka = ch * 8;
        am = m;
        va = AB ? (uint32_t)(((p * (KW / 32)) * M + m0 + m) * 64 + ch * 16)
                : (uint32_t)(((p * M + m0 + m) * K + ch * 8) * 2);
    }
    {
        const int s = wave * XPW * 64 + lane;
        const int p = s / (BK * 16), k = (s / 16) % BK, ch = (s & 15) ^ G::swzX(k);
        kb = k;
        vb = (n0 + ch * 8 < N) ? (uint32_t)(((p * K + k) * N + n0 + ch * 8) * 2) : OOB;
    }
    const bool rows_full = m0 + TM <= M;

    // LDS byte offsets of this lane's MFMA fragments in a stage (plane 0):
    // W fragment for 16-receiver step s: beam wm*64 + l32, chunk 2s + hl;
    // X fragment for sample sub-tile j: this lane supplies row 8*(g/2) + (l%16)/4
    // and samples wn*64 + 32j + 16*(g%2) + 4*(l%4), g = l/16 (the transposing
    // read then hands lane l the 4 receivers of sample l%16 of its group).
    constexpr int KS = BK / 16;  // 16-receiver steps per stage
    int ow[2], ox[2];
    static_assert(KS <= 2, "steps per stage");
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int m = wm * 64 + l32;
        ow[s] = m * (BK * 2) + (((2 * s + hl) ^ G::swzW(m)) * 16);
    }
    {
        const int g = lane >> 4, j16 = lane & 15;
        const int krow = 8 * (g >> 1) + (j16 >> 2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ns = wn * 64 + 32 * j + 16 * (g & 1) + 4 * (j16 & 3);
            ox[j] = G::WREG + krow * 256 + (((ns >> 3) ^ G::swzX(krow)) * 16) + (ns & 7) * 2;
        }
    }

    auto issue = [&](char *base, int k0) __attribute__((always_inline)) {
        const bool tail = k0 + BK > K;
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            uint32_t off = va;
            if (!rows_full && m0 + am + q * WROWS >= M) off = OOB;  // beams past M
            if (tail && k0 + ka >= K) off = OOB;                    // receivers past K
            // uniform part: the stage's receiver block and this piece's rows
            const int so = AB ? (k0 / 32) * M * 64 + q * WROWS * 64 : k0 * 2 + q * WROWS * K * 2;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (LDS_AS void *)(base + (wave * WPW + q) * 1024), 16,
                                                     off, so, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            uint32_t off = vb;
            if (tail && k0 + kb + q * XROWS >= K) off = OOB;        // rows past K
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LDS_AS void *)(base + G::WREG + (wave * XPW + q) * 1024),
                                                     16, off, (k0 + q * XROWS) * N * 2, 0, 0);
        }
    };

    Acc acc;
    acc.zero();
    auto compute = [&](const char *st) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            half8 wr[2], wi[2], xr[2], xi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                wr[i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * BK * 2);
                wi[i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * BK * 2 + TM * BK * 2);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int o = ox[j] + s * 16 * 256;
                xr[j] = tr_frag(st, o, o + 4 * 256);
                xi[j] = tr_frag(st, o + BK * BN * 2, o + BK * BN * 2 + 4 * 256);
            }
            mma_step<BF>(acc, wr, wi, xr, xi);
            // keep one step's fragments live at a time (two workgroups per CU
            // leave 256 registers per lane)
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Ring: stage kt lives in buffer kt % NS; NS-1 stages are in flight.
    constexpr int PER_STAGE = WPW + XPW;  // loads per wave per stage
    static_assert((NS - 2) * PER_STAGE < 64, "vmcnt range");
    constexpr int kWaitRing = vmcnt_imm((NS - 2) * PER_STAGE), kWaitAll = vmcnt_imm(0);
    const int nk = (K + BK - 1) / BK;
    auto stage_step = [&](int kt, int u) __attribute__((always_inline)) {
        // stage kt's loads (issued NS-1 stages ago) must have landed; the NS-2
        // younger stages may still be in flight
        if (kt + NS - 2 < nk) __builtin_amdgcn_s_waitcnt(kWaitRing);
        else __builtin_amdgcn_s_waitcnt(kWaitAll);
        // Every wave's loads for stage kt landed; stage kt-1 fully read (its
        // fragments fed MFMAs already issued).  A bare barrier: the release
        // fence of __syncthreads would also wait for the younger stages'
        // loads that the ring keeps in flight.  The clobber keeps the compiler
        // from moving LDS accesses across it.
        asm volatile("s_barrier" ::: "memory");
        if (kt + NS - 1 < nk) issue(bufs((u + NS - 1) % NS), (kt + NS - 1) * BK);
        compute(bufs(u));
    };
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(bufs(s), s * BK);
    // whole groups of NS stages, then the remainder; no early exits, so the
    // accumulators keep a single home through the loop
    int kt0 = 0;
    for (; kt0 + NS <= nk; kt0 += NS) {
#pragma unroll
        for (int u = 0; u < NS; ++u) stage_step(kt0 + u, u);
    }
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
        if (kt0 + u < nk) stage_step(kt0 + u, u);

    // Epilogue through the (now idle) stage buffers.
    constexpr int ROWS_PER_BUF = G::STAGE / staging_pitch<CIL>();
    static_assert(G::STAGE % staging_pitch<CIL>() == 0, "staged rows stay inside one buffer");
    static_assert(ROWS_PER_BUF * NS >= staging_rows<WM, CIL>(), "stage buffers hold a staging round");
    auto row_ptr = [&](int row) __attribute__((always_inline)) -> char * {  // select chain: no dynamically indexed array
        constexpr int NB = (staging_rows<WM, CIL>() + ROWS_PER_BUF - 1) / ROWS_PER_BUF;  // buffers in use
        const int b = row / ROWS_PER_BUF;
        char *base = lds0;
        if (NB > 1 && b == 1) base = lds1;
        if (NB > 2 && b == 2) base = lds2;
        if (NB > 3 && b == 3) base = lds3;
        if (NB > 4 && b == 4) base = lds4;
        if (NB > 5 && b == 5) base = lds5;
        return base + (row % ROWS_PER_BUF) * staging_pitch<CIL>();
    };
    store_tile_staged<WM, CIL>(acc, row_ptr, C + (int64_t)c * 2 * M * N, M, N, m0, n0, wave, lane);
}

template <int WM, int BK, int NS, int CIL, int AB, int BF = 0>
__global__ __launch_bounds__(128 * WM, WM == 2 ? 2 : 1) void cgemm_f16_fast_kernel(
    const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, float *__restrict__ C,
    int M, int N, int K, int64_t a_stride, int tiles_m, int tiles_n, int nblocks) {
    TCBF_FAST_LDS(WM, BK, NS)
    const int t = (int)xcd_remap(blockIdx.x, nblocks);
    const int per_c = tiles_m * tiles_n;
    const int c = t / per_c;
    const int rem = t - c * per_c;
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    fast_tile<WM, BK, NS, CIL, AB, BF>(A, B, C, M, N, K, a_stride, c, tm, tn, lds0, lds1, lds2, lds3, lds4, lds5);
}

// ===========================================================================
// Split-ring variant: separate rings for the two operands.
// ===========================================================================
//
// Same tile, waves, fragments and MFMA sequence as the fast kernel with 32
// receivers per stage, but W and X stage through rings of their own: W two
// stages deep, X three, in five 16 KiB buffers (80 KiB: still two workgroups
// per CU).  X, the operand that comes from HBM on a batched radio-astronomy
// shape (W is re-read from L2 by every sample tile of its channel), is issued
// two stages ahead, W one.  At stage kt the wave issues W(kt+1) and then
// X(kt+2); loads retire in order, so waiting until only the newest X stage is
// in flight means W(kt) and X(kt) have landed while X(kt+1) may still come.
#define TCBF_SPLIT_LDS                                                             \
    __shared__ __attribute__((aligned(1024))) char wb0[FastGeo<2, 32>::WREG];      \
    __shared__ __attribute__((aligned(1024))) char wb1[FastGeo<2, 32>::WREG];      \
    __shared__ __attribute__((aligned(1024))) char xb0[FastGeo<2, 32>::XREG];      \
    __shared__ __attribute__((aligned(1024))) char xb1[FastGeo<2, 32>::XREG];      \
    __shared__ __attribute__((aligned(1024))) char xb2[FastGeo<2, 32>::XREG];

template <int CIL, int AB>
__device__ __forceinline__ void split_tile(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                           float *__restrict__ C, int M, int N, int K, int64_t a_stride, int c,
                                           int tm, int tn, char *wb0, char *wb1, char *xb0, char *xb1, char *xb2) {
    constexpr int WM = 2, BK = 32;
    typedef FastGeo<WM, BK> G;
    constexpr int TM = G::TM, NW = G::NW;
    static_assert(G::WREG == G::XREG, "equal operand regions");
    // select chains, not arrays (see fast_tile)
    auto wbs = [&](int i) __attribute__((always_inline)) -> char * { return i == 1 ? wb1 : wb0; };
    auto xbs = [&](int i) __attribute__((always_inline)) -> char * {
        char *b = xb0;
        if (i == 1) b = xb1;
        if (i == 2) b = xb2;
        return b;
    };

    const int tid = threadIdx.x;
    const int m0 = tm * TM, n0 = tn * BN;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    const int KW = AB ? (K + 31) / 32 * 32 : K;
    const uint16_t *Wc = A + (int64_t)c * a_stride;
    const uint16_t *Xc = B + (int64_t)c * 2 * K * N;
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc((void *)Wc, 0, 4 * M * KW, RSRC_FLAGS);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, 0, 4 * K * N, RSRC_FLAGS);

    // per-lane chunks, as in the fast kernel (X slots counted from the X
    // region's own start)
    constexpr int WPIECES = G::WREG / 1024, XPIECES = G::XREG / 1024;
    constexpr int WPW = WPIECES / NW, XPW = XPIECES / NW;
    constexpr int WROWS = 64 / G::WCH, XROWS = 64 / 16;
    uint32_t va, vb;
    int ka, kb, am;
    {
        const int s = wave * WPW * 64 + lane;
        const int p = s / (TM * G::WCH), m = (s / G::WCH) % TM;
        const int ch = (s % G::WCH) ^ G::swzW(m);
        ka = ch * 8;
        am = m;
        va = AB ? (uint32_t)(((p * (KW / 32)) * M + m0 + m) * 64 + ch * 16)
                : (uint32_t)(((p * M + m0 + m) * K + ch * 8) * 2);
    }
    {
        const int s = wave * XPW * 64 + lane;
        const int p = s / (BK * 16), k = (s / 16) % BK, ch = (s & 15) ^ G::swzX(k);
        kb = k;
        vb = (n0 + ch * 8 < N) ? (uint32_t)(((p * K + k) * N + n0 + ch * 8) * 2) : OOB;
    }
    const bool rows_full = m0 + TM <= M;

    constexpr int KS = BK / 16;
    int ow[KS], ox[2];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int m = wm * 64 + l32;
        ow[s] = m * (BK * 2) + (((2 * s + hl) ^ G::swzW(m)) * 16);
    }
    {
        const int g = lane >> 4, j16 = lane & 15;
        const int krow = 8 * (g >> 1) + (j16 >> 2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ns = wn * 64 + 32 * j + 16 * (g & 1) + 4 * (j16 & 3);
            ox[j] = krow * 256 + (((ns >> 3) ^ G::swzX(krow)) * 16) + (ns & 7) * 2;
        }
    }

    const int nk = (K + BK - 1) / BK;
    // Stages past the last one are issued all the same with every offset out
    // of range (the loads write zeros into a buffer no stage reads again), so
    // the sequence of loads, and with it every wait count, is the same on
    // every path; the compiler then needs no conservative full waits.
    auto issue_w = [&](char *base, int kt) __attribute__((always_inline)) {
        const int k0 = kt * BK;
        const bool tail = k0 + BK > K;
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            uint32_t off = va;
            if (!rows_full && m0 + am + q * WROWS >= M) off = OOB;
            if (tail && k0 + ka >= K) off = OOB;   // also every lane of a stage past the last
            const int so = kt >= nk ? 0
                           : AB   ? (k0 / 32) * M * 64 + q * WROWS * 64
                                  : k0 * 2 + q * WROWS * K * 2;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (LDS_AS void *)(base + (wave * WPW + q) * 1024), 16, off,
                                                     so, 0, 0);
        }
    };
    auto issue_x = [&](char *base, int kt) __attribute__((always_inline)) {
        const int k0 = kt * BK;
        const bool tail = k0 + BK > K;
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            uint32_t off = vb;
            if (tail && k0 + kb + q * XROWS >= K) off = OOB;   // also every lane of a stage past the last
            // (a stage past the last: no uniform offset, so OOB + offset cannot wrap into range)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LDS_AS void *)(base + (wave * XPW + q) * 1024), 16, off,
                                                     kt < nk ? (k0 + q * XROWS) * N * 2 : 0, 0, 0);
        }
    };

    Acc acc;
    acc.zero();
    auto compute = [&](const char *wst, const char *xst) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            half8 wr[2], wi[2], xr[2], xi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                wr[i] = *reinterpret_cast<const half8 *>(wst + ow[s] + i * 32 * BK * 2);
                wi[i] = *reinterpret_cast<const half8 *>(wst + ow[s] + i * 32 * BK * 2 + TM * BK * 2);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int o = ox[j] + s * 16 * 256;
                xr[j] = tr_frag(xst, o, o + 4 * 256);
                xi[j] = tr_frag(xst, o + BK * BN * 2, o + BK * BN * 2 + 4 * 256);
            }
            mma_step(acc, wr, wi, xr, xi);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    static_assert(XPW < 64, "vmcnt range");
    constexpr int kWaitNewestX = vmcnt_imm(XPW), kWaitAll = vmcnt_imm(0);
    // stage kt: W in wbs[kt % 2], X in xbs[kt % 3]
    auto stage_step = [&](int kt, int uw, int ux) __attribute__((always_inline)) {
        // W(kt) and X(kt) landed; X(kt+1), issued last, may be in flight
        __builtin_amdgcn_s_waitcnt(kWaitNewestX);
        // every wave's loads landed and stage kt-1 fully read (bare barrier:
        // the release fence of __syncthreads would wait for X(kt+1) too)
        asm volatile("s_barrier" ::: "memory");
        issue_w(wbs((uw + 1) % 2), kt + 1);
        issue_x(xbs((ux + 2) % 3), kt + 2);
        compute(wbs(uw), xbs(ux));
    };
    // prologue, in the order of the steady state: X(0), then W(0), X(1)
    issue_x(xbs(0), 0);
    issue_w(wbs(0), 0);
    issue_x(xbs(1), 1);
    // groups of 6 stages keep both rings' buffer choices compile-time
    int kt0 = 0;
    for (; kt0 + 6 <= nk; kt0 += 6) {
#pragma unroll
        for (int u = 0; u < 6; ++u) stage_step(kt0 + u, u % 2, u % 3);
    }
#pragma unroll
    for (int u = 0; u < 5; ++u)
        if (kt0 + u < nk) stage_step(kt0 + u, u % 2, u % 3);

    // epilogue through the idle buffers (four of the five: 64 KiB), once the
    // zero-filling loads past the last stage have landed
    __builtin_amdgcn_s_waitcnt(kWaitAll);
    constexpr int ROWS_PER_BUF = G::WREG / staging_pitch<CIL>();
    static_assert(ROWS_PER_BUF * 4 >= staging_rows<WM, CIL>(), "four buffers hold a staging round");
    auto row_ptr = [&](int row) __attribute__((always_inline)) -> char * {
        const int b = row / ROWS_PER_BUF;
        char *base = wb0;
        if (b == 1) base = wb1;
        if (b == 2) base = xb0;
        if (b == 3) base = xb1;
        return base + (row % ROWS_PER_BUF) * staging_pitch<CIL>();
    };
    store_tile_staged<WM, CIL>(acc, row_ptr, C + (int64_t)c * 2 * M * N, M, N, m0, n0, wave, lane);
}

template <int CIL, int AB>
__global__ __launch_bounds__(256, 2) void cgemm_f16_split_kernel(const uint16_t *__restrict__ A,
                                                                 const uint16_t *__restrict__ B,
                                                                 float *__restrict__ C, int M, int N, int K,
                                                                 int64_t a_stride, int tiles_m, int tiles_n,
                                                                 int nblocks) {
    TCBF_SPLIT_LDS
    const int t = (int)xcd_remap(blockIdx.x, nblocks);
    const int per_c = tiles_m * tiles_n;
    const int c = t / per_c;
    const int rem = t - c * per_c;
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    split_tile<CIL, AB>(A, B, C, M, N, K, a_stride, c, tm, tn, wb0, wb1, xb0, xb1, xb2);
}

// ===========================================================================
// Ping-pong persistent kernel (variant 9).
// ===========================================================================
//
// One 512-thread workgroup per CU runs output tiles of 256 beams x 128
// samples, 32 receivers per stage, through a ring of three 48 KiB stages.
// All eight waves share each staged W and X tile (every wave owns 64 x 64
// complex outputs), so per receiver a CU moves 4 (256 + 128) bytes into LDS
// for 256 x 128 outputs, against 2 x 4 (128 + 128) for two 128 x 128 tiles.
//
// Waves w and w + 4 share a SIMD.  Waves 0-3 (group 0) and 4-7 (group 1) run
// the same program, group 1 one barrier phase behind group 0.  The program
// alternates two phases, each ended by a workgroup barrier:
//   data phase of stage s: issue this wave's share of the global->LDS loads
//     of stage s + 2, read its MFMA fragments of stage s from LDS into
//     registers, wait for its own loads of stage s + 1, and, when a tile
//     ended with stage s - 1, store that tile straight from the accumulators;
//   matrix phase of stage s: 32 matrix instructions on registers only.
// So while one wave of a SIMD is in its matrix phase the other is in its data
// phase, and the matrix pipe gets one wave's instructions back to back.
//
// Why the barriers suffice (phase p = the interval between two consecutive
// barriers; group 0 runs the data phase of stage s in phase 2s + 1, group 1
// in phase 2s + 2):
//  * stage s's fragments are read after every wave waited for its own loads
//    of stage s (in its data phase of stage s - 1, phase 2s - 1 or 2s) and
//    then passed a barrier;
//  * stage s + 2 goes into the buffer of stage s - 1, whose last readers (the
//    data phases of stage s - 1, phases 2s - 1 and 2s, which end by waiting
//    for their LDS reads) are behind a barrier when the loads are issued.
// Both groups pass the same number of barriers (one extra at the start for
// group 1, one at the end for group 0).
//
// The workgroup walks a static list of tiles (round i: tile i * grid +
// its position, with the positions of one XCD consecutive), and the stage
// sequence runs on across tiles: a tile's first loads are issued while the
// previous tile is still being multiplied.  The matrix instructions take W
// as the first operand, so a register of the accumulators holds two runs of
// 32 consecutive samples (128 bytes of fp32 each) of two beams, and the tile
// is stored from the registers in whole lines with no LDS staging.

// One 16-receiver step with W as the first matrix operand (same products and
// the same order per accumulator as mma_step: Re gets Wr.Xr, then (-Wi).Xi;
// Im gets Wr.Xi, then Wi.Xr).  Element r of lane l of a 32 x 32 sub-tile
// holds sample l%32 of beam 8*(r/4) + 4*(l/32) + r%4.
template <int BF = 0>
__device__ __forceinline__ void mma_step_wx(Acc &a, const half8 (&wr)[2], const half8 (&wi)[2],
                                            const half8 (&xr)[2], const half8 (&xi)[2]) {
    half8 wn[2] = {negate(wi[0]), negate(wi[1])};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            a.re[i][j] = mfma16<BF>(wr[i], xr[j], a.re[i][j]);
            a.im[i][j] = mfma16<BF>(wr[i], xi[j], a.im[i][j]);
            a.re[i][j] = mfma16<BF>(wn[i], xi[j], a.re[i][j]);
            a.im[i][j] = mfma16<BF>(wi[i], xr[j], a.im[i][j]);
        }
}

// Store a wave's 64 x 64 block (beams mw.., samples nw.. of channel output
// Cc) from accumulators laid out as mma_step_wx leaves them.  Planar: one
// 4-byte store per register and plane, each writing two 128-byte row runs;
// interleaved: one 8-byte (re, im) store per register pair, two 256-byte
// runs.  Beams past M and samples past N are dropped by the range check.
template <int CIL>
__device__ __forceinline__ void store_block_wx(const Acc &acc, float *Cc, int M, int N, int mw, int nw,
                                               int lane) {
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)Cc, 0, 8 * M * N, RSRC_FLAGS);
    const int hl = lane >> 5, l32 = lane & 31;
    const bool whole = mw + 64 <= M && nw + 64 <= N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = nw + 32 * j + l32;
            const int mb = mw + 32 * i + 4 * hl;
            const bool n_ok = n < N;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = mb + 8 * (r >> 2) + (r & 3);
                const bool ok = whole || (n_ok && m < M);
                const float re = acc.re[i][j][r], im = acc.im[i][j][r];
                if (CIL) {
                    const uint32_t off = ok ? (uint32_t)((m * N + n) * 8) : OOB;
                    const u32x2 v = {__builtin_bit_cast(uint32_t, re), __builtin_bit_cast(uint32_t, im)};
                    __builtin_amdgcn_raw_buffer_store_b64(v, rc, off, 0, kStoreStreaming);
                } else {
                    const uint32_t off = ok ? (uint32_t)((m * N + n) * 4) : OOB;
                    const uint32_t offi = ok ? (uint32_t)(((M + m) * N + n) * 4) : OOB;
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, re), rc, off, 0,
                                                          kStoreStreaming);
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, im), rc, offi, 0,
                                                          kStoreStreaming);
                }
            }
        }
}

__device__ __forceinline__ void pp_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Interleaved data (X as [K][N][2], BIL = 1).  A stage's X tile is 32 rows
// of 128 complex samples = 256 real columns (512 bytes: re, im, re, im, ...)
// in LDS, read with the same transposing fragment reads as a plane of 256
// "samples"; a fragment then holds 32 real columns, re and im alternating
// with the lane (real column 2n + p in lane parity p).  The complex product
// stays the same four real products in the same order per output: for
// weights-first matrix instructions the real column is the output row, so
//   out[2n]     += Wr . Xr[n]  then  Wi . (-Xi[n])     (Re)
//   out[2n + 1] += Wr . Xi[n]  then  Wi . Xr[n]        (Im)
// i.e. one product with the fragment as read and one with a fragment whose
// adjacent lanes are exchanged and whose even lanes are negated (DPP quad
// permute plus a sign flip: exact).  Every output gets the same two exact
// products in the same order as from planar data, so results are bitwise
// identical; the accumulator row of an element is its real column, so the
// tile stores as rows of 2 x 64 floats per wave.
__device__ __forceinline__ half8 swap_negate_even(half8 v, uint32_t sign) {
    u32x4 u = __builtin_bit_cast(u32x4, v);
    u32x4 w;
    w.x = (uint32_t)__builtin_amdgcn_mov_dpp((int)u.x, 0xB1, 0xF, 0xF, false) ^ sign;  // quad_perm [1, 0, 3, 2]
    w.y = (uint32_t)__builtin_amdgcn_mov_dpp((int)u.y, 0xB1, 0xF, 0xF, false) ^ sign;
    w.z = (uint32_t)__builtin_amdgcn_mov_dpp((int)u.z, 0xB1, 0xF, 0xF, false) ^ sign;
    w.w = (uint32_t)__builtin_amdgcn_mov_dpp((int)u.w, 0xB1, 0xF, 0xF, false) ^ sign;
    return __builtin_bit_cast(half8, w);
}

// One 16-receiver step on interleaved data: a[i][j] rows are the real
// columns 32 j .. 32 j + 31 of the wave's 128.
__device__ __forceinline__ void mma_step_wx_il(f32x16 (&a)[2][4], const half8 (&wr)[2], const half8 (&wi)[2],
                                               const half8 (&x)[4], uint32_t sign) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const half8 y = swap_negate_even(x[j], sign);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wr[i], x[j], a[i][j], 0, 0, 0);
            a[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wi[i], y, a[i][j], 0, 0, 0);
        }
    }
}

// Store a wave's 64 beams x 128 real columns (64 samples from sample nw)
// from accumulators laid out as mma_step_wx_il leaves them, one 4-byte store
// per register, each writing two whole 128-byte row runs.  Interleaved output:
// the registers as they are.  Planar output: a register holds Re and Im of
// 16 samples in alternating lanes (a store of it would write half lines,
// measured 14 times slower), so the two registers of the same beam rows in
// fragments j and j + 1 (samples 16 j .. 16 j + 31) are regrouped across
// lanes first (ds_bpermute, no LDS memory): lane t then holds Re, and in a
// second register Im, of sample 16 j + t.
template <int CIL>
__device__ __forceinline__ void store_block_wx_il(const f32x16 (&a)[2][4], float *Cc, int M, int N, int mw, int nw,
                                                  int lane) {
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)Cc, 0, 8 * M * N, RSRC_FLAGS);
    const int hl = lane >> 5, l32 = lane & 31;
    const bool whole = mw + 64 <= M && nw + 64 <= N;
    if constexpr (!CIL) {
        // source lanes (byte addresses for ds_bpermute) of Re and Im of sample t % 16
        const int src_re = ((lane & 32) + 2 * (l32 & 15)) * 4, src_im = src_re + 4;
        const bool upper = l32 >= 16;  // samples 16..31 of the pair come from fragment j + 1
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int jp = 2 * q;
                const int n = nw + 16 * jp + l32;
                const bool n_ok = n < N;
                const int mb = mw + 32 * i + 4 * hl;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float f0 = a[i][jp][r], f1 = a[i][jp + 1][r];  // through scalars (see below)
                    const int v0 = __builtin_bit_cast(int, f0), v1 = __builtin_bit_cast(int, f1);
                    const int re0 = __builtin_amdgcn_ds_bpermute(src_re, v0), re1 = __builtin_amdgcn_ds_bpermute(src_re, v1);
                    const int im0 = __builtin_amdgcn_ds_bpermute(src_im, v0), im1 = __builtin_amdgcn_ds_bpermute(src_im, v1);
                    const int m = mb + 8 * (r >> 2) + (r & 3);
                    const bool ok = whole || (n_ok && m < M);
                    const uint32_t off = ok ? (uint32_t)((m * N + n) * 4) : OOB;
                    const uint32_t offi = ok ? (uint32_t)(((M + m) * N + n) * 4) : OOB;
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(upper ? re1 : re0), rc, off, 0, kStoreStreaming);
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(upper ? im1 : im0), rc, offi, 0, kStoreStreaming);
                }
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 2 * nw + 32 * j + l32;  // real column of this lane
            const bool n_ok = (c >> 1) < N;
            const int mb = mw + 32 * i + 4 * hl;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = mb + 8 * (r >> 2) + (r & 3);
                const bool ok = whole || (n_ok && m < M);
                const uint32_t off = ok ? (uint32_t)((m * 2 * N + c) * 4) : OOB;
                const float v = a[i][j][r];  // through a scalar: a bit cast of a vector element reads element 0
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rc, off, 0, kStoreStreaming);
            }
        }
}

template <int CIL, int AB, int BIL, int BF = 0>
__global__ __launch_bounds__(512, 1) void cgemm_f16_pp_kernel(const uint16_t *__restrict__ A,
                                                              const uint16_t *__restrict__ B,
                                                              float *__restrict__ C, int M, int N, int K,
                                                              int64_t a_stride, int tiles_m, int tiles_n,
                                                              int total_tiles) {
    static_assert(!(BIL && BF), "interleaved data: fp16 products only");
    typedef FastGeo<4, 32> G;
    constexpr int TM = G::TM, NW = G::NW;
    __shared__ __attribute__((aligned(1024))) char lds0[G::STAGE];
    __shared__ __attribute__((aligned(1024))) char lds1[G::STAGE];
    __shared__ __attribute__((aligned(1024))) char lds2[G::STAGE];

    const int grid = (int)gridDim.x;
    // Tile order.  With a grid that is a multiple of the 8 XCDs (workgroup b
    // runs on XCD b mod 8), each XCD takes a contiguous eighth of the tile
    // sequence and its workgroups step through it together, so the tiles in
    // flight on one XCD (one L2) are neighbours: a channel's weights stay in
    // that L2 while all its tiles pass.  Otherwise workgroup b takes tiles b,
    // b + grid, ...  Workgroup tiles: first, first + stride, ... (ntiles).
    int first, stride, ntiles;
    if (grid % 8 == 0) {
        const int xcd = (int)blockIdx.x % 8, j = (int)blockIdx.x / 8, per = grid / 8;
        const int q = total_tiles / 8, rem = total_tiles % 8;
        const int count = q + (xcd < rem ? 1 : 0);  // >= per: grid <= total_tiles
        first = xcd * q + min(xcd, rem) + j;
        stride = per;
        ntiles = (count - j + per - 1) / per;
    } else {
        first = (int)blockIdx.x;
        stride = grid;
        ntiles = (total_tiles - first + grid - 1) / grid;  // >= 1: grid <= total_tiles
    }
    const int nk = (K + 31) / 32;
    const int S = ntiles * nk;  // stages this workgroup runs
    const int per_c = tiles_m * tiles_n;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1, grp = wave >> 2;
    const int hl = lane >> 5, l32 = lane & 31;
    const int KW = AB ? (K + 31) / 32 * 32 : K;

    // This lane's 16-byte chunks of a stage (the fast kernel's assignment);
    // the tile's first beam goes into the uniform offset.
    constexpr int WPW = G::WREG / 1024 / NW, XPW = G::XREG / 1024 / NW;  // 4 and 2
    constexpr int WROWS = 64 / G::WCH, XROWS = 64 / 16;
    constexpr int PER_STAGE = WPW + XPW;
    uint32_t va, vb0;
    int ka, kb, am, xch;
    {
        const int s = wave * WPW * 64 + lane;
        const int p = s / (TM * G::WCH), m = (s / G::WCH) % TM;
        const int ch = (s % G::WCH) ^ G::swzW(m);
        ka = ch * 8;
        am = m;
        va = AB ? (uint32_t)(((p * (KW / 32)) * M + m) * 64 + ch * 16) : (uint32_t)(((p * M + m) * K + ch * 8) * 2);
    }
    // interleaved data: piece q of this wave is rows 2 (wave XPW + q) and +1
    // (512 bytes each, 32 chunks of 4 complex samples); the chunk swizzle
    // follows the row, so each piece has its own lane offset
    uint32_t vbi[XPW];
    int xchi[XPW];
    if constexpr (!BIL) {
        const int s = wave * XPW * 64 + lane;
        const int p = s / (32 * 16), k = (s / 16) % 32, ch = (s & 15) ^ G::swzX(k);
        kb = k;
        xch = ch;
        vb0 = (uint32_t)(((p * K + k) * N + ch * 8) * 2);
    } else {
        kb = 2 * wave * XPW + hl;  // row of piece 0
        xch = 0;
        vb0 = 0;
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            const int k = kb + 2 * q;
            xchi[q] = l32 ^ G::swzX(k);
            vbi[q] = (uint32_t)((k * N + 4 * xchi[q]) * 4);
        }
    }
    // fragment offsets in a stage (plane 0), as in the fast kernel with TM = 256
    int ow[2], ox[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int m = wm * 64 + l32;
        ow[s] = m * 64 + (((2 * s + hl) ^ G::swzW(m)) * 16);
    }
    int oxi[4];  // interleaved data: 4 fragments of 32 real columns, rows of 512 bytes
    {
        const int g = lane >> 4, j16 = lane & 15;
        const int krow = 8 * (g >> 1) + (j16 >> 2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ns = wn * 64 + 32 * j + 16 * (g & 1) + 4 * (j16 & 3);
            ox[j] = G::WREG + krow * 256 + (((ns >> 3) ^ G::swzX(krow)) * 16) + (ns & 7) * 2;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cs = wn * 128 + 32 * j + 16 * (g & 1) + 4 * (j16 & 3);
            oxi[j] = G::WREG + krow * 512 + (((cs >> 3) ^ G::swzX(krow)) * 16) + (cs & 7) * 2;
        }
    }
    const uint32_t neg_even = (lane & 1) ? 0u : 0x80008000u;  // sign flip of both halves in even lanes

    auto tile_of = [&](int round, int &c, int &m0, int &n0) __attribute__((always_inline)) {
        const int t = first + round * stride;
        c = t / per_c;
        int tm, tn;
        tile_coords(t - c * per_c, tiles_m, tiles_n, tm, tn);
        m0 = tm * TM;
        n0 = tn * BN;
    };

    // load cursor: the tile and stage the next issue() loads
    int l_round = 0, l_kt = 0, l_m0 = 0, l_wso = 0;
    bool l_live = true, l_rows_full = true;
    uint32_t l_vb = OOB;
    uint32_t l_vbi[XPW];
#pragma unroll
    for (int q = 0; q < XPW; ++q) l_vbi[q] = OOB;
    __amdgpu_buffer_rsrc_t rw, rx;
    auto load_tile = [&]() __attribute__((always_inline)) {
        l_live = l_round < ntiles;
        if (l_live) {
            int c, m0, n0;
            tile_of(l_round, c, m0, n0);
            const uint16_t *Wc = A + (int64_t)c * a_stride;
            const uint16_t *Xc = B + (int64_t)c * 2 * K * N;
            rw = __builtin_amdgcn_make_buffer_rsrc((void *)Wc, 0, 4 * M * KW, RSRC_FLAGS);
            rx = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, 0, 4 * K * N, RSRC_FLAGS);
            l_m0 = m0;
            l_rows_full = m0 + TM <= M;
            l_wso = AB ? m0 * 64 : m0 * K * 2;
            l_vb = (n0 + xch * 8 < N) ? vb0 + (uint32_t)(n0 * 2) : OOB;
            if constexpr (BIL) {
#pragma unroll
                for (int q = 0; q < XPW; ++q) l_vbi[q] = (n0 + 4 * xchi[q] < N) ? vbi[q] + (uint32_t)(n0 * 4) : OOB;
            }
        }
    };
    // Issue this wave's loads of the cursor's stage into `base` and advance.
    // Stages past the last are issued too, with every offset out of range
    // (zero fills of buffers nobody reads again), so every wait count is the
    // same on every path.
    auto issue = [&](char *base) __attribute__((always_inline)) {
        const int k0 = l_kt * 32;
        const bool tail = k0 + 32 > K;
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            uint32_t off = va;
            if (!l_rows_full && l_m0 + am + q * WROWS >= M) off = OOB;  // beams past M
            if (tail && k0 + ka >= K) off = OOB;                         // receivers past K
            if (!l_live) off = OOB;
            const int so = !l_live ? 0 : l_wso + (AB ? (k0 / 32) * M * 64 + q * WROWS * 64 : k0 * 2 + q * WROWS * K * 2);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (LDS_AS void *)(base + (wave * WPW + q) * 1024), 16, off, so,
                                                     0, 0);
        }
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            uint32_t off = BIL ? l_vbi[q] : l_vb;
            const int krow = BIL ? kb + 2 * q : kb + q * XROWS;
            if (tail && k0 + krow >= K) off = OOB;  // receivers past K
            if (!l_live) off = OOB;
            const int so = !l_live ? 0 : BIL ? k0 * N * 4 : (k0 + q * XROWS) * N * 2;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LDS_AS void *)(base + G::WREG + (wave * XPW + q) * 1024),
                                                     16, off, so, 0, 0);
        }
        if (++l_kt == nk) {
            l_kt = 0;
            ++l_round;
            load_tile();
        }
    };

    half8 wr[2][2], wi[2][2], xr[2][2], xi[2][2];  // [step][sub-tile]
    half8 xc[2][4];                                 // interleaved data: [step][32 real columns]
    auto read_frags = [&](const char *st) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                wr[s][i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * 64);
                wi[s][i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * 64 + TM * 64);
            }
            if constexpr (BIL) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = oxi[j] + s * 16 * 512;
                    xc[s][j] = tr_frag(st, o, o + 4 * 512);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int o = ox[j] + s * 16 * 256;
                    xr[s][j] = tr_frag(st, o, o + 4 * 256);
                    xi[s][j] = tr_frag(st, o + 32 * BN * 2, o + 32 * BN * 2 + 4 * 256);
                }
            }
        }
    };

    Acc acc;  // planar data; interleaved data keeps its rows (real columns) in ail
    f32x16 ail[2][4];
    auto acc_zero = [&]() __attribute__((always_inline)) {
        if constexpr (BIL) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) ail[i][j] = (f32x16){};
        } else {
            acc.zero();
        }
    };
    acc_zero();
    int c_round = 0, c_kt = 0;  // compute cursor
    auto store_round = [&](int round) __attribute__((always_inline)) {
        int c, m0, n0;
        tile_of(round, c, m0, n0);
        if constexpr (BIL)
            store_block_wx_il<CIL>(ail, C + (int64_t)c * 2 * M * N, M, N, m0 + wm * 64, n0 + wn * 64, lane);
        else
            store_block_wx<CIL>(acc, C + (int64_t)c * 2 * M * N, M, N, m0 + wm * 64, n0 + wn * 64, lane);
    };
    constexpr int kWaitNext = vmcnt_imm(PER_STAGE), kWaitAll = vmcnt_imm(0);
    auto step = [&](char *rd, char *ld) __attribute__((always_inline)) {
        // data phase
        issue(ld);
        read_frags(rd);
        __builtin_amdgcn_s_waitcnt(kWaitNext);  // own loads of the next stage landed
        if (c_kt == 0 && c_round > 0) {         // the previous stage ended a tile
            store_round(c_round - 1);
            acc_zero();
        }
        __builtin_amdgcn_s_waitcnt(kWaitLds);
        pp_barrier();
        // matrix phase
        if constexpr (BIL) {
            mma_step_wx_il(ail, wr[0], wi[0], xc[0], neg_even);
            mma_step_wx_il(ail, wr[1], wi[1], xc[1], neg_even);
        } else {
            mma_step_wx<BF>(acc, wr[0], wi[0], xr[0], xi[0]);
            mma_step_wx<BF>(acc, wr[1], wi[1], xr[1], xi[1]);
        }
        if (++c_kt == nk) {
            c_kt = 0;
            ++c_round;
        }
        pp_barrier();
    };

    load_tile();
    issue(lds0);
    issue(lds1);
    __builtin_amdgcn_s_waitcnt(kWaitNext);  // own loads of stage 0 landed
    pp_barrier();
    if (grp == 1) pp_barrier();
    // stage s reads buffer s % 3 and loads stage s + 2 into buffer (s + 2) % 3;
    // whole groups of three stages, then the remainder (no early exit, so the
    // accumulators keep a single home through the loop)
    int s = 0;
    for (; s + 3 <= S; s += 3) {
        step(lds0, lds2);
        step(lds1, lds0);
        step(lds2, lds1);
    }
    if (s < S) step(lds0, lds2);
    if (s + 1 < S) step(lds1, lds0);
    store_round(c_round - 1);
    if (grp == 0) pp_barrier();
    __builtin_amdgcn_s_waitcnt(kWaitAll);
}

// ===========================================================================
// Grouped persistent kernel: many problems of different shapes in one launch.
// ===========================================================================
//
// The problems' tiles form one list (problem by problem, each in the order of
// the plain kernel); a workgroup takes the next tile index from a device
// counter, finds its problem among the problem table's first-tile offsets,
// runs the same tile code as the fast kernel (128 x 128, 32 receivers per
// stage, 2-deep ring; planar or receiver-blocked W, one layout per launch)
// and asks again until the list is exhausted.  The table
// travels in the kernel arguments, so a captured graph replays it unchanged.
struct GroupProblem {
    const uint16_t *A;
    const uint16_t *B;
    float *C;
    int M, N, K, a_shared;
    int tiles_m, tiles_n;  // per channel
    int first_tile;        // index of this problem's first tile in the list
    int pad;
};
struct GroupArgs {
    GroupProblem p[TCBF_GROUP_MAX];
    int count, total_tiles;
};

template <int CIL, int AB>
__global__ __launch_bounds__(256, 2) void cgemm_f16_group_kernel(const GroupArgs args,
                                                                 unsigned int *__restrict__ counter) {
    TCBF_FAST_LDS(2, 32, 2)
    __shared__ int next_tile;
    for (;;) {
        if (threadIdx.x == 0) next_tile = (int)atomicAdd(counter, 1u);
        // the index is visible, and every wave has finished the previous
        // tile's LDS use before the next tile's loads land in the ring
        lds_barrier();
        const int t = __builtin_amdgcn_readfirstlane(next_tile);
        if (t >= args.total_tiles) break;
        int pi = 0;
        for (int i = 1; i < args.count; ++i)
            if (t >= args.p[i].first_tile) pi = i;
        const GroupProblem &q = args.p[pi];
        const int local = t - q.first_tile;
        const int per_c = q.tiles_m * q.tiles_n;
        const int c = local / per_c;
        const int rem = local - c * per_c;
        int tm, tn;
        tile_coords(rem, q.tiles_m, q.tiles_n, tm, tn);
        const int64_t a_stride = q.a_shared ? 0 : 2 * (int64_t)q.M * (AB ? (q.K + 31) / 32 * 32 : q.K);
        fast_tile<2, 32, 2, CIL, AB>(q.A, q.B, q.C, q.M, q.N, q.K, a_stride, c, tm, tn, lds0, lds1, lds2, lds3,
                                     lds4, lds5);
        // next_tile is rewritten only after the tile's own barriers, which
        // every wave passes after reading it
    }
}

// Grouped form of the ping-pong kernel: the tiles (256 beams x 128 samples)
// of several problems form one list, longest receiver count first, and
// workgroup `pos` runs tiles pos, pos + grid, ... (a static list: the stage
// sequence runs on across tiles, so each workgroup must know its next tile
// two stages ahead).  The loop is the ping-pong kernel's, with the problem
// of the load cursor's tile and of the compute cursor's tile looked up in
// the table when each cursor moves on; the per-lane load offsets, which
// depend on the problem's sizes, are recomputed then.  Same fragments, same
// matrix instructions in the same order: every problem's output equals its
// plan's bit for bit.  Planar X.
struct PpGroupProblem {
    const uint16_t *A;
    const uint16_t *B;
    float *C;
    int M, N, K, a_shared;
    int tiles_m, tiles_n;  // 256 x 128 tiles per channel
    int first_tile;
    int nk;  // 32-receiver stages per tile
};
struct PpGroupArgs {
    PpGroupProblem p[TCBF_GROUP_MAX];
    int count, total_tiles;
};

template <int CIL, int AB>
__global__ __launch_bounds__(512, 1) void cgemm_f16_pp_group_kernel(const PpGroupArgs args) {
    typedef FastGeo<4, 32> G;
    constexpr int TM = G::TM, NW = G::NW;
    __shared__ __attribute__((aligned(1024))) char lds0[G::STAGE];
    __shared__ __attribute__((aligned(1024))) char lds1[G::STAGE];
    __shared__ __attribute__((aligned(1024))) char lds2[G::STAGE];

    const int grid = (int)gridDim.x;
    const int pos = (int)xcd_remap(blockIdx.x, grid);
    const int total = args.total_tiles;
    const int ntiles = (total - pos + grid - 1) / grid;  // >= 1: grid <= total

    auto problem_of = [&](int t) __attribute__((always_inline)) {
        int pi = 0;
        for (int i = 1; i < args.count; ++i)
            if (t >= args.p[i].first_tile) pi = i;
        return pi;
    };
    // stages this workgroup runs
    int S = 0;
    for (int r = 0; r < ntiles; ++r) S += args.p[problem_of(r * grid + pos)].nk;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1, grp = wave >> 2;
    const int hl = lane >> 5;

    // this lane's chunk coordinates in a stage (problem-independent); the
    // byte offsets follow from the problem's sizes
    constexpr int WPW = G::WREG / 1024 / NW, XPW = G::XREG / 1024 / NW;
    constexpr int WROWS = 64 / G::WCH, XROWS = 64 / 16;
    constexpr int PER_STAGE = WPW + XPW;
    int wp, wrow, wch, xp, xk, xch;
    {
        const int s = wave * WPW * 64 + lane;
        wp = s / (TM * G::WCH);
        wrow = (s / G::WCH) % TM;
        wch = (s % G::WCH) ^ G::swzW(wrow);
    }
    {
        const int s = wave * XPW * 64 + lane;
        xp = s / (32 * 16);
        xk = (s / 16) % 32;
        xch = (s & 15) ^ G::swzX(xk);
    }
    int ow[2], ox[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int m = wm * 64 + (lane & 31);
        ow[s] = m * 64 + (((2 * s + hl) ^ G::swzW(m)) * 16);
    }
    {
        const int g = lane >> 4, j16 = lane & 15;
        const int krow = 8 * (g >> 1) + (j16 >> 2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ns = wn * 64 + 32 * j + 16 * (g & 1) + 4 * (j16 & 3);
            ox[j] = G::WREG + krow * 256 + (((ns >> 3) ^ G::swzX(krow)) * 16) + (ns & 7) * 2;
        }
    }

    auto tile_of = [&](int round, int &pi, int &c, int &m0, int &n0) __attribute__((always_inline)) {
        const int t = round * grid + pos;
        pi = problem_of(t);
        const PpGroupProblem &q = args.p[pi];
        const int local = t - q.first_tile, per_c = q.tiles_m * q.tiles_n;
        c = local / per_c;
        int tm, tn;
        tile_coords(local - c * per_c, q.tiles_m, q.tiles_n, tm, tn);
        m0 = tm * TM;
        n0 = tn * BN;
    };

    // load cursor
    int l_round = 0, l_kt = 0, l_m0 = 0, l_wso = 0, l_M = 0, l_N = 0, l_K = 0, l_nk = 1;
    bool l_live = true, l_rows_full = true;
    uint32_t l_va = OOB, l_vb = OOB;
    __amdgpu_buffer_rsrc_t rw, rx;
    auto load_tile = [&]() __attribute__((always_inline)) {
        l_live = l_round < ntiles;
        if (l_live) {
            int pi, c, m0, n0;
            tile_of(l_round, pi, c, m0, n0);
            const PpGroupProblem &q = args.p[pi];
            l_M = q.M;
            l_N = q.N;
            l_K = q.K;
            l_nk = q.nk;
            const int KW = AB ? (l_K + 31) / 32 * 32 : l_K;
            const uint16_t *Wc = q.A + (q.a_shared ? (int64_t)0 : (int64_t)c * 2 * l_M * KW);
            const uint16_t *Xc = q.B + (int64_t)c * 2 * l_K * l_N;
            rw = __builtin_amdgcn_make_buffer_rsrc((void *)Wc, 0, 4 * l_M * KW, RSRC_FLAGS);
            rx = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, 0, 4 * l_K * l_N, RSRC_FLAGS);
            l_m0 = m0;
            l_rows_full = m0 + TM <= l_M;
            l_wso = AB ? m0 * 64 : m0 * l_K * 2;
            l_va = AB ? (uint32_t)(((wp * (KW / 32)) * l_M + wrow) * 64 + wch * 16)
                      : (uint32_t)(((wp * l_M + wrow) * l_K + wch * 8) * 2);
            l_vb = (n0 + xch * 8 < l_N) ? (uint32_t)(((xp * l_K + xk) * l_N + n0 + xch * 8) * 2) : OOB;
        }
    };
    auto issue = [&](char *base) __attribute__((always_inline)) {
        const int k0 = l_kt * 32;
        const bool tail = k0 + 32 > l_K;
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            uint32_t off = l_va;
            if (!l_rows_full && l_m0 + wrow + q * WROWS >= l_M) off = OOB;
            if (tail && k0 + wch * 8 >= l_K) off = OOB;
            if (!l_live) off = OOB;
            const int so = !l_live ? 0
                                   : l_wso + (AB ? (k0 / 32) * l_M * 64 + q * WROWS * 64 : k0 * 2 + q * WROWS * l_K * 2);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (LDS_AS void *)(base + (wave * WPW + q) * 1024), 16, off, so,
                                                     0, 0);
        }
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            uint32_t off = l_vb;
            if (tail && k0 + xk + q * XROWS >= l_K) off = OOB;
            if (!l_live) off = OOB;
            const int so = !l_live ? 0 : (k0 + q * XROWS) * l_N * 2;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LDS_AS void *)(base + G::WREG + (wave * XPW + q) * 1024),
                                                     16, off, so, 0, 0);
        }
        if (++l_kt == l_nk) {
            l_kt = 0;
            ++l_round;
            load_tile();
        }
    };

    half8 wr[2][2], wi[2][2], xr[2][2], xi[2][2];
    auto read_frags = [&](const char *st) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                wr[s][i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * 64);
                wi[s][i] = *reinterpret_cast<const half8 *>(st + ow[s] + i * 32 * 64 + TM * 64);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int o = ox[j] + s * 16 * 256;
                xr[s][j] = tr_frag(st, o, o + 4 * 256);
                xi[s][j] = tr_frag(st, o + 32 * BN * 2, o + 32 * BN * 2 + 4 * 256);
            }
        }
    };

    Acc acc;
    acc.zero();
    // compute cursor: its tile's stage count, and where its output goes
    int c_round = 0, c_kt = 0, c_nk = 1;
    auto compute_tile = [&]() __attribute__((always_inline)) {
        if (c_round < ntiles) {
            int pi, c, m0, n0;
            tile_of(c_round, pi, c, m0, n0);
            c_nk = args.p[pi].nk;
        }
    };
    auto store_round = [&](int round) __attribute__((always_inline)) {
        int pi, c, m0, n0;
        tile_of(round, pi, c, m0, n0);
        const PpGroupProblem &q = args.p[pi];
        store_block_wx<CIL>(acc, q.C + (int64_t)c * 2 * q.M * q.N, q.M, q.N, m0 + wm * 64, n0 + wn * 64, lane);
    };
    constexpr int kWaitNext = vmcnt_imm(PER_STAGE), kWaitAll = vmcnt_imm(0);
    auto step = [&](char *rd, char *ld) __attribute__((always_inline)) {
        issue(ld);
        read_frags(rd);
        __builtin_amdgcn_s_waitcnt(kWaitNext);
        if (c_kt == 0 && c_round > 0) {
            store_round(c_round - 1);
            acc.zero();
        }
        __builtin_amdgcn_s_waitcnt(kWaitLds);
        pp_barrier();
        mma_step_wx(acc, wr[0], wi[0], xr[0], xi[0]);
        mma_step_wx(acc, wr[1], wi[1], xr[1], xi[1]);
        if (++c_kt == c_nk) {
            c_kt = 0;
            ++c_round;
            compute_tile();
        }
        pp_barrier();
    };

    load_tile();
    compute_tile();
    issue(lds0);
    issue(lds1);
    __builtin_amdgcn_s_waitcnt(kWaitNext);
    pp_barrier();
    if (grp == 1) pp_barrier();
    int s = 0;
    for (; s + 3 <= S; s += 3) {
        step(lds0, lds2);
        step(lds1, lds0);
        step(lds2, lds1);
    }
    if (s < S) step(lds0, lds2);
    if (s + 1 < S) step(lds1, lds0);
    store_round(c_round - 1);
    if (grp == 0) pp_barrier();
    __builtin_amdgcn_s_waitcnt(kWaitAll);
}

__global__ void group_reset_kernel(unsigned int *counter) { *counter = 0u; }

typedef void (*KernFn)(const uint16_t *, const uint16_t *, float *, int64_t, int64_t, int64_t, int64_t,
                       int, int, int64_t, int, int);
typedef void (*FastFn)(const uint16_t *, const uint16_t *, float *, int, int, int, int64_t, int, int, int);

// bil: 0 planar, 1 interleaved, 2 planar receiver-contiguous, 3 interleaved
// receiver-contiguous; bf: bfloat16 operands
template <int BF> KernFn pick_of(int ail, int bil, int cil) {
    static const KernFn table[16] = {
        cgemm_f16_kernel<0, 0, 0, BF>, cgemm_f16_kernel<0, 0, 1, BF>, cgemm_f16_kernel<0, 1, 0, BF>,
        cgemm_f16_kernel<0, 1, 1, BF>, cgemm_f16_kernel<0, 2, 0, BF>, cgemm_f16_kernel<0, 2, 1, BF>,
        cgemm_f16_kernel<0, 3, 0, BF>, cgemm_f16_kernel<0, 3, 1, BF>, cgemm_f16_kernel<1, 0, 0, BF>,
        cgemm_f16_kernel<1, 0, 1, BF>, cgemm_f16_kernel<1, 1, 0, BF>, cgemm_f16_kernel<1, 1, 1, BF>,
        cgemm_f16_kernel<1, 2, 0, BF>, cgemm_f16_kernel<1, 2, 1, BF>, cgemm_f16_kernel<1, 3, 0, BF>,
        cgemm_f16_kernel<1, 3, 1, BF>,
    };
    return table[(ail << 3) | (bil << 1) | cil];
}
KernFn pick(int ail, int bil, int cil, bool bf) { return bf ? pick_of<1>(ail, bil, cil) : pick_of<0>(ail, bil, cil); }

// Fast-kernel configurations (variant: beam waves WM, receivers per stage,
// ring depth):  2: 2, 32, 2   3: 2, 16, 4   4: 2, 16, 5   5: 2, 32, 3
//               6: 4, 32, 3   7: 4, 16, 6   8: 2, 32, split (W 2, X 3)
//               9: 4, 32, 3 ping-pong persistent
// WM = 2 runs two 256-thread workgroups per CU; WM = 4 one 512-thread
// workgroup with a 256 x 128 tile.
constexpr int kFirstFast = 2;
constexpr int kNumFast = 8;
constexpr int kDefaultFast = 2;
constexpr int kPingPong = 9;

struct FastShape {
    int wm, bk;
};
FastShape fast_shape(int v) {
    switch (v) {
    case 2: return {2, 32};
    case 3: case 4: return {2, 16};
    case 5: return {2, 32};
    case 6: case 9: return {4, 32};
    case 8: return {2, 32};
    default: return {4, 16};
    }
}

template <int AB> FastFn fast_fn_of(int v, bool cil) {
    switch (v) {
    case 2: return cil ? cgemm_f16_fast_kernel<2, 32, 2, 1, AB> : cgemm_f16_fast_kernel<2, 32, 2, 0, AB>;
    case 5: return cil ? cgemm_f16_fast_kernel<2, 32, 3, 1, AB> : cgemm_f16_fast_kernel<2, 32, 3, 0, AB>;
    case 6: return cil ? cgemm_f16_fast_kernel<4, 32, 3, 1, AB> : cgemm_f16_fast_kernel<4, 32, 3, 0, AB>;
    case 8: return cil ? cgemm_f16_split_kernel<1, AB> : cgemm_f16_split_kernel<0, AB>;
    }
    return nullptr;
}

FastFn fast_fn(int v, bool cil, bool ab) {
    if (ab) return fast_fn_of<1>(v, cil);
    switch (v) {
    case 3: return cil ? cgemm_f16_fast_kernel<2, 16, 4, 1, 0> : cgemm_f16_fast_kernel<2, 16, 4, 0, 0>;
    case 4: return cil ? cgemm_f16_fast_kernel<2, 16, 5, 1, 0> : cgemm_f16_fast_kernel<2, 16, 5, 0, 0>;
    case 7: return cil ? cgemm_f16_fast_kernel<4, 16, 6, 1, 0> : cgemm_f16_fast_kernel<4, 16, 6, 0, 0>;
    }
    return fast_fn_of<0>(v, cil);
}

}  // namespace

// Variant 1: generic kernel.  Variants 2..: fast kernel (planar X, N a
// multiple of 8; planar W with K a multiple of 8, or blocked W with any K;
// every per-channel operand and output below 2 GiB so 32-bit buffer offsets
// reach it).  Blocked W: only the fast kernel, variants with 32 receivers per
// stage (2, 5, 6, 8).
static bool fast_ok(const Problem &p) {
    const int64_t lim = (int64_t)1 << 31;
    const bool ab = p.a_layout == TCBF_BLOCKED;
    const int64_t kw = ab ? (p.K + 31) / 32 * 32 : p.K;
    return (ab || (p.a_layout == TCBF_PLANAR && p.K % 8 == 0)) && p.b_layout == TCBF_PLANAR && !p.b_kmajor &&
           p.N % 8 == 0 &&
           4 * p.M * kw < lim && 4 * p.K * p.N < lim && 8 * p.M * p.N < lim && p.M < lim && p.N < lim &&
           p.batch * ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN) < lim;
}

static bool reads_blocked(int v) { return v == 2 || v == 5 || v == 6 || v == 8 || v == 9; }

// The ping-pong kernel also reads interleaved data (X as [K][N][2]): the
// fast kernels' conditions with X planar or interleaved.
static bool pp_ok(const Problem &p) {
    if (p.b_layout != TCBF_INTERLEAVED) return fast_ok(p);
    Problem q = p;
    q.b_layout = TCBF_PLANAR;
    return fast_ok(q);
}

// Compute units of `device` (the persistent kernels run one workgroup on
// each); 256, the MI355X's count, when the runtime cannot say (no device).
int device_cus(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        (void)hipGetLastError();   // a planning query: leave no error for the caller's next check
        return 256;
    }
    return n > 0 ? n : 256;
}

// Default choice: the persistent ping-pong kernel once the problem has at
// least a 256 x 128 tile for every compute unit (it runs one workgroup per
// CU and measured 4-13% faster than variant 2 on such shapes) and a tile
// runs at least 2 stages of 32 receivers; variant 2 for smaller problems and
// for one-stage tiles (there the ping-pong kernel's end-of-tile stores
// dominate, while variant 2's second workgroup on the CU multiplies during
// them: 256 x 1024 x 1024 x K, K = 8..32, 4-9% faster with inputs streamed
// from memory; from K = 48 the ping-pong kernel is 7-19% faster so), the
// generic kernel where the fast ones do not apply.
static int default_variant_f16(const Problem &p) {
    if (p.b_kmajor) return 1;  // receiver-contiguous X: the generic kernel
    const int64_t tiles = p.batch * ((p.M + 255) / 256) * ((p.N + BN - 1) / BN);
    const bool big = tiles >= device_cus(p.device) && tiles * ((p.K + 31) / 32) < ((int64_t)1 << 31);
    // interleaved data: the ping-pong kernel (also for fewer tiles than CUs
    // when W is receiver-blocked, which only the fast kernels read)
    if (p.b_layout == TCBF_INTERLEAVED)
        return pp_ok(p) && tiles * ((p.K + 31) / 32) < ((int64_t)1 << 31) && (big || p.a_layout == TCBF_BLOCKED)
                   ? kPingPong
                   : 1;
    if (!fast_ok(p)) return 1;
    const bool deep = (p.K + 31) / 32 >= 2;  // stages per tile
    return big && deep ? kPingPong : kDefaultFast;
}

// bfloat16 operands run in variants 1, 2 and 9 (planar X for 9).
static bool bf16_variant(const Problem &p, int v) {
    return v == 1 || v == 2 || (v == kPingPong && p.b_layout == TCBF_PLANAR);
}

static int default_variant(const Problem &p) {
    const int v = default_variant_f16(p);
    return !p.bf16 || bf16_variant(p, v) ? v : 1;
}

bool f16_select(const Problem &p, int forced_variant, F16Config *cfg) {
    const bool ab = p.a_layout == TCBF_BLOCKED;
    int v = forced_variant;
    if (v == 0) v = default_variant(p);
    if (v < 1 || v >= kFirstFast + kNumFast) return false;
    if (p.bf16 && !bf16_variant(p, v)) return false;
    if (v >= kFirstFast && !(v == kPingPong ? pp_ok(p) : fast_ok(p))) return false;
    if (ab && !reads_blocked(v)) return false;
    if (v == kPingPong) {
        // the persistent kernel counts a workgroup's stages in 32 bits
        const int64_t tiles = p.batch * ((p.M + 255) / 256) * ((p.N + BN - 1) / BN);
        if (tiles * ((p.K + 31) / 32) >= ((int64_t)1 << 31)) return false;
    }
    cfg->variant = v;
    cfg->tile_m = v >= kFirstFast ? 64 * fast_shape(v).wm : BM;
    cfg->tile_n = BN;
    cfg->tile_k = v >= kFirstFast ? fast_shape(v).bk : BK;
    cfg->threads = v >= kFirstFast ? 128 * fast_shape(v).wm : NT;
    // 16-byte loads need every row start 16-byte aligned (base pointers are
    // required to be 16-byte aligned by the ABI).
    cfg->a_vec = p.a_layout == TCBF_PLANAR ? (p.K % 8 == 0) : (p.K % 4 == 0);
    // (receiver-contiguous X: rows of K samples' receivers, like W's)
    const int64_t xrow = p.b_kmajor ? p.K : p.N;
    cfg->b_vec = p.b_layout == TCBF_PLANAR ? (xrow % 8 == 0) : (xrow % 4 == 0);
    return true;
}

int64_t f16_workgroups(const Problem &p, const F16Config &cfg) {
    int64_t tm = (p.M + cfg.tile_m - 1) / cfg.tile_m;
    int64_t tn = (p.N + cfg.tile_n - 1) / cfg.tile_n;
    return p.batch * tm * tn;
}

const char *f16_kernel_name(const F16Config &cfg) {
    if (cfg.variant == 8) return "cgemm_f16_split_kernel";
    if (cfg.variant == kPingPong) return "cgemm_f16_pp_kernel";
    return cfg.variant >= kFirstFast ? "cgemm_f16_fast_kernel" : "cgemm_f16_kernel";
}

hipError_t f16_launch(const Problem &p, const F16Config &cfg, const void *A, const void *B,
                      void *C, hipStream_t stream) {
    int tiles_m = (int)((p.M + cfg.tile_m - 1) / cfg.tile_m);
    int tiles_n = (int)((p.N + BN - 1) / BN);
    int64_t nblocks = p.batch * tiles_m * tiles_n;
    if (cfg.variant == kPingPong) {
        const bool ab = p.a_layout == TCBF_BLOCKED, cil = p.c_layout == TCBF_INTERLEAVED;
        static const FastFn pp[8] = {cgemm_f16_pp_kernel<0, 0, 0>, cgemm_f16_pp_kernel<0, 0, 1>,
                                     cgemm_f16_pp_kernel<0, 1, 0>, cgemm_f16_pp_kernel<0, 1, 1>,
                                     cgemm_f16_pp_kernel<1, 0, 0>, cgemm_f16_pp_kernel<1, 0, 1>,
                                     cgemm_f16_pp_kernel<1, 1, 0>, cgemm_f16_pp_kernel<1, 1, 1>};
        static const FastFn pp_bf[4] = {cgemm_f16_pp_kernel<0, 0, 0, 1>, cgemm_f16_pp_kernel<0, 1, 0, 1>,
                                        cgemm_f16_pp_kernel<1, 0, 0, 1>, cgemm_f16_pp_kernel<1, 1, 0, 1>};
        const FastFn fn = p.bf16 ? pp_bf[(cil << 1) | ab] : pp[(cil << 2) | (ab << 1) | (p.b_layout == TCBF_INTERLEAVED)];
        const int grid = (int)std::min<int64_t>(nblocks, device_cus(p.device));
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(cfg.threads), 0, stream, (const uint16_t *)A,
                           (const uint16_t *)B, (float *)C, (int)p.M, (int)p.N, (int)p.K, p.a_stride, tiles_m,
                           tiles_n, (int)nblocks);
        return hipGetLastError();
    }
    if (cfg.variant >= kFirstFast) {
        const bool cil = p.c_layout == TCBF_INTERLEAVED, ab = p.a_layout == TCBF_BLOCKED;
        static const FastFn v2_bf[4] = {cgemm_f16_fast_kernel<2, 32, 2, 0, 0, 1>, cgemm_f16_fast_kernel<2, 32, 2, 0, 1, 1>,
                                        cgemm_f16_fast_kernel<2, 32, 2, 1, 0, 1>, cgemm_f16_fast_kernel<2, 32, 2, 1, 1, 1>};
        FastFn fn = p.bf16 ? v2_bf[(cil << 1) | ab] : fast_fn(cfg.variant, cil, ab);
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(cfg.threads), 0, stream, (const uint16_t *)A,
                           (const uint16_t *)B, (float *)C, (int)p.M, (int)p.N, (int)p.K, p.a_stride,
                           tiles_m, tiles_n, (int)nblocks);
        return hipGetLastError();
    }
    KernFn fn = pick(p.a_layout == TCBF_INTERLEAVED, (p.b_layout == TCBF_INTERLEAVED) + 2 * (p.b_kmajor != 0),
                     p.c_layout == TCBF_INTERLEAVED, p.bf16 != 0);
    hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(NT), 0, stream,
                       (const uint16_t *)A, (const uint16_t *)B, (float *)C, p.M, p.N, p.K,
                       p.a_stride, tiles_m, tiles_n, nblocks, (int)cfg.a_vec, (int)cfg.b_vec);
    return hipGetLastError();
}

bool f16_group_problem_ok(const Problem &p) { return fast_ok(p); }

int64_t f16_group_tiles(const Problem &p) { return p.batch * ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN); }

bool f16_group_pp(int variant) { return variant == 6 || variant == 7 || variant == kPingPong; }

hipError_t f16_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                            const int *order, const int *variants, int count, int c_layout, int cus,
                            unsigned int *counter, hipStream_t stream) {
    // one operand layout per launch (the API checks it)
    const bool ab = probs[order[0]].a_layout == TCBF_BLOCKED, cil = c_layout == TCBF_INTERLEAVED;
    GroupArgs args;
    PpGroupArgs pargs;
    memset(&args, 0, sizeof(args));
    memset(&pargs, 0, sizeof(pargs));
    int64_t first = 0, pfirst = 0;
    int n = 0, pn = 0;
    for (int j = 0; j < count; ++j) {
        const int i = order[j];
        const Problem &p = probs[i];
        if (f16_group_pp(variants[i])) {
            PpGroupProblem &q = pargs.p[pn++];
            q.A = (const uint16_t *)A[i];
            q.B = (const uint16_t *)B[i];
            q.C = (float *)C[i];
            q.M = (int)p.M;
            q.N = (int)p.N;
            q.K = (int)p.K;
            q.a_shared = p.a_shared;
            q.tiles_m = (int)((p.M + 255) / 256);
            q.tiles_n = (int)((p.N + BN - 1) / BN);
            q.first_tile = (int)pfirst;
            q.nk = (int)((p.K + 31) / 32);
            pfirst += p.batch * q.tiles_m * q.tiles_n;
        } else {
            GroupProblem &q = args.p[n++];
            q.A = (const uint16_t *)A[i];
            q.B = (const uint16_t *)B[i];
            q.C = (float *)C[i];
            q.M = (int)p.M;
            q.N = (int)p.N;
            q.K = (int)p.K;
            q.a_shared = p.a_shared;
            q.tiles_m = (int)((p.M + BM - 1) / BM);
            q.tiles_n = (int)((p.N + BN - 1) / BN);
            q.first_tile = (int)first;
            first += f16_group_tiles(p);
        }
    }
    if (n > 0) {
        args.count = n;
        args.total_tiles = (int)first;
        const int grid = (int)std::min<int64_t>(first, 2 * (int64_t)cus);
        hipLaunchKernelGGL(group_reset_kernel, dim3(1), dim3(1), 0, stream, counter);
        void (*fn)(const GroupArgs, unsigned int *) =
            ab ? (cil ? cgemm_f16_group_kernel<1, 1> : cgemm_f16_group_kernel<0, 1>)
               : (cil ? cgemm_f16_group_kernel<1, 0> : cgemm_f16_group_kernel<0, 0>);
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(NT), 0, stream, args, counter);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (pn > 0) {
        pargs.count = pn;
        pargs.total_tiles = (int)pfirst;
        const int grid = (int)std::min<int64_t>(pfirst, (int64_t)cus);
        void (*fn)(const PpGroupArgs) = ab ? (cil ? cgemm_f16_pp_group_kernel<1, 1> : cgemm_f16_pp_group_kernel<0, 1>)
                                           : (cil ? cgemm_f16_pp_group_kernel<1, 0> : cgemm_f16_pp_group_kernel<0, 0>);
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(512), 0, stream, pargs);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace tcbf
