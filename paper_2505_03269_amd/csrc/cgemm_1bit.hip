// 1-bit batched complex product (Sec. III-D) on gfx950.
//
// Inputs are packed sign bits (bit 1 = +1, bit 0 = -1 per component, Fig. 1),
// 32 samples along K per uint32, LSB first: W [c][2][M][kw], X [c][2][N][kw].
// Output is the exact int32 complex product.
//
// gfx950 has no binary matrix instruction, so two routes exist:
//
// Variant 1 (int8 MFMA).  Each packed word is expanded in registers to bytes
// in {0, 1} and fed to v_mfma_i32_32x32x32_i8.  With s = 2a - 1, t = 2b - 1 for
// bits a, b, every +-1 product is s t = 4ab - 2a - 2b + 1, so a sum over K
// needs the bit-products P = sum ab plus the row and column bit counts.  The
// kernel accumulates
//     Qr = sum (ar br + ai ~bi),      Qi = sum (ar bi + ai br)
// (~bi is the complemented bit, the 1-bit form of the negated Im(X) of
// Sec. III-B) and finishes with
//     Re = 4 Qr - 2 (Ar + Ai) - 2 Br + 2 Bi
//     Im = 4 Qi - 2 (Ar + Ai) - 2 (Br + Bi) + 2 K
// where Ar, Ai are W's row bit counts and Br, Bi X's column bit counts.
// Bits past K are masked to 0 on load; a zero bit of W contributes nothing to
// any product, so padding needs no further correction.
// The expansion uses a fixed permutation of K inside each word (byte j of
// dword d takes bit 8j + d), identical for W and X, which leaves every sum
// unchanged.
//
// Variant 2 (VALU).  XOR and popcount per word, the paper's own equations:
//     Re = 2 (Kp - (popc(Ar ^ Br) + popc(Ai ^ ~Bi)))
//     Im = 2 (Kp - Kpad - (popc(Ar ^ Bi) + popc(Ai ^ Br)))
// with Kp the number of bit positions processed and Kpad = Kp - K.
#include <cstring>

#include "tcbf_tile.h"

namespace tcbf {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t tail_mask(int64_t K, int64_t w) {
    int64_t valid = K - 32 * w;
    if (valid >= 32) return 0xffffffffu;
    if (valid <= 0) return 0u;
    return (1u << valid) - 1u;
}

// Load 4 consecutive words [w0, w0+4) of a row of kw words, masking past K.
__device__ __forceinline__ u32x4 load_words4(const uint32_t *row, int64_t w0, int64_t kw, int64_t K,
                                             bool ok, bool vec) {
    u32x4 r = (u32x4){0u, 0u, 0u, 0u};
    if (!ok) return r;
    if (vec && w0 + 4 <= kw) {
        r = *reinterpret_cast<const u32x4 *>(row + w0);
    } else {
        r.x = (w0 + 0 < kw) ? row[w0 + 0] : 0u;
        r.y = (w0 + 1 < kw) ? row[w0 + 1] : 0u;
        r.z = (w0 + 2 < kw) ? row[w0 + 2] : 0u;
        r.w = (w0 + 3 < kw) ? row[w0 + 3] : 0u;
    }
    if (32 * (w0 + 4) > K) {
        r.x &= tail_mask(K, w0 + 0);
        r.y &= tail_mask(K, w0 + 1);
        r.z &= tail_mask(K, w0 + 2);
        r.w &= tail_mask(K, w0 + 3);
    }
    return r;
}

__device__ __forceinline__ uint32_t wsel(const u32x4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// ---------------------------------------------------------------------------
// Variant 1: int8 MFMA.  256 threads, 128 x 128 complex outputs, 4 words
// (128 k) per stage, 2 x 2 waves of 64 x 64.
// ---------------------------------------------------------------------------
constexpr int U_BM = 128, U_BN = 128, U_BKW = 4, U_NT = 256;
constexpr int U_STAGE = 2 * U_BM * U_BKW + 2 * U_BN * U_BKW;  // words

// 16 bytes of {0,1}: byte j of dword d holds bit 8j + d of x (x already
// shifted so that this lane's 4 bit columns sit at d = 0..3).
__device__ __forceinline__ i32x4 expand(uint32_t x) {
    i32x4 v;
    v.x = (int)(x & 0x01010101u);
    v.y = (int)((x >> 1) & 0x01010101u);
    v.z = (int)((x >> 2) & 0x01010101u);
    v.w = (int)((x >> 3) & 0x01010101u);
    return v;
}

// One 128 x 128 output tile of channel c; lds holds the two stages,
// popA / popB the row bit counts of the tile's operands.
template <int CIL>
__device__ __forceinline__ void int1_tile(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B,
                                          int32_t *__restrict__ C, int64_t M, int64_t N, int64_t K, int64_t kw,
                                          int64_t a_stride, int64_t c, int tm, int tn, int vec, uint32_t *lds,
                                          int (*popA)[U_BM], int (*popB)[U_BN]) {
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)tm * U_BM, n0 = (int64_t)tn * U_BN;

    // loader: thread -> (plane, row) of both tiles; 4 words per stage each
    const int lplane = tid >> 7, lrow = tid & 127;
    const int64_t am = m0 + lrow, bn = n0 + lrow;
    const bool aok = am < M, bok = bn < N;
    const uint32_t *arow = A + c * a_stride + (int64_t)lplane * M * kw + (aok ? am : 0) * kw;
    const uint32_t *brow = B + c * 2 * N * kw + (int64_t)lplane * N * kw + (bok ? bn : 0) * kw;
    int pa = 0, pb = 0;

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    i32x16 acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc_r[i][j] = (i32x16){};
            acc_i[i][j] = (i32x16){};
        }

    const int nk = (int)((kw + U_BKW - 1) / U_BKW);
    u32x4 ra = load_words4(arow, 0, kw, K, aok, vec);
    u32x4 rb = load_words4(brow, 0, kw, K, bok, vec);
    // LDS stage: A planes [2][128][4], then B planes [2][128][4]
    *reinterpret_cast<u32x4 *>(lds + (lplane * U_BM + lrow) * U_BKW) = ra;
    *reinterpret_cast<u32x4 *>(lds + 2 * U_BM * U_BKW + (lplane * U_BN + lrow) * U_BKW) = rb;
    pa += __builtin_popcount(ra.x) + __builtin_popcount(ra.y) + __builtin_popcount(ra.z) + __builtin_popcount(ra.w);
    pb += __builtin_popcount(rb.x) + __builtin_popcount(rb.y) + __builtin_popcount(rb.z) + __builtin_popcount(rb.w);
    __syncthreads();

    const int sh = 4 * hl;
    for (int kt = 0; kt < nk; ++kt) {
        const uint32_t *st = lds + (kt & 1) * U_STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            ra = load_words4(arow, (int64_t)(kt + 1) * U_BKW, kw, K, aok, vec);
            rb = load_words4(brow, (int64_t)(kt + 1) * U_BKW, kw, K, bok, vec);
        }
        u32x4 war[2], wai[2], wbr[2], wbi[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            int row = wm * 64 + i * 32 + l32;
            war[i] = *reinterpret_cast<const u32x4 *>(st + (0 * U_BM + row) * U_BKW);
            wai[i] = *reinterpret_cast<const u32x4 *>(st + (1 * U_BM + row) * U_BKW);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            int col = wn * 64 + j * 32 + l32;
            wbr[j] = *reinterpret_cast<const u32x4 *>(st + 2 * U_BM * U_BKW + (0 * U_BN + col) * U_BKW);
            wbi[j] = *reinterpret_cast<const u32x4 *>(st + 2 * U_BM * U_BKW + (1 * U_BN + col) * U_BKW);
        }
#pragma unroll
        for (int w = 0; w < U_BKW; ++w) {
            i32x4 xar[2], xai[2], xbr[2], xbi[2], xbn[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                xar[i] = expand(wsel(war[i], w) >> sh);
                xai[i] = expand(wsel(wai[i], w) >> sh);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                xbr[j] = expand(wsel(wbr[j], w) >> sh);
                xbi[j] = expand(wsel(wbi[j], w) >> sh);
                xbn[j] = xbi[j] ^ 0x01010101;  // complemented bits of Im(X)
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc_r[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xar[i], xbr[j], acc_r[i][j], 0, 0, 0);
                    acc_i[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xar[i], xbi[j], acc_i[i][j], 0, 0, 0);
                    acc_r[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xai[i], xbn[j], acc_r[i][j], 0, 0, 0);
                    acc_i[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xai[i], xbr[j], acc_i[i][j], 0, 0, 0);
                }
        }
        if (more) {
            uint32_t *nx = lds + ((kt + 1) & 1) * U_STAGE;
            *reinterpret_cast<u32x4 *>(nx + (lplane * U_BM + lrow) * U_BKW) = ra;
            *reinterpret_cast<u32x4 *>(nx + 2 * U_BM * U_BKW + (lplane * U_BN + lrow) * U_BKW) = rb;
            pa += __builtin_popcount(ra.x) + __builtin_popcount(ra.y) + __builtin_popcount(ra.z) + __builtin_popcount(ra.w);
            pb += __builtin_popcount(rb.x) + __builtin_popcount(rb.y) + __builtin_popcount(rb.z) + __builtin_popcount(rb.w);
        }
        __syncthreads();
    }
    popA[lplane][lrow] = pa;
    popB[lplane][lrow] = pb;
    __syncthreads();

    const bool full = (m0 + U_BM <= M) && (n0 + U_BN <= N);
    const int K2 = (int)(2 * K);
    // the lane's row and column offsets, opaque to the compiler: in the
    // grouped persistent kernel it would otherwise hoist the 32 row offsets
    // below out of the tile loop and spill them
    int hl_e = hl, l32_e = l32;
    asm volatile("" : "+v"(hl_e), "+v"(l32_e));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lc = wn * 64 + j * 32 + l32_e;
            const int64_t col = n0 + lc;
            const int bsr = popB[0][lc], bsi = popB[1][lc];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int lr = wm * 64 + i * 32 + (r >> 2) * 8 + hl_e * 4 + (r & 3);
                const int64_t row = m0 + lr;
                if (full || (row < M && col < N)) {
                    const int asum = popA[0][lr] + popA[1][lr];
                    const int re = 4 * acc_r[i][j][r] - 2 * asum - 2 * bsr + 2 * bsi;
                    const int im = 4 * acc_i[i][j][r] - 2 * asum - 2 * (bsr + bsi) + K2;
                    if (CIL) {
                        *reinterpret_cast<int2 *>(C + ((c * M + row) * N + col) * 2) = make_int2(re, im);
                    } else {
                        int32_t *o = C + c * 2 * M * N + row * N + col;
                        o[0] = re;
                        o[M * N] = im;
                    }
                }
            }
        }
}

template <int CIL>
__global__ __launch_bounds__(U_NT, 2) void cgemm_1bit_mfma_kernel(
    const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, int32_t *__restrict__ C,
    int64_t M, int64_t N, int64_t K, int64_t kw, int64_t a_stride, int tiles_m, int tiles_n,
    int64_t nblocks, int vec) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[2 * U_STAGE];
    __shared__ int popA[2][U_BM], popB[2][U_BN];
    const int64_t t = xcd_remap(blockIdx.x, nblocks);
    const int64_t per_c = (int64_t)tiles_m * tiles_n;
    const int64_t c = t / per_c;
    const int rem = (int)(t - c * per_c);
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    int1_tile<CIL>(A, B, C, M, N, K, kw, a_stride, c, tm, tn, vec, lds, popA, popB);
}

// Grouped persistent launch of the int8-MFMA variant: problems of different
// shapes in one launch, tiles taken from a device counter, each problem's
// output equal to its own plan's.  The table travels in the kernel arguments.
struct Int1GroupProblem {
    const uint32_t *A;
    const uint32_t *B;
    int32_t *C;
    int M, N, K, kw;  // 2 M N < 2^31 and K <= 2^26 (the plan limits)
    int a_shared, vec;
    int tiles_m, tiles_n;  // per channel
    int first_tile;        // index of this problem's first tile in the list
    int pad;
};
struct Int1GroupArgs {
    Int1GroupProblem p[TCBF_GROUP_MAX];
    int count, total_tiles;
};

template <int CIL>
__global__ __launch_bounds__(U_NT, 2) void cgemm_1bit_group_kernel(const Int1GroupArgs args,
                                                                    unsigned int *__restrict__ counter) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[2 * U_STAGE];
    __shared__ int popA[2][U_BM], popB[2][U_BN];
    __shared__ int next_tile;
    for (;;) {
        if (threadIdx.x == 0) next_tile = (int)atomicAdd(counter, 1u);
        // the index is visible, and every wave has finished the previous
        // tile (its epilogue reads the bit counts) before the next one
        // overwrites the stages and counts
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(next_tile);
        if (t >= args.total_tiles) break;
        int pi = 0;
        for (int i = 1; i < args.count; ++i)
            if (t >= args.p[i].first_tile) pi = i;
        const Int1GroupProblem &q = args.p[pi];
        const int local = t - q.first_tile;
        const int per_c = q.tiles_m * q.tiles_n;
        const int c = local / per_c;
        const int rem = local - c * per_c;
        int tm, tn;
        tile_coords(rem, q.tiles_m, q.tiles_n, tm, tn);
        int1_tile<CIL>(q.A, q.B, q.C, q.M, q.N, q.K, q.kw, q.a_shared ? 0 : 2 * (int64_t)q.M * q.kw, c, tm, tn, q.vec, lds,
                       popA, popB);
        // next_tile is rewritten only after the tile's own barriers, which
        // every wave passes after reading it
    }
}

__global__ void int1_group_reset_kernel(unsigned int *counter) { *counter = 0u; }

// ---------------------------------------------------------------------------
// Variant 2: VALU xor/popcount.  256 threads, 64 x 64 complex outputs, each
// thread 4 x 4 outputs; 4 words per stage.
// ---------------------------------------------------------------------------
constexpr int V_BM = 64, V_BN = 64, V_BKW = 4, V_NT = 256;
constexpr int V_STAGE = 2 * V_BM * V_BKW + 2 * V_BN * V_BKW;

template <int CIL>
__global__ __launch_bounds__(V_NT, 2) void cgemm_1bit_valu_kernel(
    const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, int32_t *__restrict__ C,
    int64_t M, int64_t N, int64_t K, int64_t kw, int64_t a_stride, int tiles_m, int tiles_n,
    int64_t nblocks, int vec) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[2 * V_STAGE];

    const int tid = threadIdx.x;
    const int64_t t = xcd_remap(blockIdx.x, nblocks);
    const int64_t per_c = (int64_t)tiles_m * tiles_n;
    const int64_t c = t / per_c;
    const int rem = (int)(t - c * per_c);
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * V_BM, n0 = (int64_t)tn * V_BN;

    // loader: threads 0..127 -> W (plane, row), 128..255 -> X (plane, row)
    const bool isA = tid < 128;
    const int lt = tid & 127, lplane = lt >> 6, lrow = lt & 63;
    const int64_t lr = (isA ? m0 : n0) + lrow;
    const bool lok = lr < (isA ? M : N);
    const uint32_t *src = isA
        ? A + c * a_stride + (int64_t)lplane * M * kw + (lok ? lr : 0) * kw
        : B + c * 2 * N * kw + (int64_t)lplane * N * kw + (lok ? lr : 0) * kw;
    const int loff = (isA ? 0 : 2 * V_BM * V_BKW) + (lplane * 64 + lrow) * V_BKW;

    const int tx = tid & 15, ty = tid >> 4;  // outputs: rows ty + 16 a, cols tx + 16 b
    int sr[4][4], si[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { sr[a][b] = 0; si[a][b] = 0; }

    const int nk = (int)((kw + V_BKW - 1) / V_BKW);
    u32x4 rw = load_words4(src, 0, kw, K, lok, vec);
    *reinterpret_cast<u32x4 *>(lds + loff) = rw;
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const uint32_t *st = lds + (kt & 1) * V_STAGE;
        const bool more = kt + 1 < nk;
        if (more) rw = load_words4(src, (int64_t)(kt + 1) * V_BKW, kw, K, lok, vec);
        u32x4 ar[4], ai[4], br[4], bi[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ar[a] = *reinterpret_cast<const u32x4 *>(st + (0 * 64 + ty + 16 * a) * V_BKW);
            ai[a] = *reinterpret_cast<const u32x4 *>(st + (1 * 64 + ty + 16 * a) * V_BKW);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            br[b] = *reinterpret_cast<const u32x4 *>(st + 2 * V_BM * V_BKW + (0 * 64 + tx + 16 * b) * V_BKW);
            bi[b] = *reinterpret_cast<const u32x4 *>(st + 2 * V_BM * V_BKW + (1 * 64 + tx + 16 * b) * V_BKW);
        }
#pragma unroll
        for (int w = 0; w < V_BKW; ++w)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t xr = wsel(br[b], w), xi = wsel(bi[b], w), xn = ~xi;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const uint32_t wr = wsel(ar[a], w), wi = wsel(ai[a], w);
                    sr[a][b] += __builtin_popcount(wr ^ xr) + __builtin_popcount(wi ^ xn);
                    si[a][b] += __builtin_popcount(wr ^ xi) + __builtin_popcount(wi ^ xr);
                }
            }
        if (more) *reinterpret_cast<u32x4 *>(lds + ((kt + 1) & 1) * V_STAGE + loff) = rw;
        __syncthreads();
    }

    const int64_t Kp = (int64_t)nk * V_BKW * 32, Kpad = Kp - K;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t row = m0 + ty + 16 * a, col = n0 + tx + 16 * b;
            if (row < M && col < N) {
                const int re = (int)(2 * (Kp - sr[a][b]));
                const int im = (int)(2 * (Kp - Kpad - si[a][b]));
                if (CIL) {
                    *reinterpret_cast<int2 *>(C + ((c * M + row) * N + col) * 2) = make_int2(re, im);
                } else {
                    int32_t *o = C + c * 2 * M * N + row * N + col;
                    o[0] = re;
                    o[M * N] = im;
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Variant 3: e2m1 matrix instructions on the +-1 values themselves.
// ---------------------------------------------------------------------------
// Every sign bit becomes the 4-bit float +1 (code 0x2) or -1 (code 0xA), and
// v_mfma_scale_f32_32x32x64_f8f6f4 (e2m1 operands, unit scales) multiplies
// them with the complex product of Sec. III-B: Re += Wr.Xr + (-Wi).Xi,
// Im += Wr.Xi + Wi.Xr, -Wi by flipping the sign bit of every code.  Every
// partial sum is an integer of magnitude at most 2K, exact in the fp32
// accumulators while 2K <= 2^24, so the plan takes this variant for K <= 2^23
// only.  Bits of receivers past K are cleared in both operands, as the
// paper's padding does (Sec. III-D): each such receiver then adds
// (-1)(-1) + (-(-1))(-1) = 0 to Re and 2 to Im, and the epilogue takes
// 2 K_pad off Im (K_pad: receivers processed past K).  A word
// expands into four dwords of eight codes: code i of dword d is bit 4i + d of
// the word, the same fixed permutation of the word's 32 receivers for both
// operands, which leaves every sum unchanged.  The instruction takes 64
// receivers per lane pair: lanes 0-31 supply one word and lanes 32-63 another.
//
// Workgroup: 128 beams x 128 samples, 4 waves of 64 x 64, two workgroups per
// CU.  A stage holds 16 words (512 receivers) of every row of both operands
// (2 operands x 2 planes x 128 rows x 64 bytes = 32 KiB), moved with
// direct-to-LDS loads through a two-deep ring; the 16-byte chunks of a row sit
// XOR-swizzled by (row / 4) % 4, so the fragment reads (16 rows per phase)
// meet no bank conflicts.  Lane half h of a wave takes words 8h .. 8h + 7 of
// each staged row: step s of the stage contracts words s and 8 + s (any
// split works, as long as both operands use the same one).  The
// matrix instructions take W as the first operand, so the tile is stored
// straight from the accumulators in whole 128-byte row runs.
constexpr int F_BKW = 16;                // words per stage
constexpr int F_ROWB = F_BKW * 4;        // staged row bytes
constexpr int F_PLANE = U_BM * F_ROWB;   // 8 KiB
constexpr int F_STAGE = 4 * F_PLANE;     // W planes then X planes: 32 KiB
constexpr int F_MAX_K = 1 << 23;         // exact fp32 sums

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16v __attribute__((ext_vector_type(16)));

// Four dwords of e2m1 codes from one word: +1 (0x2) for a set bit, -1 (0xA)
// for a clear one; code i of dword d takes bit 4i + d.  Bit 3 of a code (the
// sign) is the complement of its sample bit, so each dword is
// (~(x << (3 - d)) & 0x88888888) | 0x22222222: one shift and one three-input
// bit operation (truth table 0xAE = (~a & b) | c, indexed by the bits
// (a, b, c) from the most significant).
__device__ __forceinline__ i32x8 e2m1_expand(uint32_t x) {
    constexpr uint32_t kSign = 0x88888888u, kOne = 0x22222222u;
    constexpr unsigned kNotAAndBOrC = 0xAE;
    i32x8 v;
    v[0] = (int)__builtin_amdgcn_bitop3_b32(x << 3, kSign, kOne, kNotAAndBOrC);
    v[1] = (int)__builtin_amdgcn_bitop3_b32(x << 2, kSign, kOne, kNotAAndBOrC);
    v[2] = (int)__builtin_amdgcn_bitop3_b32(x << 1, kSign, kOne, kNotAAndBOrC);
    v[3] = (int)__builtin_amdgcn_bitop3_b32(x, kSign, kOne, kNotAAndBOrC);
    v[4] = v[5] = v[6] = v[7] = 0;
    return v;
}

__device__ __forceinline__ i32x8 e2m1_negate(i32x8 v) {
#pragma unroll
    for (int d = 0; d < 4; ++d) v[d] ^= (int)0x88888888u;
    return v;
}

__device__ __forceinline__ f32x16v mma4(const i32x8 &a, const i32x8 &b, const f32x16v &c) {
    // format 4 = e2m1 for both operands, E8M0 scales 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

template <int CIL>
__global__ __launch_bounds__(U_NT, 2) void cgemm_1bit_fp4_kernel(const uint32_t *__restrict__ A,
                                                                 const uint32_t *__restrict__ B,
                                                                 int32_t *__restrict__ C, int M, int N, int K,
                                                                 int kw, int64_t a_stride, int tiles_m, int tiles_n,
                                                                 int nblocks) {
    __shared__ __attribute__((aligned(1024))) char lds0[F_STAGE];
    __shared__ __attribute__((aligned(1024))) char lds1[F_STAGE];
    const int t = (int)xcd_remap(blockIdx.x, nblocks);
    const int per_c = tiles_m * tiles_n;
    const int c = t / per_c;
    int tm, tn;
    tile_coords(t - c * per_c, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * U_BM, n0 = tn * U_BN;

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    // Loads: wave w moves the 8 KiB plane (w % 2) of operand (w / 2) in eight
    // 1 KiB pieces of 16 rows; lane l fills LDS slot l of a piece: row l / 4,
    // stored chunk l % 4, which holds global chunk (l % 4) ^ ((row / 4) % 4).
    const int op = wave >> 1, plane = wave & 1;
    const int rows = op ? N : M, r0 = op ? n0 : m0;
    const uint32_t *base = op ? B + (int64_t)c * 2 * N * kw : A + (int64_t)c * a_stride;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, 8 * rows * kw, tile::RSRC_FLAGS);
    const int lrow = lane >> 2;
    const int gch = (lane & 3) ^ ((lane >> 4) & 3);
    const uint32_t voff = (uint32_t)(((plane * rows + r0 + lrow) * kw + gch * 4) * 4);
    const int lds_piece0 = (op * 2 + plane) * F_PLANE;
    const int nk = (kw + F_BKW - 1) / F_BKW;
    // A stage past the last is issued too, all out of range (zeros into a
    // buffer nobody reads again): the code has no branch around the loads,
    // so nothing can be moved across the stage barriers.
    auto issue = [&](char *buf, int kt) __attribute__((always_inline)) {
        const int k0w = kt < nk ? kt * F_BKW : 0;
        const bool chunk_ok = kt < nk && k0w + gch * 4 < kw;  // kw % 4 == 0: a chunk is wholly in or out
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // per-lane range check in the lane offset; the uniform offset
            // (< 2^31, so OOB plus it cannot wrap into range) stays uniform
            const bool ok = chunk_ok && r0 + q * 16 + lrow < rows;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (TCBF_LDS_AS void *)(buf + lds_piece0 + q * 1024), 16,
                                                     ok ? voff : tile::OOB, (q * 16 * kw + k0w) * 4, 0, 0);
        }
    };

    // fragment offsets: row R of a plane, chunk (2h or 2h + 1) ^ ((R / 4) % 4)
    int fo[2][2][2];  // [operand][sub-tile][chunk]
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int R = (o ? wn : wm) * 64 + i * 32 + l32;
#pragma unroll
            for (int ch = 0; ch < 2; ++ch)
                fo[o][i][ch] = o * 2 * F_PLANE + R * F_ROWB + (((2 * hl + ch) ^ ((R >> 2) & 3)) * 16);
        }

    f32x16v acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc_r[i][j] = (f32x16v){};
            acc_i[i][j] = (f32x16v){};
        }

    auto compute = [&](const char *st, int kt) __attribute__((always_inline)) {
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            __builtin_amdgcn_sched_barrier(0);
            // this lane's words of steps 4ch .. 4ch + 3: [operand][sub-tile][plane]
            tile::u32x4 wd[2][2][2];
#pragma unroll
            for (int o = 0; o < 2; ++o)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int p = 0; p < 2; ++p)
                        wd[o][i][p] = *reinterpret_cast<const tile::u32x4 *>(st + fo[o][i][ch] + p * F_PLANE);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // bits of receivers past K cleared in both operands (their
                // -1 x -1 products are taken out of Im in the epilogue)
                const int valid = K - 32 * (kt * F_BKW + 8 * hl + 4 * ch + q);
                const uint32_t vm = valid >= 32 ? 0xffffffffu : valid <= 0 ? 0u : (1u << valid) - 1u;
                i32x8 ar[2], ai[2], br[2], bi[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    ar[i] = e2m1_expand(wd[0][i][0][q] & vm);
                    ai[i] = e2m1_expand(wd[0][i][1][q] & vm);
                    br[i] = e2m1_expand(wd[1][i][0][q] & vm);
                    bi[i] = e2m1_expand(wd[1][i][1][q] & vm);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc_r[i][j] = mma4(ar[i], br[j], acc_r[i][j]);
                        acc_i[i][j] = mma4(ar[i], bi[j], acc_i[i][j]);
                        acc_i[i][j] = mma4(ai[i], br[j], acc_i[i][j]);
                    }
                    ai[i] = e2m1_negate(ai[i]);  // -Wi
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc_r[i][j] = mma4(ai[i], bi[j], acc_r[i][j]);
                }
                // one step's operands live at a time (two workgroups per CU
                // leave 256 registers per lane)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    // two-deep ring: stage kt in buffer kt % 2, stage kt + 1 in flight
    constexpr int kWait0 = tile::vmcnt_imm(0);
    issue(lds0, 0);
    int kt = 0;
    auto step = [&](char *cur, char *nxt) __attribute__((always_inline)) {
        // this wave's loads of stage kt landed; then every wave's, and stage
        // kt - 1 fully read.  The scheduling barriers keep the previous
        // stage's matrix instructions from being moved past the wait.
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(kWait0);
        asm volatile("s_barrier" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        issue(nxt, kt + 1);
        compute(cur, kt);
        ++kt;
    };
    for (; kt + 2 <= nk;) {
        step(lds0, lds1);
        step(lds1, lds0);
    }
    if (kt < nk) step(lds0, lds1);

    // store from the accumulators: element r of lane l = sample l % 32 of
    // beam 8 (r / 4) + 4 (l / 32) + r % 4 of the 32 x 32 sub-tile
    __builtin_amdgcn_s_waitcnt(kWait0);  // the zero fills past the last stage landed
    // every processed receiver past K (cleared bits, -1 in both operands)
    // added (-1)(-1) + (-1)(-1) = 2 to Im and (-1)(-1) - (-1)(-1) = 0 to Re
    const int kpad2 = 2 * (nk * F_BKW * 32 - K);
    int32_t *Cc = C + (int64_t)c * 2 * M * N;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)Cc, 0, 8 * M * N, tile::RSRC_FLAGS);
    const int mw = m0 + wm * 64, nw = n0 + wn * 64;
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
                const int re = (int)acc_r[i][j][r], im = (int)acc_i[i][j][r] - kpad2;
                if (CIL) {
                    const uint32_t off = ok ? (uint32_t)((m * N + n) * 8) : tile::OOB;
                    const tile::u32x2 v = {(uint32_t)re, (uint32_t)im};
                    __builtin_amdgcn_raw_buffer_store_b64(v, rc, off, 0, tile::kStoreStreaming);
                } else {
                    const uint32_t off = ok ? (uint32_t)((m * N + n) * 4) : tile::OOB;
                    const uint32_t offi = ok ? (uint32_t)(((M + m) * N + n) * 4) : tile::OOB;
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)re, rc, off, 0, tile::kStoreStreaming);
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)im, rc, offi, 0, tile::kStoreStreaming);
                }
            }
        }
}

}  // namespace

// Variant 3 (e2m1): exact fp32 sums (K <= 2^23), whole 16-byte chunks of
// packed words (kw a multiple of 4), and 32-bit byte offsets for every
// per-channel operand and output.
static bool fp4_ok(const Problem &p) {
    const int64_t kw = (p.K + 31) / 32, lim = (int64_t)1 << 31;
    return p.K <= F_MAX_K && kw % 4 == 0 && 8 * p.M * kw < lim && 8 * p.N * kw < lim && 8 * p.M * p.N < lim;
}

bool int1_select(const Problem &p, int forced_variant, Int1Config *cfg) {
    // default: e2m1 where it applies (measured 1.5x the int8 variant on the
    // 64 x 2048 x 8192 x 8192 workload), else int8
    int v = forced_variant == 0 ? (fp4_ok(p) ? 3 : 1) : forced_variant;
    if (v == 1) {
        *cfg = Int1Config{1, U_BM, U_BN, U_BKW, U_NT};
        return true;
    }
    if (v == 2) {
        *cfg = Int1Config{2, V_BM, V_BN, V_BKW, V_NT};
        return true;
    }
    if (v == 3 && fp4_ok(p)) {
        *cfg = Int1Config{3, U_BM, U_BN, F_BKW, U_NT};
        return true;
    }
    return false;
}

int64_t int1_workgroups(const Problem &p, const Int1Config &cfg) {
    return p.batch * ((p.M + cfg.tile_m - 1) / cfg.tile_m) * ((p.N + cfg.tile_n - 1) / cfg.tile_n);
}

const char *int1_kernel_name(const Int1Config &cfg) {
    return cfg.variant == 1 ? "cgemm_1bit_mfma_kernel"
           : cfg.variant == 3 ? "cgemm_1bit_fp4_kernel"
                              : "cgemm_1bit_valu_kernel";
}

hipError_t int1_launch(const Problem &p, const Int1Config &cfg, const uint32_t *A, const uint32_t *B,
                       int32_t *C, hipStream_t stream) {
    const int64_t kw = (p.K + 31) / 32;
    const int tiles_m = (int)((p.M + cfg.tile_m - 1) / cfg.tile_m);
    const int tiles_n = (int)((p.N + cfg.tile_n - 1) / cfg.tile_n);
    const int64_t nblocks = p.batch * tiles_m * tiles_n;
    const int vec = (kw % 4) == 0;
    const bool cil = p.c_layout == TCBF_INTERLEAVED;
    if (cfg.variant == 3) {
        auto fn = cil ? cgemm_1bit_fp4_kernel<1> : cgemm_1bit_fp4_kernel<0>;
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(U_NT), 0, stream, A, B, C, (int)p.M, (int)p.N, (int)p.K,
                           (int)kw, p.a_stride, tiles_m, tiles_n, (int)nblocks);
    } else if (cfg.variant == 1) {
        auto fn = cil ? cgemm_1bit_mfma_kernel<1> : cgemm_1bit_mfma_kernel<0>;
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(U_NT), 0, stream, A, B, C, p.M, p.N, p.K,
                           kw, p.a_stride, tiles_m, tiles_n, nblocks, vec);
    } else {
        auto fn = cil ? cgemm_1bit_valu_kernel<1> : cgemm_1bit_valu_kernel<0>;
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(V_NT), 0, stream, A, B, C, p.M, p.N, p.K,
                           kw, p.a_stride, tiles_m, tiles_n, nblocks, vec);
    }
    return hipGetLastError();
}

int64_t int1_group_tiles(const Problem &p) {
    return p.batch * ((p.M + U_BM - 1) / U_BM) * ((p.N + U_BN - 1) / U_BN);
}

hipError_t int1_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                             const int *order, int count, int c_layout, int grid, unsigned int *counter,
                             hipStream_t stream) {
    Int1GroupArgs args;
    memset(&args, 0, sizeof(args));
    int64_t first = 0;
    for (int j = 0; j < count; ++j) {
        const int i = order[j];
        const Problem &p = probs[i];
        Int1GroupProblem &q = args.p[j];
        q.A = (const uint32_t *)A[i];
        q.B = (const uint32_t *)B[i];
        q.C = (int32_t *)C[i];
        q.M = (int)p.M;
        q.N = (int)p.N;
        q.K = (int)p.K;
        q.kw = (int)((p.K + 31) / 32);
        q.a_shared = p.a_shared;
        q.vec = (q.kw % 4) == 0;
        q.tiles_m = (int)((p.M + U_BM - 1) / U_BM);
        q.tiles_n = (int)((p.N + U_BN - 1) / U_BN);
        q.first_tile = (int)first;
        first += int1_group_tiles(p);
    }
    args.count = count;
    args.total_tiles = (int)first;
    hipLaunchKernelGGL(int1_group_reset_kernel, dim3(1), dim3(1), 0, stream, counter);
    if (c_layout == TCBF_INTERLEAVED)
        hipLaunchKernelGGL(cgemm_1bit_group_kernel<1>, dim3((uint32_t)grid), dim3(U_NT), 0, stream, args, counter);
    else
        hipLaunchKernelGGL(cgemm_1bit_group_kernel<0>, dim3((uint32_t)grid), dim3(U_NT), 0, stream, args, counter);
    return hipGetLastError();
}

}  // namespace tcbf
