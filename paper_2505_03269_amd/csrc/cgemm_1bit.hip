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

#include "tcbf_internal.h"

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
                                          int a_shared, int64_t c, int tm, int tn, int vec, uint32_t *lds,
                                          int (*popA)[U_BM], int (*popB)[U_BN]) {
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)tm * U_BM, n0 = (int64_t)tn * U_BN;

    // loader: thread -> (plane, row) of both tiles; 4 words per stage each
    const int lplane = tid >> 7, lrow = tid & 127;
    const int64_t am = m0 + lrow, bn = n0 + lrow;
    const bool aok = am < M, bok = bn < N;
    const uint32_t *arow = A + (a_shared ? 0 : c * 2 * M * kw) + (int64_t)lplane * M * kw + (aok ? am : 0) * kw;
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
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lc = wn * 64 + j * 32 + l32;
            const int64_t col = n0 + lc;
            const int bsr = popB[0][lc], bsi = popB[1][lc];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int lr = wm * 64 + i * 32 + (r >> 2) * 8 + hl * 4 + (r & 3);
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
    int64_t M, int64_t N, int64_t K, int64_t kw, int a_shared, int tiles_m, int tiles_n,
    int64_t nblocks, int vec) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[2 * U_STAGE];
    __shared__ int popA[2][U_BM], popB[2][U_BN];
    const int64_t t = xcd_remap(blockIdx.x, nblocks);
    const int64_t per_c = (int64_t)tiles_m * tiles_n;
    const int64_t c = t / per_c;
    const int rem = (int)(t - c * per_c);
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    int1_tile<CIL>(A, B, C, M, N, K, kw, a_shared, c, tm, tn, vec, lds, popA, popB);
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
        int1_tile<CIL>(q.A, q.B, q.C, q.M, q.N, q.K, q.kw, q.a_shared, c, tm, tn, q.vec, lds, popA, popB);
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
    int64_t M, int64_t N, int64_t K, int64_t kw, int a_shared, int tiles_m, int tiles_n,
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
        ? A + (a_shared ? 0 : c * 2 * M * kw) + (int64_t)lplane * M * kw + (lok ? lr : 0) * kw
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

}  // namespace

bool int1_select(const Problem &p, int forced_variant, Int1Config *cfg) {
    (void)p;
    int v = forced_variant == 0 ? 1 : forced_variant;
    if (v == 1) {
        *cfg = Int1Config{1, U_BM, U_BN, U_BKW, U_NT};
        return true;
    }
    if (v == 2) {
        *cfg = Int1Config{2, V_BM, V_BN, V_BKW, V_NT};
        return true;
    }
    return false;
}

int64_t int1_workgroups(const Problem &p, const Int1Config &cfg) {
    return p.batch * ((p.M + cfg.tile_m - 1) / cfg.tile_m) * ((p.N + cfg.tile_n - 1) / cfg.tile_n);
}

const char *int1_kernel_name(const Int1Config &cfg) {
    return cfg.variant == 1 ? "cgemm_1bit_mfma_kernel" : "cgemm_1bit_valu_kernel";
}

hipError_t int1_launch(const Problem &p, const Int1Config &cfg, const uint32_t *A, const uint32_t *B,
                       int32_t *C, hipStream_t stream) {
    const int64_t kw = (p.K + 31) / 32;
    const int tiles_m = (int)((p.M + cfg.tile_m - 1) / cfg.tile_m);
    const int tiles_n = (int)((p.N + cfg.tile_n - 1) / cfg.tile_n);
    const int64_t nblocks = p.batch * tiles_m * tiles_n;
    const int vec = (kw % 4) == 0;
    const bool cil = p.c_layout == TCBF_INTERLEAVED;
    if (cfg.variant == 1) {
        auto fn = cil ? cgemm_1bit_mfma_kernel<1> : cgemm_1bit_mfma_kernel<0>;
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(U_NT), 0, stream, A, B, C, p.M, p.N, p.K,
                           kw, p.a_shared, tiles_m, tiles_n, nblocks, vec);
    } else {
        auto fn = cil ? cgemm_1bit_valu_kernel<1> : cgemm_1bit_valu_kernel<0>;
        hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(V_NT), 0, stream, A, B, C, p.M, p.N, p.K,
                           kw, p.a_shared, tiles_m, tiles_n, nblocks, vec);
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
