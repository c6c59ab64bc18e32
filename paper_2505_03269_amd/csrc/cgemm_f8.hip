// FP8 (OCP e4m3) complex beamforming product on the gfx950 FP8 matrix cores.
//
// The 8-bit path is the library's extension of Sec. III-B (the paper names
// 8-bit floats as future work in Sec. VI).  Inputs are e4m3 codes as the
// quantiser writes them: W [batch][2][M][Kp] and X [batch][2][N][Kp], both
// receiver-contiguous with Kp = 32 * ceil(K / 32) and zero padding, or both
// receiver-blocked, [batch][2][ceil(Kp / 64)][rows][64].  The sum
// over receivers is exact-product, fp32-accumulated:
//   per-row scales (TCBF_F8_E4M3): C[m][n] = a_scale[m] * b_scale[n] * sum_k W8 X8
//     -- the scales factor out of the sum, so they are applied in the epilogue;
//   per-block scales (TCBF_MXF8_E4M3): every 32-receiver block carries its own
//     power-of-two scales, applied inside the scaled MFMA per lane.  Scale
//     codes are [batch][Ks / 16][rows][16] bytes, Ks = 16 * ceil(Kp / 512):
//     group g holds blocks 16 g .. 16 g + 15 of every row (codes past Kp / 32
//     are padding that is never used), so the codes a workgroup needs for 8
//     stages are one contiguous run per 128 rows.
// As in the 16-bit kernel, the imaginary part of the product uses W's
// imaginary plane negated in registers (a sign-bit flip, exact in e4m3).
//
// Variants 1 and 2 (variant 3, a persistent 256 x 128 kernel, is further
// down).  Workgroup: 128 beams x 128 samples, 4 waves in a 2 x 2 grid of 64 x 64
// blocks, each wave 2 x 2 MFMA tiles of v_mfma_scale_f32_32x32x64_f8f6f4 per
// real/imaginary accumulator.  One stage holds 64 receivers of both operands
// (2 planes x 128 rows x 64 bytes each, 32 KiB) and is moved by direct-to-LDS
// buffer loads; 16-byte chunks of a row sit XOR-swizzled so the fragment reads
// (32 rows x one chunk per half-wave) are free of bank conflicts.
//
// Operand layout of the 32x32x64 FP8 instruction (measured with one nonzero
// byte per row against distinct block scales): lane l supplies row l%32; its
// first 16 bytes are receivers 16*(l/32) + 0..15 of the step and its second 16
// bytes receivers 32 + 16*(l/32) + 0..15.  The block scale a lane passes
// covers receivers 32*(l/32) + 0..31 of its row.  So a lane reads staged
// chunks l/32 and 2 + l/32, and lanes 0..31 / 32..63 pass the scales of the
// step's first / second 32-receiver block.
//
// The instruction sums its products in groups of 8 and, within a group,
// keeps about 14 bits below the leading product (measured: terms 2^-14 of the
// leading one and smaller are dropped); group sums accumulate in fp32.
#include <algorithm>
#include <cstring>

#include "tcbf_tile.h"

namespace tcbf {
namespace {

using namespace tile;
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int BK = 64;                  // receivers (bytes) per stage
constexpr int ROWB = BK;                // staged row bytes
constexpr int PLANE = BM * ROWB;        // one plane of one operand: 8 KiB
constexpr int REG = 2 * PLANE;          // one operand (2 planes): 16 KiB
constexpr int STAGE = 2 * REG;          // W then X: 32 KiB
constexpr int PIECES_PER_WAVE = REG / 1024 / 4;  // 1 KiB wave loads per operand per wave
constexpr int PIECE_ROWS = 1024 / ROWB;          // rows per wave load
constexpr uint32_t NEG = 0x80808080u;   // sign bits of four e4m3 codes
constexpr int SCALE_ONE = 127;          // E8M0 code of 2^0
constexpr int SLAB_STAGES = 8;          // stages whose block scales one slab holds
constexpr int SLAB_ROWB = 2 * SLAB_STAGES;  // scale bytes per row per slab (16)
constexpr int SLAB = 2 * BM * SLAB_ROWB;    // W rows then X rows: 4 KiB

static_assert(BM == BN, "both operands share the staged geometry");

// Position of chunk ch (0..3) of staged row m: ch ^ swz(m).  Uses row bits
// 1..3 only, so rows 16 apart (the wave-load step) and 32 apart (the MFMA
// tile step) share a swizzle.
__device__ __forceinline__ int swz(int m) { return ((m >> 1) ^ ((m >> 3) & 1)) & 3; }

__device__ __forceinline__ i32x8 frag(const char *st, int o0, int o1) {
    const u32x4 lo = *reinterpret_cast<const u32x4 *>(st + o0);
    const u32x4 hi = *reinterpret_cast<const u32x4 *>(st + o1);
    return (i32x8){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
}

__device__ __forceinline__ f32x16 mma(const i32x8 &x, const i32x8 &w, const f32x16 &c, int sx, int sw) {
    // A = X fragment (rows: samples), B = W fragment (columns: beams); both e4m3
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, w, c, 0, 0, 0, sx, 0, sw);
}

// LDS of one workgroup: the NS-deep stage ring and (MX only) two block-scale
// slab slots; separate arrays, so the compiler sees that reads of one stage
// and direct loads into another cannot alias.
#define TCBF_F8_LDS(NS, MX)                                                                      \
    __shared__ __attribute__((aligned(1024))) char lds0[STAGE];                                 \
    __shared__ __attribute__((aligned(1024))) char lds1[STAGE];                                 \
    __shared__ __attribute__((aligned((NS) > 2 ? 1024 : 4))) char lds2[(NS) > 2 ? STAGE : 4];   \
    __shared__ __attribute__((aligned((NS) > 3 ? 1024 : 4))) char lds3[(NS) > 3 ? STAGE : 4];   \
    __shared__ __attribute__((aligned((MX) ? 1024 : 4))) char slabs[(MX) ? 2 * SLAB : 4];

// One 128 x 128 output tile of channel c.  BL: both operands in the
// receiver-blocked layout (TCBF_BLOCKED: per plane, blocks of 64 receivers,
// each block all rows x 64 bytes), so a stage's tile of each operand is one
// contiguous run per plane and every load instruction reads whole cache
// lines; receiver-contiguous rows give 64-byte pieces instead.
template <int NS, int CIL, int MX, int BL>
__device__ __forceinline__ void f8_tile(const uint8_t *__restrict__ A, const uint8_t *__restrict__ B,
                                        float *__restrict__ C, const void *__restrict__ a_scale,
                                        const void *__restrict__ b_scale, int M, int N, int Kp, int64_t a_stride,
                                        int c, int tm, int tn, char *lds0, char *lds1, char *lds2, char *lds3,
                                        char *slabs) {
    static_assert(NS >= 2 && NS <= 4 && NS <= SLAB_STAGES + 1, "ring depth");
    // stage buffer i: a select chain, not an array (an LDS pointer array the
    // compiler cannot index statically goes to scratch as generic pointers)
    auto bufs = [&](int i) __attribute__((always_inline)) -> char * {
        char *b = lds0;
        if (i == 1) b = lds1;
        if (i == 2) b = lds2;
        if (i == 3) b = lds3;
        return b;
    };
    const int tid = threadIdx.x;
    const int m0 = tm * BM, n0 = tn * BN;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    const int cw = a_stride == 0 ? 0 : c;  // scale entry (codes: a_stride bytes apart)
    const int KS = BL ? (Kp + BK - 1) / BK * BK : Kp;  // bytes per row as stored (blocked: whole blocks)
    const uint8_t *Wc = A + (int64_t)c * a_stride;
    const uint8_t *Xc = B + (int64_t)c * 2 * N * KS;
    const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc((void *)Wc, 0, 2 * M * KS, RSRC_FLAGS);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc((void *)Xc, 0, 2 * N * KS, RSRC_FLAGS);
    // row pitch inside a plane, and the uniform step from one stage to the next
    const int pitch_w = BL ? BK : Kp, pitch_x = BL ? BK : Kp;

    // This lane's 16-byte chunk in each of the wave's loads.  Slot s of an
    // operand region (16 B each, lane order within a 1 KiB wave load) holds
    // plane s/512, row (s/4)%128, chunk (s%4)^swz(row); the wave's pieces are
    // 16 rows apart within one plane.
    int row0, kc;  // staged row of piece 0, receiver offset of the chunk
    uint32_t plane_off_w, plane_off_x;
    {
        const int s = wave * PIECES_PER_WAVE * 64 + lane;
        const int p = s / (BM * 4);
        row0 = (s / 4) % BM;
        kc = ((s & 3) ^ swz(row0)) * 16;
        plane_off_w = (uint32_t)(p * M) * KS;
        plane_off_x = (uint32_t)(p * N) * KS;
    }

    // Fragment offsets within a stage (plane 0 of W; X adds REG, the
    // imaginary plane adds PLANE, the second 32-row tile adds 32 rows).
    const int fw = wm * 64 + l32, fx = wn * 64 + l32;
    const int ow0 = fw * ROWB + ((hl ^ swz(fw)) * 16), ow1 = fw * ROWB + (((2 + hl) ^ swz(fw)) * 16);
    const int ox0 = REG + fx * ROWB + ((hl ^ swz(fx)) * 16);
    const int ox1 = REG + fx * ROWB + (((2 + hl) ^ swz(fx)) * 16);

    // Block scales travel through LDS: every SLAB_STAGES stages one direct
    // 16-byte load per lane brings the next 16 block codes of one staged row
    // (waves 0, 1: W rows 0..63, 64..127; waves 2, 3: the same X rows; one
    // contiguous KiB per wave) into the slab slot (kt / SLAB_STAGES) % 2.  A slot's next load is issued
    // SLAB_STAGES + 2 - NS steps after the step that read its last stage, so
    // a ring barrier lies between them.  Compute reads this
    // lane's four codes (beams fw, fw + 32; samples fx, fx + 32; block
    // 2 kt + hl) from the slot.
    const int nkb = Kp / 32;
    const int ks = (int)mx_scale_pitch(Kp);
    static_assert(SLAB_ROWB == 16, "one slab row is the pitch granule");
    const int so = wave >> 1;                                       // slab operand of this wave
    __amdgpu_buffer_rsrc_t rss = __builtin_amdgcn_make_buffer_rsrc((void *)a_scale, 0, 0, RSRC_FLAGS);
    uint32_t slab_off = OOB;
    int group_bytes = 0;  // one group of 16 codes of every row of this operand
    if (MX) {
        const int rows = so ? N : M;
        const uint8_t *base = so ? (const uint8_t *)b_scale + (int64_t)c * N * ks
                                 : (const uint8_t *)a_scale + (int64_t)cw * M * ks;
        rss = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, rows * ks, RSRC_FLAGS);
        const int r = (so ? n0 : m0) + 64 * (wave & 1) + lane;
        slab_off = r < rows ? (uint32_t)(r * SLAB_ROWB) : OOB;
        group_bytes = rows * SLAB_ROWB;
    }

    auto issue = [&](char *base, int kt) __attribute__((always_inline)) {
        const int k0 = kt * BK;
        const bool kin = k0 + kc < Kp;
#pragma unroll
        for (int q = 0; q < PIECES_PER_WAVE; ++q) {
            const int r = row0 + q * PIECE_ROWS;
            const uint32_t off = (kin && m0 + r < M) ? plane_off_w + (uint32_t)(m0 + r) * pitch_w + kc : OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (TCBF_LDS_AS void *)(base + (wave * PIECES_PER_WAVE + q) * 1024),
                                                     16, off, BL ? kt * M * BK : k0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < PIECES_PER_WAVE; ++q) {
            const int r = row0 + q * PIECE_ROWS;
            const uint32_t off = (kin && n0 + r < N) ? plane_off_x + (uint32_t)(n0 + r) * pitch_x + kc : OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx,
                                                     (TCBF_LDS_AS void *)(base + REG + (wave * PIECES_PER_WAVE + q) * 1024),
                                                     16, off, BL ? kt * N * BK : k0, 0, 0);
        }
        if (MX && kt % SLAB_STAGES == 0)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rss, (TCBF_LDS_AS void *)(slabs + (kt / SLAB_STAGES % 2) * SLAB + so * (SLAB / 2) + (wave & 1) * 1024),
                16, slab_off, (kt / SLAB_STAGES) * group_bytes, 0, 0);
    };

    Acc acc;
    acc.zero();
    // Block codes of stage kt: [W tile i, X tile j].  A block past Kp / 32
    // (the second half of the last stage when Kp % 64 == 32) has zero data
    // and takes 2^0.  Read before the step issues its loads: the compiler
    // makes an LDS read wait for every direct load into the same array still
    // in flight; with a two-stage ring none is at that point (with three, the
    // next stage's loads are waited for here).
    auto read_scales = [&](int kt, int *sc) __attribute__((always_inline)) {
        const char *sl = slabs + (kt / SLAB_STAGES % 2) * SLAB + 2 * (kt % SLAB_STAGES) + hl;
        const bool bin = 2 * kt + hl < nkb;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int w = ((const uint8_t *)sl)[(fw + 32 * i) * SLAB_ROWB];
            const int x = ((const uint8_t *)sl)[SLAB / 2 + (fx + 32 * i) * SLAB_ROWB];
            sc[i] = bin ? w : SCALE_ONE;
            sc[2 + i] = bin ? x : SCALE_ONE;
        }
    };
    auto compute = [&](const char *st, const int *sc) __attribute__((always_inline)) {
        i32x8 xr[2], xi[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            xr[j] = frag(st, ox0 + j * 32 * ROWB, ox1 + j * 32 * ROWB);
            xi[j] = frag(st, ox0 + j * 32 * ROWB + PLANE, ox1 + j * 32 * ROWB + PLANE);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const i32x8 wr = frag(st, ow0 + i * 32 * ROWB, ow1 + i * 32 * ROWB);
            const i32x8 wi = frag(st, ow0 + i * 32 * ROWB + PLANE, ow1 + i * 32 * ROWB + PLANE);
            const i32x8 wn = wi ^ (int)NEG;
            const int sw = sc[i];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int sx = sc[2 + j];
                acc.re[i][j] = mma(xr[j], wr, acc.re[i][j], sx, sw);
                acc.im[i][j] = mma(xi[j], wr, acc.im[i][j], sx, sw);
                acc.re[i][j] = mma(xi[j], wn, acc.re[i][j], sx, sw);
                acc.im[i][j] = mma(xr[j], wi, acc.im[i][j], sx, sw);
            }
        }
    };

    // Ring: stage kt lives in buffer kt % NS; NS-1 stages are in flight.
    // loads per wave per stage; a slab load every SLAB_STAGES stages only
    // makes the count of later loads larger, which keeps the wait safe
    constexpr int PER_STAGE = 2 * PIECES_PER_WAVE;
    static_assert((NS - 2) * PER_STAGE < 64, "vmcnt range");
    constexpr int kWaitRing = vmcnt_imm((NS - 2) * PER_STAGE), kWaitAll = vmcnt_imm(0);
    const int nk = (Kp + BK - 1) / BK;
    auto stage_step = [&](int kt, int u) __attribute__((always_inline)) {
        if (kt + NS - 2 < nk) __builtin_amdgcn_s_waitcnt(kWaitRing);
        else __builtin_amdgcn_s_waitcnt(kWaitAll);
        // all waves' loads for stage kt landed, stage kt-1 fully read
        asm volatile("s_barrier" ::: "memory");
        int sc[4] = {SCALE_ONE, SCALE_ONE, SCALE_ONE, SCALE_ONE};
        if (MX) read_scales(kt, sc);
        if (kt + NS - 1 < nk) issue(bufs((u + NS - 1) % NS), kt + NS - 1);
        compute(bufs(u), sc);
    };
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(bufs(s), s);
    int kt0 = 0;
    for (; kt0 + NS <= nk; kt0 += NS) {
#pragma unroll
        for (int u = 0; u < NS; ++u) stage_step(kt0 + u, u);
    }
#pragma unroll
    for (int u = 0; u < NS - 1; ++u)
        if (kt0 + u < nk) stage_step(kt0 + u, u);

    if (!MX) {
        // per-row scales: beams fw + 32 i, samples wn*64 + 32 j + 8 q + 4 hl + (0..3)
        const float *as = (const float *)a_scale + (int64_t)cw * M;
        const float *bs = (const float *)b_scale + (int64_t)c * N;
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void *)as, 0, 4 * M, RSRC_FLAGS);
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc((void *)bs, 0, 4 * N, RSRC_FLAGS);
        float sa[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m0 + fw + 32 * i;
            sa[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, m < M ? (uint32_t)(4 * m) : OOB, 0, 0));
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = n0 + wn * 64 + 32 * j + 8 * q + 4 * hl;  // N % 4 == 0: all four or none
                // whole-vector cast: a bit_cast of one subscripted element
                // would not select that element
                const f32x4 tb = __builtin_bit_cast(
                    f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, n < N ? (uint32_t)(4 * n) : OOB, 0, 0));
#pragma unroll
                for (int i = 0; i < 2; ++i) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float f = sa[i] * tb[e];
                        acc.re[i][j][4 * q + e] *= f;
                        acc.im[i][j][4 * q + e] *= f;
                    }
                }
            }
    }

    // Epilogue through the (now idle) stage buffers.
    constexpr int ROWS_PER_BUF = STAGE / staging_pitch<CIL>();
    static_assert(ROWS_PER_BUF * 2 >= (CIL ? 64 : 128), "two stage buffers hold a staging round");
    auto row_ptr = [&](int row) __attribute__((always_inline)) -> char * {
        return (row < ROWS_PER_BUF ? lds0 : lds1) + (row % ROWS_PER_BUF) * staging_pitch<CIL>();
    };
    store_tile_staged<2, CIL>(acc, row_ptr, C + (int64_t)c * 2 * M * N, M, N, m0, n0, wave, lane);
}

template <int NS, int CIL, int MX, int BL>
__global__ __launch_bounds__(NT, 2) void cgemm_f8_kernel(
    const uint8_t *__restrict__ A, const uint8_t *__restrict__ B, float *__restrict__ C,
    const void *__restrict__ a_scale, const void *__restrict__ b_scale, int M, int N, int Kp, int64_t a_stride,
    int tiles_m, int tiles_n, int nblocks) {
    TCBF_F8_LDS(NS, MX)
    const int t = (int)xcd_remap(blockIdx.x, nblocks);
    const int per_c = tiles_m * tiles_n;
    const int c = t / per_c;
    const int rem = t - c * per_c;
    int tm, tn;
    tile_coords(rem, tiles_m, tiles_n, tm, tn);
    f8_tile<NS, CIL, MX, BL>(A, B, C, a_scale, b_scale, M, N, Kp, a_stride, c, tm, tn, lds0, lds1, lds2, lds3,
                             slabs);
}

// Grouped persistent launch: problems of different shapes (and their own
// scales) in one launch; workgroups take tile indices from a device counter
// and run the plain kernel's tile code (two-stage ring), so every problem's
// output equals its own plan's bit for bit.  The table travels in the kernel
// arguments.
struct F8GroupProblem {
    const uint8_t *A;
    const uint8_t *B;
    float *C;
    const void *a_scale;
    const void *b_scale;
    int M, N, Kp, a_shared;
    int tiles_m, tiles_n;  // per channel
    int first_tile;        // index of this problem's first tile in the list
    int pad;
};
struct F8GroupArgs {
    F8GroupProblem p[TCBF_GROUP_MAX];
    int count, total_tiles;
};

template <int CIL, int MX, int BL>
__global__ __launch_bounds__(NT, 2) void cgemm_f8_group_kernel(const F8GroupArgs args,
                                                                unsigned int *__restrict__ counter) {
    TCBF_F8_LDS(2, MX)
    __shared__ int next_tile;
    for (;;) {
        if (threadIdx.x == 0) next_tile = (int)atomicAdd(counter, 1u);
        // the index is visible, and every wave has finished the previous
        // tile's LDS use (epilogue staging, scale slabs) before the next
        // tile's loads land
        lds_barrier();
        const int t = __builtin_amdgcn_readfirstlane(next_tile);
        if (t >= args.total_tiles) break;
        int pi = 0;
        for (int i = 1; i < args.count; ++i)
            if (t >= args.p[i].first_tile) pi = i;
        const F8GroupProblem &q = args.p[pi];
        const int local = t - q.first_tile;
        const int per_c = q.tiles_m * q.tiles_n;
        const int c = local / per_c;
        const int rem = local - c * per_c;
        int tm, tn;
        tile_coords(rem, q.tiles_m, q.tiles_n, tm, tn);
        const int64_t a_stride = q.a_shared ? 0 : 2 * (int64_t)q.M * (BL ? (q.Kp + BK - 1) / BK * BK : q.Kp);
        f8_tile<2, CIL, MX, BL>(q.A, q.B, q.C, q.a_scale, q.b_scale, q.M, q.N, q.Kp, a_stride, c, tm, tn, lds0, lds1,
                                lds2, lds3, slabs);
        // next_tile is rewritten only after the tile's own barriers, which
        // every wave passes after reading it
    }
}

__global__ void f8_group_reset_kernel(unsigned int *counter) { *counter = 0u; }

// ===========================================================================
// Ping-pong persistent kernel (variant 3): one 512-thread workgroup per CU,
// 256 beams x 128 samples per tile, 64 receivers per stage.
// ===========================================================================
//
// The fp16 ping-pong schedule on FP8 codes.  Eight waves in a 4 x 2 grid of
// 64 x 64 blocks share each staged tile of W (2 planes x 256 rows x 64 bytes)
// and X (2 x 128 x 64), 48 KiB per stage through a ring of three; waves w and
// w + 4 share a SIMD, and the groups of waves 0..3 and 4..7 alternate a matrix
// phase (16 scaled MFMAs) with a data phase (the next-but-one stage's loads,
// this stage's fragment reads, the wait for the next stage, and after a
// tile's last stage the tile's stores straight from the accumulators).  The
// workgroup walks its tiles (XCD-contiguous order) as one stage sequence.
//
// W is the matrix instruction's first operand here (rows: beams), so a lane
// of the result holds one sample and its registers beams; the products, the
// order in which each accumulator takes them and the scales are those of the
// 128 x 128 kernels, so the results equal theirs bit for bit.
//
// Scales.  Per-row: each tile's 256 W and 128 X row scales are moved into LDS
// together with the tile's first stage (slot = tile % 4, so a slot is
// rewritten only after its tile's epilogue has read it, whatever the stage
// count) and applied in the epilogue.  Per-block: the 16-code groups of 8
// stages travel as in the 128 x 128 kernel, in two slab slots taken in turn
// by the workgroup's running group count; a slot is refilled with the loads
// of its next group's first stage, two stages ahead, so every group must span
// at least two stages (ceil(Kp / 64) % 8 != 1, checked at plan time).  The
// codes are read with an LDS read the compiler does not track (see
// read_codes): reads of an array that direct loads fill make it wait for
// every load in flight, which here would be the next stages' loads.
namespace pp {
constexpr int TM = 256, TN = 128;
constexpr int PLANE_W = TM * ROWB;            // 16 KiB
constexpr int PLANE_X = TN * ROWB;            // 8 KiB
constexpr int REG_W = 2 * PLANE_W;            // W region of a stage: 32 KiB
constexpr int PP_STAGE = REG_W + 2 * PLANE_X;    // 48 KiB
constexpr int WPW = REG_W / 1024 / 8;         // W wave loads per wave per stage (4)
constexpr int XPW = 2 * PLANE_X / 1024 / 8;   // X wave loads per wave per stage (2)
constexpr int SLAB_W = TM * SLAB_ROWB;        // W rows of a block-scale slab: 4 KiB
constexpr int PP_SLAB = SLAB_W + TN * SLAB_ROWB; // 6 KiB
constexpr int ROWSCALE = 2048;                // per-row scale slot: 256 W floats, 128 X floats, padding
constexpr int ROWSCALE_SLOTS = 4;
static_assert(WPW * 8 * 1024 == REG_W && XPW * 8 * 1024 == 2 * PLANE_X, "whole wave loads");
static_assert(3 * PP_STAGE + 2 * PP_SLAB <= 160 * 1024, "LDS");
}  // namespace pp

__device__ __forceinline__ void f8_pp_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Four block-scale codes from the slab: bytes at LDS addresses aw, aw + 512
// (W rows 32 apart) and ax, ax + 512 (X rows).  Written as one asm block that
// waits for its own reads, so the compiler neither tracks these reads against
// the direct loads into the slab array nor sees a read still in flight.
__device__ __forceinline__ void read_codes(uint32_t aw, uint32_t ax, int (&code)[4]) {
    asm volatile(
        "ds_read_u8 %0, %4\n\t"
        "ds_read_u8 %1, %4 offset:512\n\t"
        "ds_read_u8 %2, %5\n\t"
        "ds_read_u8 %3, %5 offset:512\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(code[0]), "=&v"(code[1]), "=&v"(code[2]), "=&v"(code[3])
        : "v"(aw), "v"(ax)
        : "memory");
}

__device__ __forceinline__ f32x16 mma_wx(const i32x8 &w, const i32x8 &x, const f32x16 &c, int sw, int sx) {
    // A = W fragment (rows: beams), B = X fragment (columns: samples)
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(w, x, c, 0, 0, 0, sw, 0, sx);
}

// Store a wave's 64 x 64 block (beams mw.., samples nw.. of the channel's
// output Cc) from accumulators with lane = sample, registers = beams: one
// 4-byte store per register and plane (two whole 128-byte row runs) or one
// 8-byte (re, im) store per register pair.  Per-row scales (rs: this tile's
// slot, W scales then X scales, tile-relative rows) multiply each sum by
// a_scale[m] * b_scale[n], the product and rounding of the 128 x 128 kernels.
template <int CIL, int MX>
__device__ __forceinline__ void f8_store_block(const Acc &acc, float *Cc, const char *rs, int M, int N, int mw,
                                               int nw, int rw, int rx, int lane) {
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)Cc, 0, 8 * M * N, RSRC_FLAGS);
    const int hl = lane >> 5, l32 = lane & 31;
    const bool whole = mw + 64 <= M && nw + 64 <= N;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        f32x4 sa[4];
        if (!MX) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                sa[q] = *reinterpret_cast<const f32x4 *>(rs + 4 * (rw + 32 * i + 8 * q + 4 * hl));
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = nw + 32 * j + l32;
            const bool n_ok = n < N;
            const float sb = MX ? 1.0f : *reinterpret_cast<const float *>(rs + 4 * pp::TM + 4 * (rx + 32 * j + l32));
            const int mb = mw + 32 * i + 4 * hl;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = mb + 8 * (r >> 2) + (r & 3);
                const bool ok = whole || (n_ok && m < M);
                float re = acc.re[i][j][r], im = acc.im[i][j][r];
                if (!MX) {
                    const float f = sa[r >> 2][r & 3] * sb;
                    re *= f;
                    im *= f;
                }
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
}

template <int CIL, int MX, int BL>
__global__ __launch_bounds__(512, 1) void cgemm_f8_pp_kernel(
    const uint8_t *__restrict__ A, const uint8_t *__restrict__ B, float *__restrict__ C,
    const void *__restrict__ a_scale, const void *__restrict__ b_scale, int M, int N, int Kp, int64_t a_stride,
    int tiles_m, int tiles_n, int total_tiles) {
    using namespace pp;
    __shared__ __attribute__((aligned(1024))) char lds0[PP_STAGE];
    __shared__ __attribute__((aligned(1024))) char lds1[PP_STAGE];
    __shared__ __attribute__((aligned(1024))) char lds2[PP_STAGE];
    // per-block scale slabs (MX) or per-row scale slots
    __shared__ __attribute__((aligned(1024))) char scl[MX ? 2 * PP_SLAB : ROWSCALE_SLOTS * ROWSCALE];

    const int grid = (int)gridDim.x;
    // tile order as in the fp16 ping-pong kernel: with a grid that is a
    // multiple of the 8 XCDs each XCD takes a contiguous eighth of the tiles
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
    const int nk = (Kp + BK - 1) / BK;        // stages per tile
    const int ngr = (nk + SLAB_STAGES - 1) / SLAB_STAGES;  // block-scale groups per tile
    const int S = ntiles * nk;                // stages this workgroup runs
    const int per_c = tiles_m * tiles_n;
    const int KS = BL ? nk * BK : Kp;         // stored bytes per row
    const int pitch = BL ? BK : Kp;           // row step inside a staged run
    const int nkb = Kp / 32;                  // 32-receiver blocks per row

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1, grp = wave >> 2;
    const int hl = lane >> 5, l32 = lane & 31;

    // This lane's 16-byte chunk in each of its wave loads (slot s of a region
    // holds plane s / (4 rows), row (s / 4) % rows, chunk (s % 4) ^ swz(row);
    // a wave's loads are 16 rows apart, which keeps the swizzle).
    int roww, kcw, rowx, kcx;
    uint32_t pw_off, px_off;
    {
        const int s = wave * WPW * 64 + lane;
        roww = (s / 4) % TM;
        kcw = ((s & 3) ^ swz(roww)) * 16;
        pw_off = (uint32_t)((s / (TM * 4)) * M) * (uint32_t)KS;
        const int t = wave * XPW * 64 + lane;
        rowx = (t / 4) % TN;
        kcx = ((t & 3) ^ swz(rowx)) * 16;
        px_off = (uint32_t)((t / (TN * 4)) * N) * (uint32_t)KS;
    }
    // fragment offsets in a stage (real planes; imaginary planes add a plane)
    const int fw = wm * 64 + l32, fx = wn * 64 + l32;
    const int ow0 = fw * ROWB + ((hl ^ swz(fw)) * 16), ow1 = fw * ROWB + (((2 + hl) ^ swz(fw)) * 16);
    const int ox0 = REG_W + fx * ROWB + ((hl ^ swz(fx)) * 16);
    const int ox1 = REG_W + fx * ROWB + (((2 + hl) ^ swz(fx)) * 16);
    const int ks = (int)mx_scale_pitch(Kp);

    auto tile_of = [&](int round, int &c, int &m0, int &n0) __attribute__((always_inline)) {
        const int t = first + round * stride;
        c = t / per_c;
        int tm, tn;
        tile_coords(t - c * per_c, tiles_m, tiles_n, tm, tn);
        m0 = tm * TM;
        n0 = tn * TN;
    };

    // load cursor: the tile and stage the next issue() loads
    int l_round = 0, l_kt = 0;
    bool l_live = true;
    uint32_t l_w[WPW], l_x[XPW], l_s = OOB;  // per-lane offsets of this tile (OOB: rows past M / N)
    __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(nullptr, 0, 0, RSRC_FLAGS), rx = rw, rs = rw;
    auto load_tile = [&]() __attribute__((always_inline)) {
        l_live = l_round < ntiles;
        if (!l_live) return;
        int c, m0, n0;
        tile_of(l_round, c, m0, n0);
        const int cw = a_stride == 0 ? 0 : c;  // scale entry
        rw = __builtin_amdgcn_make_buffer_rsrc((void *)(A + (int64_t)c * a_stride), 0, 2 * M * KS, RSRC_FLAGS);
        rx = __builtin_amdgcn_make_buffer_rsrc((void *)(B + (int64_t)c * 2 * N * KS), 0, 2 * N * KS, RSRC_FLAGS);
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            const int m = m0 + roww + 16 * q;
            l_w[q] = m < M ? pw_off + (uint32_t)m * (uint32_t)pitch + (uint32_t)kcw : OOB;
        }
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            const int n = n0 + rowx + 16 * q;
            l_x[q] = n < N ? px_off + (uint32_t)n * (uint32_t)pitch + (uint32_t)kcx : OOB;
        }
        // scale rows: waves 0..3 W rows 64 w + lane, waves 4, 5 X rows
        l_s = OOB;
        if (wave < 6) {
            const bool xs = wave >= 4;
            const int rows = xs ? N : M;
            const int r = (xs ? n0 + 64 * (wave - 4) : m0 + 64 * wave) + lane;
            if (MX) {
                const uint8_t *base = xs ? (const uint8_t *)b_scale + (int64_t)c * N * ks
                                         : (const uint8_t *)a_scale + (int64_t)cw * M * ks;
                rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, rows * ks, RSRC_FLAGS);
                if (r < rows) l_s = (uint32_t)(r * SLAB_ROWB);
            } else {
                const float *base = xs ? (const float *)b_scale + (int64_t)c * N : (const float *)a_scale + (int64_t)cw * M;
                rs = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, 4 * rows, RSRC_FLAGS);
                if (r < rows) l_s = (uint32_t)(4 * r);
            }
        }
    };
    // Issue this wave's loads of the cursor's stage into `base` and advance.
    // Stages past the last are issued too, every offset out of range (zero
    // fills of buffers nobody reads again), so the wait counts are the same
    // on every path; scale loads come after the stage's own loads, so a wait
    // for the stage's loads only ever waits for more.
    auto issue = [&](char *base) __attribute__((always_inline)) {
        const int k0 = l_kt * BK;
#pragma unroll
        for (int q = 0; q < WPW; ++q) {
            const uint32_t off = (l_live && k0 + kcw < Kp) ? l_w[q] : OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rw, (TCBF_LDS_AS void *)(base + (wave * WPW + q) * 1024), 16,
                                                     off, BL ? l_kt * M * BK : k0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < XPW; ++q) {
            const uint32_t off = (l_live && k0 + kcx < Kp) ? l_x[q] : OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (TCBF_LDS_AS void *)(base + REG_W + (wave * XPW + q) * 1024),
                                                     16, off, BL ? l_kt * N * BK : k0, 0, 0);
        }
        if (l_live && wave < 6) {
            if (MX && l_kt % SLAB_STAGES == 0) {
                const int g = l_round * ngr + l_kt / SLAB_STAGES;  // running group count: slots alternate
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (TCBF_LDS_AS void *)(scl + (g % 2) * PP_SLAB + wave * 1024), 16, l_s,
                    (l_kt / SLAB_STAGES) * (wave >= 4 ? N : M) * SLAB_ROWB, 0, 0);
            }
            if (!MX && l_kt == 0)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rs, (TCBF_LDS_AS void *)(scl + (l_round % ROWSCALE_SLOTS) * ROWSCALE + wave * 256), 4, l_s, 0, 0,
                    0);
        }
        if (++l_kt == nk) {
            l_kt = 0;
            ++l_round;
            load_tile();
        }
    };

    i32x8 wr[2], wi[2], xr[2], xi[2];
    int sc[4] = {SCALE_ONE, SCALE_ONE, SCALE_ONE, SCALE_ONE};
    int c_round = 0, c_kt = 0;  // compute cursor
    auto read_frags = [&](const char *st) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            wr[i] = frag(st, ow0 + i * 32 * ROWB, ow1 + i * 32 * ROWB);
            wi[i] = frag(st, ow0 + i * 32 * ROWB + PLANE_W, ow1 + i * 32 * ROWB + PLANE_W);
            xr[i] = frag(st, ox0 + i * 32 * ROWB, ox1 + i * 32 * ROWB);
            xi[i] = frag(st, ox0 + i * 32 * ROWB + PLANE_X, ox1 + i * 32 * ROWB + PLANE_X);
        }
        if (MX) {
            // codes of this stage's blocks: [W beams fw, fw + 32][X samples fx, fx + 32];
            // a block past Kp / 32 has zero data and takes 2^0
            const int g = c_round * ngr + c_kt / SLAB_STAGES;
            const uint32_t sl = (uint32_t)(uintptr_t)(TCBF_LDS_AS char *)scl + (uint32_t)((g % 2) * PP_SLAB) +
                                (uint32_t)(2 * (c_kt % SLAB_STAGES) + hl);
            const bool bin = 2 * c_kt + hl < nkb;
            int code[4];
            read_codes(sl + (uint32_t)(fw * SLAB_ROWB), sl + (uint32_t)(SLAB_W + fx * SLAB_ROWB), code);
#pragma unroll
            for (int q = 0; q < 4; ++q) sc[q] = bin ? code[q] : SCALE_ONE;
        }
    };
    Acc acc;
    acc.zero();
    auto store_round = [&](int round) __attribute__((always_inline)) {
        int c, m0, n0;
        tile_of(round, c, m0, n0);
        f8_store_block<CIL, MX>(acc, C + (int64_t)c * 2 * M * N, scl + (round % ROWSCALE_SLOTS) * ROWSCALE, M, N,
                                m0 + wm * 64, n0 + wn * 64, wm * 64, wn * 64, lane);
    };
    constexpr int PER_STAGE = WPW + XPW;
    constexpr int kWaitNext = vmcnt_imm(PER_STAGE), kWaitAll = vmcnt_imm(0);
    auto step = [&](char *rd, char *ld) __attribute__((always_inline)) {
        // data phase
        issue(ld);
        read_frags(rd);
        __builtin_amdgcn_s_waitcnt(kWaitNext);  // own loads of the next stage landed
        if (c_kt == 0 && c_round > 0) {         // the previous stage ended a tile
            store_round(c_round - 1);
            acc.zero();
        }
        __builtin_amdgcn_s_waitcnt(kWaitLds);
        f8_pp_barrier();
        // matrix phase: per accumulator the order of the 128 x 128 kernels
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const i32x8 wn = wi[i] ^ (int)NEG;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc.re[i][j] = mma_wx(wr[i], xr[j], acc.re[i][j], sc[i], sc[2 + j]);
                acc.im[i][j] = mma_wx(wr[i], xi[j], acc.im[i][j], sc[i], sc[2 + j]);
                acc.re[i][j] = mma_wx(wn, xi[j], acc.re[i][j], sc[i], sc[2 + j]);
                acc.im[i][j] = mma_wx(wi[i], xr[j], acc.im[i][j], sc[i], sc[2 + j]);
            }
        }
        if (++c_kt == nk) {
            c_kt = 0;
            ++c_round;
        }
        f8_pp_barrier();
    };

    load_tile();
    issue(lds0);
    issue(lds1);
    __builtin_amdgcn_s_waitcnt(kWaitNext);  // own loads of stage 0 (and its scale group) landed
    f8_pp_barrier();
    if (grp == 1) f8_pp_barrier();
    // stage s reads buffer s % 3 and loads stage s + 2 into buffer (s + 2) % 3
    int s = 0;
    for (; s + 3 <= S; s += 3) {
        step(lds0, lds2);
        step(lds1, lds0);
        step(lds2, lds1);
    }
    if (s < S) step(lds0, lds2);
    if (s + 1 < S) step(lds1, lds0);
    store_round(c_round - 1);
    if (grp == 0) f8_pp_barrier();
    __builtin_amdgcn_s_waitcnt(kWaitAll);
}

typedef void (*F8Fn)(const uint8_t *, const uint8_t *, float *, const void *, const void *, int, int, int, int64_t,
                     int, int, int);

template <int BL> F8Fn f8_fn_of(int v, bool cil, bool mx) {
    if (mx) {
        if (v == 2) return cil ? cgemm_f8_kernel<3, 1, 1, BL> : cgemm_f8_kernel<3, 0, 1, BL>;
        return cil ? cgemm_f8_kernel<2, 1, 1, BL> : cgemm_f8_kernel<2, 0, 1, BL>;
    }
    if (v == 2) return cil ? cgemm_f8_kernel<3, 1, 0, BL> : cgemm_f8_kernel<3, 0, 0, BL>;
    return cil ? cgemm_f8_kernel<2, 1, 0, BL> : cgemm_f8_kernel<2, 0, 0, BL>;
}

F8Fn f8_fn(int v, bool cil, bool mx, bool bl) { return bl ? f8_fn_of<1>(v, cil, mx) : f8_fn_of<0>(v, cil, mx); }

F8Fn f8_pp_fn(bool cil, bool mx, bool bl) {
    static const F8Fn fns[8] = {cgemm_f8_pp_kernel<0, 0, 0>, cgemm_f8_pp_kernel<0, 0, 1>, cgemm_f8_pp_kernel<0, 1, 0>,
                                cgemm_f8_pp_kernel<0, 1, 1>, cgemm_f8_pp_kernel<1, 0, 0>, cgemm_f8_pp_kernel<1, 0, 1>,
                                cgemm_f8_pp_kernel<1, 1, 0>, cgemm_f8_pp_kernel<1, 1, 1>};
    return fns[(cil << 2) | (mx << 1) | bl];
}

// 1: two-stage ring (default), 2: three-stage ring, 3: ping-pong persistent
constexpr int kNumVariants = 3, kPingPong = 3;

int64_t pp_tiles(const Problem &p) {
    return p.batch * ((p.M + pp::TM - 1) / pp::TM) * ((p.N + pp::TN - 1) / pp::TN);
}

}  // namespace

int64_t f8_kp(int64_t K) { return (K + 31) / 32 * 32; }

bool f8_select(const Problem &p, bool mx, int forced_variant, F8Config *cfg) {
    int v = forced_variant == 0 ? 1 : forced_variant;
    if (v < 1 || v > kNumVariants) return false;
    if (p.N % 4 != 0) return false;
    // both operands planar, or both receiver-blocked
    if (p.a_layout != p.b_layout || (p.a_layout != TCBF_PLANAR && p.a_layout != TCBF_BLOCKED)) return false;
    if (v == kPingPong) {
        const int64_t nk = (f8_kp(p.K) + BK - 1) / BK;
        // the persistent kernel counts a workgroup's stages in 32 bits; with
        // per-block scales every 8-stage scale group spans at least 2 stages
        if (pp_tiles(p) * nk >= ((int64_t)1 << 31)) return false;
        if (mx && nk % SLAB_STAGES == 1) return false;
    }
    cfg->variant = v;
    cfg->tile_m = v == kPingPong ? pp::TM : BM;
    cfg->tile_n = BN;
    cfg->tile_k = BK;
    cfg->threads = v == kPingPong ? 512 : NT;
    return true;
}

int64_t f8_workgroups(const Problem &p, const F8Config &cfg) {
    return p.batch * ((p.M + cfg.tile_m - 1) / cfg.tile_m) * ((p.N + cfg.tile_n - 1) / cfg.tile_n);
}

const char *f8_kernel_name(const F8Config &cfg) {
    return cfg.variant == kPingPong ? "cgemm_f8_pp_kernel" : "cgemm_f8_kernel";
}

hipError_t f8_launch(const Problem &p, const F8Config &cfg, bool mx, const void *A, const void *B, void *C,
                     const void *a_scale, const void *b_scale, hipStream_t stream) {
    const bool cil = p.c_layout == TCBF_INTERLEAVED, bl = p.a_layout == TCBF_BLOCKED;
    if (cfg.variant == kPingPong) {
        const int tiles_m = (int)((p.M + pp::TM - 1) / pp::TM);
        const int tiles_n = (int)((p.N + pp::TN - 1) / pp::TN);
        const int64_t total = pp_tiles(p);
        const int grid = (int)std::min<int64_t>(total, device_cus(p.device));
        hipLaunchKernelGGL(f8_pp_fn(cil, mx, bl), dim3((uint32_t)grid), dim3(512), 0, stream, (const uint8_t *)A,
                           (const uint8_t *)B, (float *)C, a_scale, b_scale, (int)p.M, (int)p.N, (int)f8_kp(p.K),
                           p.a_stride, tiles_m, tiles_n, (int)total);
        return hipGetLastError();
    }
    const int tiles_m = (int)((p.M + BM - 1) / BM);
    const int tiles_n = (int)((p.N + BN - 1) / BN);
    const int64_t nblocks = p.batch * tiles_m * tiles_n;
    F8Fn fn = f8_fn(cfg.variant, cil, mx, bl);
    hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(NT), 0, stream, (const uint8_t *)A, (const uint8_t *)B,
                       (float *)C, a_scale, b_scale, (int)p.M, (int)p.N, (int)f8_kp(p.K), p.a_stride, tiles_m,
                       tiles_n, (int)nblocks);
    return hipGetLastError();
}

int64_t f8_group_tiles(const Problem &p) {
    return p.batch * ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
}

hipError_t f8_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                           const void *const *SA, const void *const *SB, const int *order, int count, bool mx,
                           int c_layout, int grid, unsigned int *counter, hipStream_t stream) {
    F8GroupArgs args;
    memset(&args, 0, sizeof(args));
    int64_t first = 0;
    for (int j = 0; j < count; ++j) {
        const int i = order[j];
        const Problem &p = probs[i];
        F8GroupProblem &q = args.p[j];
        q.A = (const uint8_t *)A[i];
        q.B = (const uint8_t *)B[i];
        q.C = (float *)C[i];
        q.a_scale = SA[i];
        q.b_scale = SB[i];
        q.M = (int)p.M;
        q.N = (int)p.N;
        q.Kp = (int)f8_kp(p.K);
        q.a_shared = p.a_shared;
        q.tiles_m = (int)((p.M + BM - 1) / BM);
        q.tiles_n = (int)((p.N + BN - 1) / BN);
        q.first_tile = (int)first;
        first += f8_group_tiles(p);
    }
    args.count = count;
    args.total_tiles = (int)first;
    hipLaunchKernelGGL(f8_group_reset_kernel, dim3(1), dim3(1), 0, stream, counter);
    const bool cil = c_layout == TCBF_INTERLEAVED;
    // one operand layout per launch (the API checks it)
    const bool bl = probs[order[0]].a_layout == TCBF_BLOCKED;
    void (*fn)(const F8GroupArgs, unsigned int *) =
        bl ? (mx ? (cil ? cgemm_f8_group_kernel<1, 1, 1> : cgemm_f8_group_kernel<0, 1, 1>)
                 : (cil ? cgemm_f8_group_kernel<1, 0, 1> : cgemm_f8_group_kernel<0, 0, 1>))
           : (mx ? (cil ? cgemm_f8_group_kernel<1, 1, 0> : cgemm_f8_group_kernel<0, 1, 0>)
                 : (cil ? cgemm_f8_group_kernel<1, 0, 0> : cgemm_f8_group_kernel<0, 0, 0>));
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(NT), 0, stream, args, counter);
    return hipGetLastError();
}

}  // namespace tcbf
