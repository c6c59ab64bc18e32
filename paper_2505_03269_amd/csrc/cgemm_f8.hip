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
// Workgroup: 128 beams x 128 samples, 4 waves in a 2 x 2 grid of 64 x 64
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

constexpr int kNumVariants = 2;  // 1: two-stage ring (default), 2: three-stage ring

}  // namespace

int64_t f8_kp(int64_t K) { return (K + 31) / 32 * 32; }

bool f8_select(const Problem &p, int forced_variant, F8Config *cfg) {
    int v = forced_variant == 0 ? 1 : forced_variant;
    if (v < 1 || v > kNumVariants) return false;
    if (p.N % 4 != 0) return false;
    // both operands planar, or both receiver-blocked
    if (p.a_layout != p.b_layout || (p.a_layout != TCBF_PLANAR && p.a_layout != TCBF_BLOCKED)) return false;
    cfg->variant = v;
    cfg->tile_m = BM;
    cfg->tile_n = BN;
    cfg->tile_k = BK;
    cfg->threads = NT;
    return true;
}

int64_t f8_workgroups(const Problem &p, const F8Config &cfg) {
    return p.batch * ((p.M + cfg.tile_m - 1) / cfg.tile_m) * ((p.N + cfg.tile_n - 1) / cfg.tile_n);
}

const char *f8_kernel_name(const F8Config &) { return "cgemm_f8_kernel"; }

hipError_t f8_launch(const Problem &p, const F8Config &cfg, bool mx, const void *A, const void *B, void *C,
                     const void *a_scale, const void *b_scale, hipStream_t stream) {
    const int tiles_m = (int)((p.M + BM - 1) / BM);
    const int tiles_n = (int)((p.N + BN - 1) / BN);
    const int64_t nblocks = p.batch * tiles_m * tiles_n;
    F8Fn fn = f8_fn(cfg.variant, p.c_layout == TCBF_INTERLEAVED, mx, p.a_layout == TCBF_BLOCKED);
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
