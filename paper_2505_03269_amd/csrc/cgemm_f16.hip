// FP16 batched complex product B[c] = W[c] . X[c] on gfx950 MFMA.
//
// Complex product as four real products with the imaginary part of X negated
// in registers (Sec. III-B): Re += Wr.Xr + Wi.(-Xi), Im += Wr.Xi + Wi.Xr,
// fp16 x fp16 products accumulated in fp32 by v_mfma_f32_32x32x16_f16.
//
// Design (one workgroup = 256 threads = 4 waves, 128 x 128 complex outputs):
//  * per K stage (32 receivers) the workgroup loads the W tile (both planes,
//    128 x 32) and the X tile (both planes, 32 x 128) once into LDS; the four
//    real products of every wave read from that single copy (Sec. III-C data
//    reuse, at the LDS level).
//  * X arrives N-contiguous; MFMA wants 8 consecutive k per lane for both
//    operands, so the X tile is transposed to [n][k] while it is written to
//    LDS.  Interleaved (re, im) inputs are split into planes at the same
//    point, so every layout feeds the identical MFMA sequence and gives
//    bitwise-identical results.
//  * LDS holds two stages (2 x 32 KiB): global loads for stage k+1 are in
//    flight while stage k is multiplied; one barrier per stage.  Rows are
//    grouped in 128-byte lines with an XOR swizzle of the 16-byte chunks so
//    that neither the transposing writes nor the MFMA operand reads conflict.
//  * each wave owns a 64 x 64 complex sub-tile: 2 x 2 MFMA tiles of 32 x 32,
//    each with a real and an imaginary fp32 accumulator (128 registers).
//  * two workgroups per CU (64 KiB LDS, <= 256 VGPRs each) so one can drain
//    its fp32 stores while the other multiplies.
//  * workgroup ids are remapped so consecutive tiles stay on one XCD's L2.
#include "tcbf_internal.h"

namespace tcbf {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int BM = 128, BN = 128, BK = 32, NT = 256;
constexpr int PLANE_A = BM * BK;          // halves per W plane in a stage
constexpr int PLANE_B = BN * BK;          // halves per X plane in a stage
constexpr int STAGE = 2 * PLANE_A + 2 * PLANE_B;  // 16384 halves = 32 KiB

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

template <int AIL> struct ASel { typedef ALoaderPlanar T; };
template <> struct ASel<1> { typedef ALoaderInter T; };
template <int BIL> struct BSel { typedef BLoaderPlanar T; };
template <> struct BSel<1> { typedef BLoaderInter T; };

__device__ __forceinline__ half8 lds_frag(const uint16_t *plane, int row, int ch) {
    return *reinterpret_cast<const half8 *>(plane + lds_off(row, ch));
}

__device__ __forceinline__ half8 negate(half8 v) {
    u32x4 u = __builtin_bit_cast(u32x4, v);
    u ^= 0x80008000u;  // flip both fp16 sign bits: exact negation
    return __builtin_bit_cast(half8, u);
}

template <int AIL, int BIL, int CIL>
__global__ __launch_bounds__(NT, 2) void cgemm_f16_kernel(
    const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, float *__restrict__ C,
    int64_t M, int64_t N, int64_t K, int a_shared, int tiles_m, int tiles_n, int64_t nblocks,
    int a_vec, int b_vec) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];

    const int tid = threadIdx.x;
    const int64_t t = xcd_remap(blockIdx.x, nblocks);
    const int64_t per_c = (int64_t)tiles_m * tiles_n;
    const int64_t c = t / per_c;
    const int rem = (int)(t - c * per_c);
    const int tn = rem / tiles_m, tm = rem - tn * tiles_m;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

    const uint16_t *Wc = A + (a_shared ? 0 : c * 2 * M * K);
    const uint16_t *Xc = B + c * 2 * K * N;

    typename ASel<AIL>::T al;
    typename BSel<BIL>::T bl;
    al.init(Wc, M, K, m0, tid);
    bl.init(Xc, K, N, n0, tid);

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int hl = lane >> 5, l32 = lane & 31;

    f32x16 acc_r[2][2], acc_i[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc_r[i][j] = (f32x16){};
            acc_i[i][j] = (f32x16){};
        }

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
            half8 ar[2], ai[2], br[2], bi[2], bn[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                int row = wm * 64 + i * 32 + l32;
                ar[i] = lds_frag(st, row, ch);
                ai[i] = lds_frag(st + PLANE_A, row, ch);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                int col = wn * 64 + j * 32 + l32;
                br[j] = lds_frag(st + 2 * PLANE_A, col, ch);
                bi[j] = lds_frag(st + 2 * PLANE_A + PLANE_B, col, ch);
                bn[j] = negate(bi[j]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc_r[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ar[i], br[j], acc_r[i][j], 0, 0, 0);
                    acc_i[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ar[i], bi[j], acc_i[i][j], 0, 0, 0);
                    acc_r[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ai[i], bn[j], acc_r[i][j], 0, 0, 0);
                    acc_i[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ai[i], br[j], acc_i[i][j], 0, 0, 0);
                }
        }
        if (more) {
            uint16_t *nx = lds + ((kt + 1) & 1) * STAGE;
            ASel<AIL>::T::store(nx, tid, ra);
            BSel<BIL>::T::store(nx, tid, rb);
        }
        __syncthreads();
    }

    // Epilogue: 32x32 accumulator element r of lane l sits at
    // row 8*(r/4) + 4*(l/32) + r%4, column l%32.
    const bool full = (m0 + BM <= M) && (n0 + BN <= N);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = n0 + wn * 64 + j * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wm * 64 + i * 32 + (r >> 2) * 8 + hl * 4 + (r & 3);
                if (full || (row < M && col < N)) {
                    if (CIL) {
                        float2 v = make_float2(acc_r[i][j][r], acc_i[i][j][r]);
                        *reinterpret_cast<float2 *>(C + ((c * M + row) * N + col) * 2) = v;
                    } else {
                        float *o = C + c * 2 * M * N + row * N + col;
                        o[0] = acc_r[i][j][r];
                        o[M * N] = acc_i[i][j][r];
                    }
                }
            }
        }
}

typedef void (*KernFn)(const uint16_t *, const uint16_t *, float *, int64_t, int64_t, int64_t, int,
                       int, int, int64_t, int, int);

KernFn pick(int ail, int bil, int cil) {
    static const KernFn table[8] = {
        cgemm_f16_kernel<0, 0, 0>, cgemm_f16_kernel<0, 0, 1>, cgemm_f16_kernel<0, 1, 0>,
        cgemm_f16_kernel<0, 1, 1>, cgemm_f16_kernel<1, 0, 0>, cgemm_f16_kernel<1, 0, 1>,
        cgemm_f16_kernel<1, 1, 0>, cgemm_f16_kernel<1, 1, 1>,
    };
    return table[(ail << 2) | (bil << 1) | cil];
}

}  // namespace

bool f16_select(const Problem &p, int forced_variant, F16Config *cfg) {
    if (forced_variant != 0 && forced_variant != 1) return false;
    cfg->variant = 1;
    cfg->tile_m = BM;
    cfg->tile_n = BN;
    cfg->tile_k = BK;
    cfg->threads = NT;
    // 16-byte loads need every row start 16-byte aligned (base pointers are
    // required to be 16-byte aligned by the ABI).
    cfg->a_vec = p.a_layout == TCBF_PLANAR ? (p.K % 8 == 0) : (p.K % 4 == 0);
    cfg->b_vec = p.b_layout == TCBF_PLANAR ? (p.N % 8 == 0) : (p.N % 4 == 0);
    return true;
}

int64_t f16_workgroups(const Problem &p, const F16Config &cfg) {
    int64_t tm = (p.M + cfg.tile_m - 1) / cfg.tile_m;
    int64_t tn = (p.N + cfg.tile_n - 1) / cfg.tile_n;
    return p.batch * tm * tn;
}

const char *f16_kernel_name(const F16Config &) { return "cgemm_f16_kernel"; }

hipError_t f16_launch(const Problem &p, const F16Config &cfg, const void *A, const void *B,
                      void *C, hipStream_t stream) {
    int tiles_m = (int)((p.M + BM - 1) / BM);
    int tiles_n = (int)((p.N + BN - 1) / BN);
    int64_t nblocks = p.batch * tiles_m * tiles_n;
    KernFn fn = pick(p.a_layout == TCBF_INTERLEAVED, p.b_layout == TCBF_INTERLEAVED,
                     p.c_layout == TCBF_INTERLEAVED);
    hipLaunchKernelGGL(fn, dim3((uint32_t)nblocks), dim3(NT), 0, stream,
                       (const uint16_t *)A, (const uint16_t *)B, (float *)C, p.M, p.N, p.K,
                       p.a_shared, tiles_m, tiles_n, nblocks, (int)cfg.a_vec, (int)cfg.b_vec);
    return hipGetLastError();
}

}  // namespace tcbf
