// FP8 (OCP e4m3) quantisation of complex operands for the 8-bit path.  The
// paper leaves 8-bit floats as future work (Sec. VI); the format and the two
// scale granularities are the library's own choices:
//
//  * per-row (block == 0): one fp32 scale per complex row, shared by the real
//    and imaginary parts, computed in fp32 as
//        amax  = max |x| over the row's re and im parts (NaN ignored)
//        scale = amax / 448        (1 when amax == 0)
//        inv   = 448 / amax        (1 when amax == 0)
//        q     = e4m3 nearest-even of (x * inv), saturating at +-448
//  * per-block (block == 32, the OCP MX layout): one E8M0 scale 2^e per
//    complex row and 32-receiver block, e the smallest integer with
//    amax <= 448 * 2^e (clamped to [-127, 127]; 0 for an all-zero block),
//        q = e4m3 nearest-even of ldexp(x, -e)   (exact scaling by 2^-e)
//
// Destination: [batch][2][rows][Kp] e4m3 bytes, Kp = 32 * ceil(K / 32), bytes
// past K zero.  Scales: per-row fp32 [batch][rows]; per-block uint8 E8M0
// [batch][Ks / 16][rows][16] (value 2^(code - 127), block kb of row r at
// [kb / 16][r][kb % 16]), Ks = mx_scale_pitch(Kp); the padding codes past
// Kp / 32 are not written.
//
// Work is cut into tiles of 64 rows x 64 receivers.  The tile loads follow the
// source's contiguous axis (receivers for K-major W, rows for N-major X), the
// codes are transposed through LDS and stored as whole 16-byte row pieces.
// Per-row scales need the whole row first: a max pass (integer atomic max on
// the non-negative fp32 bit patterns, so the order of arrival cannot change
// the result), the quantise pass, then amax -> scale in place.
#include "tcbf_internal.h"

namespace tcbf {
namespace {

constexpr int NT = 256;
constexpr int TR = 64, TK = 64;  // tile: rows x receivers
constexpr int QPITCH = TK + 16;   // LDS code row pitch (keeps 16-byte alignment)

template <typename T> struct Val;
template <> struct Val<int8_t> { static __device__ float get(const int8_t *p) { return (float)*p; } };
template <> struct Val<_Float16> { static __device__ float get(const _Float16 *p) { return (float)*p; } };
template <> struct Val<float> { static __device__ float get(const float *p) { return *p; } };

// Nearest e4m3 code of y, ties to an even mantissa, magnitudes above 448
// saturate to 448, NaN gives 0x7f.  Written from the format's definition:
// subnormals are multiples of 2^-9 below 2^-6; normal values keep 3 fraction
// bits, so rounding the fp32 pattern at bit 20 gives exponent and mantissa
// together (a carry moves to the next binade).
__device__ __forceinline__ uint32_t e4m3_code(float y) {
    const uint32_t b = __float_as_uint(y);
    const uint32_t sign = (b >> 24) & 0x80u;
    const uint32_t a = b & 0x7fffffffu;
    if (a > 0x7f800000u) return 0x7fu;
    uint32_t code;
    if (a >= 0x43e00000u) {                      // >= 448 (includes infinity)
        code = 0x7eu;
    } else if (a < 0x3c800000u) {                // below 2^-6: subnormal grid
        code = (uint32_t)rintf(__uint_as_float(a) * 512.0f);  // 0..8; 8 is 2^-6
    } else {
        const uint32_t r = a + 0x7ffffu + ((a >> 20) & 1u);
        code = (r >> 20) - (120u << 3);          // rebias 127 -> 7
        if (code > 0x7eu) code = 0x7eu;
    }
    return sign | code;
}

// Smallest e with amax <= 448 * 2^e, as described above.
__device__ __forceinline__ int mx_exponent(float amax) {
    if (!(amax > 0.0f)) return 0;
    if (__builtin_isinf(amax)) return 127;       // no finite e exists: the clamp
    int x;
    const float f = frexpf(amax, &x);            // amax = f * 2^x, f in [0.5, 1)
    int e = (x - 9) + (2.0f * f > 1.75f ? 1 : 0);
    return e < -127 ? -127 : (e > 127 ? 127 : e);
}

__device__ __forceinline__ float magnitude(float v) {
    const float a = fabsf(v);
    return a == a ? a : 0.0f;  // NaN never wins the max
}

struct TileIdx {
    int64_t b, r0, k0;
};
__device__ __forceinline__ TileIdx tile_of(int64_t bid, int64_t rows, int64_t kp) {
    const int64_t rt = (rows + TR - 1) / TR, kt = (kp + TK - 1) / TK;
    TileIdx t;
    t.k0 = (bid % kt) * TK;
    t.r0 = ((bid / kt) % rt) * TR;
    t.b = bid / (kt * rt);
    return t;
}

// Element (row, k) of plane p in batch entry b.
template <typename T, int IL, int KMAJ>
__device__ __forceinline__ float load_el(const T *src, int64_t b, int p, int64_t row, int64_t k, int64_t rows,
                                         int64_t K) {
    int64_t idx;
    if (KMAJ) idx = IL ? ((b * rows + row) * K + k) * 2 + p : ((b * 2 + p) * rows + row) * K + k;
    else idx = IL ? ((b * K + k) * rows + row) * 2 + p : ((b * 2 + p) * K + k) * rows + row;
    return Val<T>::get(src + idx);
}

// Thread t covers the 16 elements (row, k) of its tile with
//   K-major: k = k0 + t%64, row = r0 + t/64 + 4s      (lanes along receivers)
//   N-major: row = r0 + t%64, k = k0 + t/64 + 4s      (lanes along rows)
// for s = 0..15, so every wave load is contiguous in the source.
template <int KMAJ> __device__ __forceinline__ int el_row(int t, int s) { return KMAJ ? (t >> 6) + 4 * s : (t & 63); }
template <int KMAJ> __device__ __forceinline__ int el_k(int t, int s) { return KMAJ ? (t & 63) : (t >> 6) + 4 * s; }

template <typename T, int IL, int KMAJ>
__device__ __forceinline__ void load_tile(const T *src, const TileIdx &ti, int64_t rows, int64_t K, int t,
                                          float (&vr)[16], float (&vi)[16]) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int64_t row = ti.r0 + el_row<KMAJ>(t, s), k = ti.k0 + el_k<KMAJ>(t, s);
        const bool in = row < rows && k < K;
        vr[s] = in ? load_el<T, IL, KMAJ>(src, ti.b, 0, row, k, rows, K) : 0.0f;
        vi[s] = in ? load_el<T, IL, KMAJ>(src, ti.b, 1, row, k, rows, K) : 0.0f;
    }
}

__global__ __launch_bounds__(NT) void fill_zero_kernel(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Per-row pass 1: amax of each row, as fp32 bits, folded into amax_bits.
template <typename T, int IL, int KMAJ>
__global__ __launch_bounds__(NT) void row_amax_kernel(const T *__restrict__ src, uint32_t *__restrict__ amax_bits,
                                                      int64_t rows, int64_t K, int64_t kp) {
    __shared__ uint32_t part[TR];
    const int t = threadIdx.x;
    const TileIdx ti = tile_of(blockIdx.x, rows, kp);
    if (t < TR) part[t] = 0u;
    __syncthreads();
    float vr[16], vi[16];
    load_tile<T, IL, KMAJ>(src, ti, rows, K, t, vr, vi);
    if (KMAJ) {
        // the wave's 64 lanes share a row per s: reduce across lanes
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            float m = fmaxf(magnitude(vr[s]), magnitude(vi[s]));
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
            if ((t & 63) == 0) atomicMax(&part[el_row<KMAJ>(t, s)], __float_as_uint(m));
        }
    } else {
        float m = 0.0f;
#pragma unroll
        for (int s = 0; s < 16; ++s) m = fmaxf(m, fmaxf(magnitude(vr[s]), magnitude(vi[s])));
        atomicMax(&part[t & 63], __float_as_uint(m));
    }
    __syncthreads();
    if (t < TR && ti.r0 + t < rows && part[t] != 0u) atomicMax(&amax_bits[ti.b * rows + ti.r0 + t], part[t]);
}

// Per-row pass 3: amax -> scale, in place.
__global__ __launch_bounds__(NT) void row_scale_kernel(float *scales, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) {
        const float amax = scales[i];
        scales[i] = amax > 0.0f ? amax / 448.0f : 1.0f;
    }
}

// Quantise one tile.  MX == 0: row scales from the finished amax pass;
// MX == 1: block exponents computed here (a tile holds two whole blocks).
// BL: codes written in the receiver-blocked layout [b][2][ceil(kp/64)][rows][64]
// (one tile is one 64-receiver block of 64 rows: 4 KiB contiguous per plane);
// bytes past kp in the last block are written as zero codes too.
template <typename T, int IL, int KMAJ, int MX, int BL>
__global__ __launch_bounds__(NT) void quantize_kernel(const T *__restrict__ src, uint8_t *__restrict__ dst,
                                                      void *__restrict__ scales, int64_t rows, int64_t K,
                                                      int64_t kp) {
    __shared__ __attribute__((aligned(16))) uint8_t q[2][TR][QPITCH];
    __shared__ float rowinv[TR];
    __shared__ uint32_t bmax[TR][2];
    const int t = threadIdx.x;
    const TileIdx ti = tile_of(blockIdx.x, rows, kp);
    float vr[16], vi[16];
    load_tile<T, IL, KMAJ>(src, ti, rows, K, t, vr, vi);

    if (!MX) {
        if (t < TR) {
            const int64_t row = ti.r0 + t;
            const float amax = row < rows ? ((const float *)scales)[ti.b * rows + row] : 0.0f;
            rowinv[t] = amax > 0.0f ? 448.0f / amax : 1.0f;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int r = el_row<KMAJ>(t, s), k = el_k<KMAJ>(t, s);
            const float inv = rowinv[r];
            q[0][r][k] = (uint8_t)e4m3_code(vr[s] * inv);
            q[1][r][k] = (uint8_t)e4m3_code(vi[s] * inv);
        }
    } else {
        if (t < TR) bmax[t][0] = bmax[t][1] = 0u;
        __syncthreads();
        if (KMAJ) {
            // lanes 0..31 hold block 0 of the row, lanes 32..63 block 1
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                float m = fmaxf(magnitude(vr[s]), magnitude(vi[s]));
#pragma unroll
                for (int d = 16; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
                if ((t & 31) == 0) bmax[el_row<KMAJ>(t, s)][(t >> 5) & 1] = __float_as_uint(m);
            }
        } else {
            // k = t/64 + 4s: s < 8 is block 0, s >= 8 block 1
            float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const float m = fmaxf(magnitude(vr[s]), magnitude(vi[s]));
                if (s < 8) m0 = fmaxf(m0, m);
                else m1 = fmaxf(m1, m);
            }
            atomicMax(&bmax[t & 63][0], __float_as_uint(m0));
            atomicMax(&bmax[t & 63][1], __float_as_uint(m1));
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int r = el_row<KMAJ>(t, s), k = el_k<KMAJ>(t, s);
            const int e = mx_exponent(__uint_as_float(bmax[r][k >> 5]));
            q[0][r][k] = (uint8_t)e4m3_code(ldexpf(vr[s], -e));
            q[1][r][k] = (uint8_t)e4m3_code(ldexpf(vi[s], -e));
        }
        if (t < 2 * TR) {
            const int r = t >> 1, blk = t & 1;
            const int64_t row = ti.r0 + r, kb = ti.k0 / 32 + blk;
            if (row < rows && kb < kp / 32)
                ((uint8_t *)scales)[((ti.b * (mx_scale_pitch(kp) / 16) + kb / 16) * rows + row) * 16 + kb % 16] =
                    (uint8_t)(mx_exponent(__uint_as_float(bmax[r][blk])) + 127);
        }
    }
    __syncthreads();
    // 2 planes x 64 rows x 4 pieces of 16 bytes: two per thread
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = t + h * NT;
        const int p = c >> 8, r = (c >> 2) & 63, piece = c & 3;
        const int64_t row = ti.r0 + r, k = ti.k0 + 16 * piece;
        if (BL) {
            static_assert(TK == 64, "one tile per 64-receiver block");
            const int64_t nblk = (kp + 63) / 64;
            if (row < rows) {
                const uint4 v = *reinterpret_cast<const uint4 *>(&q[p][r][16 * piece]);
                *reinterpret_cast<uint4 *>(dst + (((ti.b * 2 + p) * nblk + ti.k0 / 64) * rows + row) * 64 +
                                           16 * piece) = v;
            }
        } else if (row < rows && k < kp) {
            const uint4 v = *reinterpret_cast<const uint4 *>(&q[p][r][16 * piece]);
            *reinterpret_cast<uint4 *>(dst + ((ti.b * 2 + p) * rows + row) * kp + k) = v;
        }
    }
}

template <typename T, int IL, int KMAJ, int BL>
hipError_t quantize_typed(const void *src, int64_t batch, int64_t rows, int64_t K, int block, uint8_t *dst,
                          void *scales, hipStream_t stream) {
    const int64_t kp = (K + 31) / 32 * 32;
    const int64_t tiles = batch * ((rows + TR - 1) / TR) * ((kp + TK - 1) / TK);
    const T *s = (const T *)src;
    if (block == 32) {
        hipLaunchKernelGGL((quantize_kernel<T, IL, KMAJ, 1, BL>), dim3((uint32_t)tiles), dim3(NT), 0, stream, s, dst,
                           scales, rows, K, kp);
        return hipGetLastError();
    }
    const int64_t n = batch * rows;
    const uint32_t nb = (uint32_t)((n + NT - 1) / NT);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nb), dim3(NT), 0, stream, (uint32_t *)scales, n);
    hipLaunchKernelGGL((row_amax_kernel<T, IL, KMAJ>), dim3((uint32_t)tiles), dim3(NT), 0, stream, s,
                       (uint32_t *)scales, rows, K, kp);
    hipLaunchKernelGGL((quantize_kernel<T, IL, KMAJ, 0, BL>), dim3((uint32_t)tiles), dim3(NT), 0, stream, s, dst,
                       scales, rows, K, kp);
    hipLaunchKernelGGL(row_scale_kernel, dim3(nb), dim3(NT), 0, stream, (float *)scales, n);
    return hipGetLastError();
}

template <typename T, int BL>
hipError_t quantize_layout(const void *src, int il, int kmaj, int64_t batch, int64_t rows, int64_t K, int block,
                           uint8_t *dst, void *scales, hipStream_t stream) {
    if (il) return kmaj ? quantize_typed<T, 1, 1, BL>(src, batch, rows, K, block, dst, scales, stream)
                        : quantize_typed<T, 1, 0, BL>(src, batch, rows, K, block, dst, scales, stream);
    return kmaj ? quantize_typed<T, 0, 1, BL>(src, batch, rows, K, block, dst, scales, stream)
                : quantize_typed<T, 0, 0, BL>(src, batch, rows, K, block, dst, scales, stream);
}

template <int BL>
hipError_t quantize_any(const void *src, int src_type, int il, int kmaj, int64_t batch, int64_t rows, int64_t K,
                        int block, uint8_t *dst, void *scales, hipStream_t stream) {
    switch (src_type) {
    case TCBF_SRC_I8: return quantize_layout<int8_t, BL>(src, il, kmaj, batch, rows, K, block, dst, scales, stream);
    case TCBF_SRC_F16:
        return quantize_layout<_Float16, BL>(src, il, kmaj, batch, rows, K, block, dst, scales, stream);
    default: return quantize_layout<float, BL>(src, il, kmaj, batch, rows, K, block, dst, scales, stream);
    }
}

}  // namespace

int64_t quantize_e4m3_tiles(int64_t batch, int64_t rows, int64_t K) {
    const int64_t kp = (K + 31) / 32 * 32;
    return batch * ((rows + TR - 1) / TR) * ((kp + TK - 1) / TK);
}

hipError_t quantize_e4m3_launch(const void *src, int src_type, int src_layout, int64_t batch, int64_t rows,
                                int64_t K, int src_k_major, int block, int dst_layout, uint8_t *dst, void *scales,
                                hipStream_t stream) {
    const int il = src_layout == TCBF_INTERLEAVED;
    if (dst_layout == TCBF_BLOCKED)
        return quantize_any<1>(src, src_type, il, src_k_major, batch, rows, K, block, dst, scales, stream);
    return quantize_any<0>(src, src_type, il, src_k_major, batch, rows, K, block, dst, scales, stream);
}

}  // namespace tcbf
