// Weight repack into the receiver-blocked layout read by the fp16 kernel.
//
// The paper's library needs its input matrices tiled in device memory and
// provides a transpose kernel for that; for the weights (the model matrix)
// this happens once, before the data stream starts (Sec. III, Sec. V-A).
// Here the tiling is along the receiver axis only: per plane, blocks of 32
// receivers, each block holding all M beam rows of 32 receivers (64 bytes).
// A 128-beam x 32-receiver tile of the product kernel is then one contiguous
// 8 KiB run per plane instead of 128 separate 64-byte pieces.
//
// One thread writes one 64-byte block row (beam m, block kb, plane p of
// channel b): consecutive threads take consecutive beams, so the stores of a
// wave are one contiguous 4 KiB run.  Receivers k >= K are written as zero.
// A pure data movement: the values are copied bit for bit.
#include "tcbf_internal.h"

namespace tcbf {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int NT = 256;

template <int IL, int VEC>
__global__ __launch_bounds__(NT) void block_weights_kernel(const uint16_t *__restrict__ src,
                                                           uint16_t *__restrict__ dst, int64_t batch, int64_t M,
                                                           int64_t K, int64_t kb_count, int64_t rows_total) {
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (r >= rows_total) return;
    const int64_t m = r % M;
    const int64_t kb = (r / M) % kb_count;
    const int64_t bp = r / (M * kb_count);  // channel * 2 + plane
    const int64_t b = bp >> 1, p = bp & 1;
    const int64_t k0 = kb * 32;
    uint16_t v[32];
    if (VEC) {
        // K a multiple of 8: every 8-receiver chunk is wholly inside or past K
        if (!IL) {
            const uint16_t *row = src + (bp * M + m) * K;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                u32x4 w = k0 + 8 * c < K ? *reinterpret_cast<const u32x4 *>(row + k0 + 8 * c) : (u32x4){0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[8 * c + 2 * j] = (uint16_t)(w[j] & 0xffffu);
                    v[8 * c + 2 * j + 1] = (uint16_t)(w[j] >> 16);
                }
            }
        } else {
            // interleaved (re, im) pairs: 8 receivers = 32 bytes, keep plane p
            const uint16_t *row = src + (b * M + m) * K * 2;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                u32x4 w = k0 + 4 * c < K ? *reinterpret_cast<const u32x4 *>(row + (k0 + 4 * c) * 2)
                                         : (u32x4){0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 4; ++j) v[4 * c + j] = (uint16_t)(p ? (w[j] >> 16) : (w[j] & 0xffffu));
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int64_t k = k0 + j;
            uint16_t x = 0;
            if (k < K) x = IL ? src[((b * M + m) * K + k) * 2 + p] : src[(bp * M + m) * K + k];
            v[j] = x;
        }
    }
    u32x4 *out = reinterpret_cast<u32x4 *>(dst + ((bp * kb_count + kb) * M + m) * 32);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        u32x4 w;
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = (uint32_t)v[8 * c + 2 * j] | ((uint32_t)v[8 * c + 2 * j + 1] << 16);
        out[c] = w;
    }
}

}  // namespace

int64_t block_weights_workgroups(int64_t batch, int64_t M, int64_t K) {
    const int64_t rows = batch * 2 * ((K + 31) / 32) * M;
    return (rows + NT - 1) / NT;
}

hipError_t block_weights_launch(const void *src, int src_layout, int64_t batch, int64_t M, int64_t K, void *dst,
                                hipStream_t stream) {
    const int64_t kb_count = (K + 31) / 32;
    const int64_t rows = batch * 2 * kb_count * M;
    const int64_t blocks = block_weights_workgroups(batch, M, K);
    const bool il = src_layout == TCBF_INTERLEAVED;
    // vector reads need 16-byte aligned 8-receiver (planar) or 4-receiver
    // (interleaved) chunks: row starts are then 16-byte aligned too
    const bool vec = il ? (K % 4 == 0) : (K % 8 == 0);
    typedef void (*Fn)(const uint16_t *, uint16_t *, int64_t, int64_t, int64_t, int64_t, int64_t);
    const Fn fn = il ? (vec ? block_weights_kernel<1, 1> : block_weights_kernel<1, 0>)
                     : (vec ? block_weights_kernel<0, 1> : block_weights_kernel<0, 0>);
    hipLaunchKernelGGL(fn, dim3((uint32_t)blocks), dim3(NT), 0, stream, (const uint16_t *)src, (uint16_t *)dst,
                       batch, M, K, kb_count, rows);
    return hipGetLastError();
}

}  // namespace tcbf
