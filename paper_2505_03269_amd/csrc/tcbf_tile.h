// Device-side pieces shared by the matrix-unit kernels: the 128 x 128 complex
// workgroup tile's accumulator layout, buffer-descriptor helpers, LDS-only
// barriers and the LDS-staged epilogue that writes whole output rows.
#pragma once

#include "tcbf_internal.h"

namespace tcbf {
namespace tile {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

#define TCBF_LDS_AS __attribute__((address_space(3)))

constexpr int BM = 128, BN = 128, NT = 256;  // complex outputs per workgroup, threads
constexpr uint32_t OOB = 0x80000000u;         // buffer offset past every range: reads 0, writes dropped
constexpr int RSRC_FLAGS = 0x00020000;        // raw buffer, 32-bit data format (gfx9 family)
// Cache policy of the output stores: non-temporal.  The output is written
// once and never read back by the kernel; marking it streaming keeps it from
// displacing the operand tiles other workgroups re-read from L2 (measured on
// the radio-astronomy fp16 shape: 1.7% faster, results identical).
constexpr int kStoreStreaming = 2;

// s_waitcnt immediates (gfx9 encoding: vmcnt bits [3:0] and [15:14], expcnt
// [6:4], lgkmcnt [11:8]); fields not named are left at their maxima.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int kWaitLds = 15 | (3 << 14) | (7 << 4);  // lgkmcnt(0)

// Workgroup barrier for LDS-only hazards: this wave's LDS accesses are
// complete, then a bare s_barrier (no release fence, so outstanding global
// stores and loads are not waited for).  The clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(kWaitLds);
    asm volatile("s_barrier" ::: "memory");
}

// Accumulators of one wave (the workgroup's 4 waves form a 2 x 2 grid of
// 64 x 64 blocks: beams wm*64.., samples wn*64.. with wm = wave/2, wn = wave%2).
// [i: 32-beam sub-tile][j: 32-sample sub-tile]; element r of lane l holds beam
// i*32 + l%32 and samples j*32 + 8*(r/4) + 4*(l/32) + r%4, i.e. each lane owns
// runs of four consecutive samples of one beam.
struct Acc {
    f32x16 re[2][2], im[2][2];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                re[i][j] = (f32x16){};
                im[i][j] = (f32x16){};
            }
    }
};

// Four consecutive accumulator elements 4q..4q+3 (a sub-register view).
__device__ __forceinline__ f32x4 quad(const f32x16 &v, int q) {
    switch (q) {
    case 0: return __builtin_shufflevector(v, v, 0, 1, 2, 3);
    case 1: return __builtin_shufflevector(v, v, 4, 5, 6, 7);
    case 2: return __builtin_shufflevector(v, v, 8, 9, 10, 11);
    default: return __builtin_shufflevector(v, v, 12, 13, 14, 15);
    }
}

// Epilogue: write the workgroup's finished tile (each wave's Acc) to C,
// staged through LDS so every store instruction writes whole rows: a planar
// plane row is 128 samples x 4 B = 512 B, an interleaved row 128 x 8 B = 1 KiB.
// The workgroup has 2*WM waves in a WM x 2 grid (wave w: beams (w/2)*64..,
// samples (w%2)*64..), so the tile is 64*WM beams x 128 samples.
// Staged rows keep their 16-byte chunks XOR-swizzled by (row % 32) so both the
// writes (32 beams, same samples) and the row reads avoid bank conflicts.
// Planar: round p stages plane p of the whole tile (64*WM rows).  Interleaved:
// round h stages the upper or lower half of the beams (32*WM rows) with
// (re, im) pairs.  row_ptr(row) must map every staged row of a round, PITCH
// bytes each, to idle LDS.  C: this channel's output; rows past M and samples
// past N are dropped through the buffer range check (N a multiple of 4).
template <int CIL> constexpr int staging_pitch() { return CIL ? 1024 : 512; }
template <int WM, int CIL> constexpr int staging_rows() { return CIL ? 32 * WM : 64 * WM; }

template <int WM, int CIL, typename RowPtr>
__device__ __forceinline__ void store_tile_staged(const Acc &acc, RowPtr row_ptr, float *Cc, int M, int N,
                                                  int m0, int n0, int wave, int lane) {
    constexpr int NW = 2 * WM, HALF = WM / 2;
    static_assert(WM % 2 == 0, "whole beam halves");
    const int wm = wave >> 1, wn = wave & 1, hl = lane >> 5, l32 = lane & 31;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)Cc, 0, 8 * M * N, RSRC_FLAGS);
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        lds_barrier();  // staging area free (main loop or previous round done)
        if (!CIL || wm / HALF == round) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = (CIL ? (wm % HALF) * 64 : wm * 64) + 32 * i + l32;
                char *rp = row_ptr(row);
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int n = wn * 64 + 32 * j + 8 * q + 4 * hl;  // first of 4 samples
                        if (CIL) {
                            const f32x4 re = quad(acc.re[i][j], q), im = quad(acc.im[i][j], q);
                            const int ch = n >> 1;  // two 16-byte chunks: samples n, n+1 and n+2, n+3
                            *reinterpret_cast<f32x4 *>(rp + ((ch ^ (row & 31)) * 16)) =
                                (f32x4){re[0], im[0], re[1], im[1]};
                            *reinterpret_cast<f32x4 *>(rp + (((ch + 1) ^ (row & 31)) * 16)) =
                                (f32x4){re[2], im[2], re[3], im[3]};
                        } else {
                            const f32x4 v = round == 0 ? quad(acc.re[i][j], q) : quad(acc.im[i][j], q);
                            *reinterpret_cast<f32x4 *>(rp + (((n >> 2) ^ (row & 31)) * 16)) = v;
                        }
                    }
            }
        }
        lds_barrier();  // round staged
        if (CIL) {
            // 32*WM rows of 1 KiB; wave w stores rows w, w+NW, ...; lane l owns chunk l
#pragma unroll 4
            for (int t = 0; t < 32 * WM / NW; ++t) {
                const int row = wave + NW * t;
                const f32x4 v = *reinterpret_cast<const f32x4 *>(row_ptr(row) + ((lane ^ (row & 31)) * 16));
                const int m = m0 + 32 * WM * round + row, n = n0 + 2 * lane;
                const uint32_t off = (m < M && n < N) ? (uint32_t)((m * N + n) * 8) : OOB;
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rc, off, 0, kStoreStreaming);
            }
        } else {
            // 64*WM rows of 512 B; one instruction covers two rows; wave w
            // stores rows 32w..32w+31
#pragma unroll 4
            for (int t = 0; t < 64 * WM / (2 * NW); ++t) {
                const int row = 32 * wave + 2 * t + hl;
                const f32x4 v = *reinterpret_cast<const f32x4 *>(row_ptr(row) + ((l32 ^ (row & 31)) * 16));
                const int m = m0 + row, n = n0 + 4 * l32;
                // the plane offset goes into the per-lane offset: a buffer
                // store with a register soffset gets no protection from the
                // compiler against its data registers being overwritten by
                // the very next instruction, which corrupts the stored data
                const uint32_t off = (m < M && n < N) ? (uint32_t)((round * M * N + m * N + n) * 4) : OOB;
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rc, off, 0, kStoreStreaming);
            }
        }
    }
}

}  // namespace tile
}  // namespace tcbf
