// Internal declarations shared by the library's translation units (not part
// of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tcbf.h"

namespace tcbf {

// Compute units of a device (the persistent kernels run one workgroup on
// each); 256, the MI355X's count, when the runtime cannot say.
int device_cus(int device);

// Geometry a launcher needs; filled by the plan from the public descriptor.
struct Problem {
    int64_t batch, M, N, K;
    int a_layout, b_layout, c_layout;  // tcbf_layout
    int a_shared;
    int device;  // HIP device ordinal the problem runs on
    // W storage elements (fp16 values, code bytes, packed words) from one
    // batch entry's W to the next: 0 for a shared W, else at least one
    // entry (set by the API layer from the descriptor)
    int64_t a_stride;
    int b_kmajor;  // fp16 X receiver-contiguous ([N][K] per plane)
    int bf16;      // 16-bit operands are bfloat16 (TCBF_BF16), not fp16
};
// W storage elements of one batch entry in the given layout.
int64_t w_entry_elems(int dtype, int a_layout, int64_t M, int64_t K);

// FP16 mode (16-bit in, fp32 out).
struct F16Config {
    int variant;
    int tile_m, tile_n, tile_k, threads;
    bool a_vec, b_vec;  // 16-byte vector loads allowed for W / X rows
};
bool f16_select(const Problem &p, int forced_variant, F16Config *cfg);
int64_t f16_workgroups(const Problem &p, const F16Config &cfg);
const char *f16_kernel_name(const F16Config &cfg);
hipError_t f16_launch(const Problem &p, const F16Config &cfg, const void *A, const void *B,
                      void *C, hipStream_t stream);

// Grouped persistent fp16 launch: problems of different shapes share one
// launch; `order` lists the problems in queue order.
bool f16_group_problem_ok(const Problem &p);
int64_t f16_group_tiles(const Problem &p);
// Per-problem fp16 variants: 6, 7 and 9 (256-beam tiles) run in a grouped
// ping-pong launch, the others in the grouped 128 x 128 launch (the tile
// counter is used by the latter only); one launch per kind present.
bool f16_group_pp(int variant);
hipError_t f16_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                            const int *order, const int *variants, int count, int c_layout, int cus,
                            unsigned int *counter, hipStream_t stream);

// FP8 modes (e4m3 codes in, fp32 out): per-row fp32 scales or per-32-block
// E8M0 scales (mx).  Operands are receiver-contiguous with row pitch f8_kp(K).
struct F8Config {
    int variant;  // 1 = two-stage ring, 2 = three-stage ring, 3 = ping-pong persistent
    int tile_m, tile_n, tile_k, threads;
};
int64_t f8_kp(int64_t K);
// Per-row count of per-block E8M0 scale codes for a code row pitch of kp
// bytes: kp / 32 block codes, padded to a multiple of 16 (the scales are
// stored in groups of 16 codes per row, [Ks / 16][rows][16], so the product
// kernel moves one group of consecutive rows with contiguous loads).
__host__ __device__ inline int64_t mx_scale_pitch(int64_t kp) { return (kp / 32 + 15) / 16 * 16; }
bool f8_select(const Problem &p, bool mx, int forced_variant, F8Config *cfg);
int64_t f8_workgroups(const Problem &p, const F8Config &cfg);
const char *f8_kernel_name(const F8Config &cfg);
// Grouped FP8 launch (per-row or per-block scales, one kind per launch).
int64_t f8_group_tiles(const Problem &p);
hipError_t f8_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                           const void *const *SA, const void *const *SB, const int *order, int count, bool mx,
                           int c_layout, int grid, unsigned int *counter, hipStream_t stream);
hipError_t f8_launch(const Problem &p, const F8Config &cfg, bool mx, const void *A, const void *B, void *C,
                     const void *a_scale, const void *b_scale, hipStream_t stream);

// e4m3 quantisation (block 0: per-row fp32 scales, 32: per-block E8M0).
int64_t quantize_e4m3_tiles(int64_t batch, int64_t rows, int64_t K);
hipError_t quantize_e4m3_launch(const void *src, int src_type, int src_layout, int64_t batch, int64_t rows,
                                int64_t K, int src_k_major, int block, int dst_layout, uint8_t *dst, void *scales,
                                hipStream_t stream);

// Steering weights from geometry (FP64 phases; fp16 or fp32 planar out, or
// fp16 receiver-blocked).
int64_t steering_blocks(int64_t batch, int64_t M, int64_t K, int blocked);
hipError_t steering_launch(const double *pos, const double *dir, const double *freq, double speed, int64_t batch,
                           int64_t M, int64_t K, int out_type, int out_layout, void *out, hipStream_t stream);

// 1-bit mode (packed sign bits in, int32 out).
struct Int1Config {
    int variant;  // 1 = int8 MFMA on unpacked bits, 2 = VALU xor/popcount
    int tile_m, tile_n, tile_kw, threads;
};
bool int1_select(const Problem &p, int forced_variant, Int1Config *cfg);
int64_t int1_workgroups(const Problem &p, const Int1Config &cfg);
const char *int1_kernel_name(const Int1Config &cfg);
// Grouped launch of the int8-MFMA 1-bit variant.
int64_t int1_group_tiles(const Problem &p);
hipError_t int1_group_launch(const Problem *probs, const void *const *A, const void *const *B, void *const *C,
                             const int *order, int count, int c_layout, int grid, unsigned int *counter,
                             hipStream_t stream);
hipError_t int1_launch(const Problem &p, const Int1Config &cfg, const uint32_t *A,
                       const uint32_t *B, int32_t *C, hipStream_t stream);

// Weight repack into the receiver-blocked layout (TCBF_BLOCKED).
int64_t block_weights_workgroups(int64_t batch, int64_t M, int64_t K);
hipError_t block_weights_launch(const void *src, int src_layout, int64_t batch, int64_t M, int64_t K, void *dst,
                                hipStream_t stream);

// Sign packing.
// Workgroups the packing launch uses (what the argument checks bound).
int64_t pack1bit_workgroups(int src_type, int64_t batch, int64_t rows, int64_t K, int src_k_major);
hipError_t pack1bit_launch(const void *src, int src_type, int src_layout, int64_t batch,
                           int64_t rows, int64_t K, int src_k_major, uint32_t *dst,
                           hipStream_t stream);

// Coordinates of tile `rem` of one channel.  Consecutive tiles walk the
// dimension with fewer tiles first, so the workgroups that run at the same
// time on one XCD (see xcd_remap) share an operand block: with few beam tiles
// they share an X column block, with few sample tiles (tall, narrow problems)
// a W row block, which then comes from HBM once instead of once per column.
__device__ __forceinline__ void tile_coords(int rem, int tiles_m, int tiles_n, int &tm, int &tn) {
    if (tiles_n < tiles_m) {
        tm = rem / tiles_n;
        tn = rem - tm * tiles_n;
    } else {
        tn = rem / tiles_m;
        tm = rem - tn * tiles_m;
    }
}

// Workgroup order: consecutive logical tiles land on the same XCD (each of the
// 8 XCDs has its own L2).  Hardware hands workgroup ids to XCDs round-robin.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
    constexpr int64_t kXcds = 8;
    int64_t full = nblocks - nblocks % kXcds;
    if (bid >= full) return bid;
    return (bid % kXcds) * (full / kXcds) + bid / kXcds;
}

// Peak probe (measurement tool): kinds as enum tcbf_probe_kind.
double peak_probe_ops(int kind, int64_t blocks, int64_t iterations);
int64_t peak_probe_sink_bytes(int64_t blocks);
hipError_t peak_probe_launch(int kind, int64_t blocks, int64_t iterations, uint32_t operand_bits, int random,
                             void *sink, hipStream_t stream);

}  // namespace tcbf
