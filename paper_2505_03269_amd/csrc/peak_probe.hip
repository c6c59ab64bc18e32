// Peak probe: the matrix-unit (and VALU xor/popcount) throughput of the chip
// with no global-memory traffic, the measured denominator beside the
// published one.  The paper measures its GPUs' tensor-core peaks with
// micro-benchmarks that keep the matrix units busy on register operands
// (Sec. III-A, Table 1) and places its kernels against them (Sec. IV-B); this
// is the gfx950 counterpart for the instructions the library uses.
//
// Every wave runs `iterations` rounds of CHAINS independent accumulations on
// register operands (independent chains so no instruction waits for the
// previous one's result), then every thread writes one 32-bit value of its
// accumulators to the sink, so nothing is dead code.  Two operand modes:
//  * uniform: every operand element has the bit pattern of a kernel argument;
//    with unit operands every accumulator element ends at a closed-form count,
//    which the tests check;
//  * random: each lane holds two sets of pseudo-random operands of moderate
//    magnitude (a hash of the argument, the lane and the workgroup) and
//    consecutive instructions alternate between them, so the multiplier
//    inputs change every instruction as they do on real data.  The chip's
//    power draw, and with it the clock it sustains, depends on that.
// Thread 0 of every workgroup also records the shader-clock counter
// (s_memtime) and the constant 100 MHz counter (s_memrealtime) before and
// after its loop, so the host can read the clock the chip ran at.
#include "tcbf_internal.h"

namespace tcbf {
namespace {

constexpr int NT = 256;
constexpr int CHAINS = 4;
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// useful operations of one instruction per wave (2 per multiply-add)
constexpr double kOpsF16 = 2.0 * 32 * 32 * 16;   // v_mfma_f32_32x32x16_f16
constexpr double kOpsI8 = 2.0 * 32 * 32 * 32;    // v_mfma_i32_32x32x32_i8
constexpr double kOpsF8 = 2.0 * 32 * 32 * 64;    // v_mfma_scale_f32_32x32x64_f8f6f4, e4m3
constexpr double kOpsF4 = 2.0 * 32 * 32 * 64;    // same instruction, e2m1 operands
constexpr double kOpsValu = 64.0 * 64;           // xor + popcount of 32 bit pairs per lane, 64 lanes

__device__ __forceinline__ void clock_marks(uint64_t *marks, int slot) {
    if (threadIdx.x == 0) {
        const uint64_t t = __builtin_amdgcn_s_memtime();
        const uint64_t r = __builtin_amdgcn_s_memrealtime();
        marks[4 * blockIdx.x + 2 * slot] = t;
        marks[4 * blockIdx.x + 2 * slot + 1] = r;
    }
}

// splitmix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): 32 well-mixed bits of a 64-bit key
__device__ __forceinline__ uint32_t mix32(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

// Operand word j of set s for this lane.  Random words keep every element
// finite and of moderate size: fp16 in +-[0.5, 1), e4m3 in +-[0.5, 1), any
// e2m1 code (the format has no infinities), any int8.
template <int KIND>
__device__ __forceinline__ uint32_t operand_word(uint32_t bits, int random, int s, int j) {
    if (!random) return KIND == TCBF_PROBE_F16 ? (bits & 0xffffu) * 0x10001u : bits;
    const uint64_t key = ((uint64_t)bits << 32) ^ ((uint64_t)blockIdx.x << 14) ^ (threadIdx.x << 5) ^ (s << 4) ^ j;
    const uint32_t r = mix32(key);
    if (KIND == TCBF_PROBE_F16) return (r & 0x83ff83ffu) | 0x38003800u;
    if (KIND == TCBF_PROBE_F8) return (r & 0x87878787u) | 0x30303030u;
    return r;
}

template <int KIND>
__global__ __launch_bounds__(NT) void peak_probe_kernel(uint32_t operand_bits, int random, int64_t iterations,
                                                        uint32_t *__restrict__ sink, uint64_t *__restrict__ marks) {
    clock_marks(marks, 0);
    uint32_t out = 0;
    if (KIND == TCBF_PROBE_F16) {
        half8 a[2], b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            u32x4 wa, wb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                wa[j] = operand_word<KIND>(operand_bits, random, s, j);
                wb[j] = operand_word<KIND>(operand_bits, random, s, 4 + j);
            }
            a[s] = __builtin_bit_cast(half8, wa);
            b[s] = __builtin_bit_cast(half8, wb);
        }
        f32x16 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = (f32x16){};
        for (int64_t it = 0; it < iterations; ++it)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[c & 1], b[c & 1], acc[c], 0, 0, 0);
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) s += acc[c][threadIdx.x % 16];
        out = __float_as_uint(s);
    } else if (KIND == TCBF_PROBE_I8) {
        i32x4 a[2], b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[s][j] = (int)operand_word<KIND>(operand_bits, random, s, j);
                b[s][j] = (int)operand_word<KIND>(operand_bits, random, s, 4 + j);
            }
        i32x16 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = (i32x16){};
        for (int64_t it = 0; it < iterations; ++it)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[c & 1], b[c & 1], acc[c], 0, 0, 0);
        int s = 0;
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) s += acc[c][threadIdx.x % 16];
        out = (uint32_t)s;
    } else if (KIND == TCBF_PROBE_F8 || KIND == TCBF_PROBE_F4) {
        // format codes of the f8f6f4 instruction: 0 = e4m3, 4 = e2m1
        constexpr int FMT = KIND == TCBF_PROBE_F8 ? 0 : 4;
        i32x8 a[2], b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a[s][j] = (int)operand_word<KIND>(operand_bits, random, s, j);
                b[s][j] = (int)operand_word<KIND>(operand_bits, random, s, 8 + j);
            }
        f32x16 acc[CHAINS];
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = (f32x16){};
        for (int64_t it = 0; it < iterations; ++it)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[c & 1], b[c & 1], acc[c], FMT, FMT, 0, 127,
                                                                          0, 127);
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) s += acc[c][threadIdx.x % 16];
        out = __float_as_uint(s);
    } else {
        // VALU: per lane, 8 words (distinct per lane, so the work stays on
        // the vector unit) against a wave-uniform word that changes every
        // round (so no round can be folded into another)
        uint32_t word[8], cnt[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            word[j] = random ? operand_word<KIND>(operand_bits, 1, 0, j)
                             : operand_bits ^ (0x01010101u * (uint32_t)j) ^ threadIdx.x;
            cnt[j] = 0;
        }
        uint32_t b = 0;
        for (int64_t it = 0; it < iterations; ++it) {
#pragma unroll
            for (int j = 0; j < 8; ++j) cnt[j] = __builtin_popcount(word[j] ^ b) + cnt[j];
            b += 0x9e3779b9u;
        }
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) s += cnt[j];
        out = s;
    }
    sink[(int64_t)blockIdx.x * NT + threadIdx.x] = out;
    clock_marks(marks, 1);
}

}  // namespace

double peak_probe_ops(int kind, int64_t blocks, int64_t iterations) {
    const double waves = (double)blocks * (NT / 64);
    switch (kind) {
    case TCBF_PROBE_F16: return waves * iterations * CHAINS * kOpsF16;
    case TCBF_PROBE_I8: return waves * iterations * CHAINS * kOpsI8;
    case TCBF_PROBE_F8: return waves * iterations * CHAINS * kOpsF8;
    case TCBF_PROBE_F4: return waves * iterations * CHAINS * kOpsF4;
    case TCBF_PROBE_VALU_XOR_POPC: return waves * iterations * 8 * kOpsValu;
    }
    return 0.0;
}

int64_t peak_probe_sink_bytes(int64_t blocks) { return blocks * NT * 4 + blocks * 32; }

hipError_t peak_probe_launch(int kind, int64_t blocks, int64_t iterations, uint32_t operand_bits, int random,
                             void *sink, hipStream_t stream) {
    typedef void (*ProbeFn)(uint32_t, int, int64_t, uint32_t *, uint64_t *);
    static const ProbeFn fns[5] = {peak_probe_kernel<TCBF_PROBE_F16>, peak_probe_kernel<TCBF_PROBE_I8>,
                                   peak_probe_kernel<TCBF_PROBE_F8>, peak_probe_kernel<TCBF_PROBE_F4>,
                                   peak_probe_kernel<TCBF_PROBE_VALU_XOR_POPC>};
    uint32_t *vals = (uint32_t *)sink;
    uint64_t *marks = (uint64_t *)((char *)sink + blocks * NT * 4);
    hipLaunchKernelGGL(fns[kind], dim3((uint32_t)blocks), dim3(NT), 0, stream, operand_bits, random, iterations, vals,
                       marks);
    return hipGetLastError();
}

}  // namespace tcbf
