// C ABI of the beamforming library: plan creation (validation and kernel
// choice, host only), execution (argument checks and one kernel launch), sign
// packing, FP8 quantisation, steering weights and the grouped launch.  No
// entry point throws, aborts or allocates device memory.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "tcbf_internal.h"

struct tcbf_plan_s {
    tcbf_plan_desc desc;
    tcbf::Problem prob;
    tcbf::F16Config f16;
    tcbf::Int1Config int1;
    tcbf::F8Config f8;
};

namespace tcbf {
int64_t w_entry_elems(int dtype, int a_layout, int64_t M, int64_t K) {
    if (dtype == TCBF_F16 || dtype == TCBF_BF16) return 2 * M * (a_layout == TCBF_BLOCKED ? (K + 31) / 32 * 32 : K);
    if (dtype == TCBF_INT1) return 2 * M * ((K + 31) / 32);
    const int64_t kp = f8_kp(K);
    return 2 * M * (a_layout == TCBF_BLOCKED ? (kp + 63) / 64 * 64 : kp);
}
}  // namespace tcbf

namespace {

// Descriptor sizes: the fields up to `variant` (TCBF_VERSION <= 3), and the
// whole struct (b_k_contiguous, a_batch_stride).
constexpr uint32_t kDescV1 = (uint32_t)offsetof(tcbf_plan_desc, b_k_contiguous);
constexpr uint32_t kDescV2 = (uint32_t)sizeof(tcbf_plan_desc);
constexpr int64_t kMaxIndex = (int64_t)1 << 31;  // per-launch workgroup limit

bool is_layout(int32_t v) { return v == TCBF_PLANAR || v == TCBF_INTERLEAVED; }
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }
bool is_f8(int32_t dtype) { return dtype == TCBF_F8_E4M3 || dtype == TCBF_MXF8_E4M3; }
// 16-bit float operands (fp16 or bfloat16): the same layouts and kernels
bool is_f16like(int32_t dtype) { return dtype == TCBF_F16 || dtype == TCBF_BF16; }
bool is_src_type(int32_t t) { return t == TCBF_SRC_I8 || t == TCBF_SRC_F16 || t == TCBF_SRC_F32; }

// Architecture check per device, remembered once it succeeded (plans are
// created per job in a serving loop; reading the device properties each time
// would dominate plan creation).
// A failed HIP call is reported through the returned status; its error is
// taken off the runtime's last-error slot so that it does not surface later
// in the caller's own launch checks.
tcbf_status from_hip(hipError_t e) {
    if (e == hipSuccess) return TCBF_SUCCESS;
    (void)hipGetLastError();
    return TCBF_ERROR_DEVICE;
}

constexpr int kMaxDevices = 64;
std::atomic<int> g_device_ok[kMaxDevices];

tcbf_status device_check(int device) {
    int count = 0;
    if (from_hip(hipGetDeviceCount(&count)) != TCBF_SUCCESS || count <= 0) return TCBF_ERROR_DEVICE;
    if (device < 0 || device >= count) return TCBF_ERROR_INVALID_VALUE;
    if (device < kMaxDevices && g_device_ok[device].load(std::memory_order_acquire) == 1) return TCBF_SUCCESS;
    hipDeviceProp_t prop;
    if (from_hip(hipGetDeviceProperties(&prop, device)) != TCBF_SUCCESS) return TCBF_ERROR_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TCBF_ERROR_NOT_SUPPORTED;
    if (device < kMaxDevices) g_device_ok[device].store(1, std::memory_order_release);
    return TCBF_SUCCESS;
}

tcbf_status current_device_is(int device) {
    int cur = -1;
    if (from_hip(hipGetDevice(&cur)) != TCBF_SUCCESS) return TCBF_ERROR_DEVICE;
    return cur == device ? TCBF_SUCCESS : TCBF_ERROR_INVALID_VALUE;
}

// A descriptor of either size as the whole struct (fields a shorter one
// lacks are zero).
tcbf_plan_desc full_desc(const tcbf_plan_desc *d) {
    tcbf_plan_desc r;
    memset(&r, 0, sizeof(r));
    memcpy(&r, d, d->struct_size >= kDescV2 ? kDescV2 : kDescV1);
    r.struct_size = kDescV2;
    return r;
}

// Bytes of one element of W's storage type.
int64_t w_elem_bytes(int32_t dtype) { return is_f16like(dtype) ? 2 : dtype == TCBF_INT1 ? 4 : 1; }

// Validate a descriptor without touching the HIP runtime.
tcbf_status validate_desc(const tcbf_plan_desc *dd) {
    if (dd->struct_size < kDescV1) return TCBF_ERROR_INVALID_VALUE;
    const tcbf_plan_desc full = full_desc(dd);
    const tcbf_plan_desc *d = &full;
    if (d->reserved != 0 || (d->b_k_contiguous != 0 && d->b_k_contiguous != 1)) return TCBF_ERROR_INVALID_VALUE;
    if (d->a_batch_stride < 0 || (d->a_batch_stride > 0 && d->a_shared != 0)) return TCBF_ERROR_INVALID_VALUE;
    if (d->batch < 1 || d->M < 1 || d->N < 1 || d->K < 1) return TCBF_ERROR_INVALID_VALUE;
    // the receiver-blocked layout: fp16 weights (A), or both FP8 operands
    const bool a_ok = is_layout(d->a_layout) || (d->a_layout == TCBF_BLOCKED && (is_f16like(d->dtype) || is_f8(d->dtype)));
    const bool b_ok = is_layout(d->b_layout) || (d->b_layout == TCBF_BLOCKED && is_f8(d->dtype));
    if (!a_ok || !b_ok || !is_layout(d->c_layout)) return TCBF_ERROR_INVALID_VALUE;
    if (d->variant < 0) return TCBF_ERROR_INVALID_VALUE;
    if (d->a_batch_stride > 0) {
        // at least one entry, whole 16-byte units, and every entry's start
        // representable
        const int64_t eb = w_elem_bytes(d->dtype);
        if (!is_f16like(d->dtype) && d->dtype != TCBF_INT1 && !is_f8(d->dtype)) return TCBF_ERROR_INVALID_VALUE;
        if (d->a_batch_stride < tcbf::w_entry_elems(d->dtype, d->a_layout, d->M, d->K)) return TCBF_ERROR_INVALID_VALUE;
        if ((d->a_batch_stride * eb) % 16 != 0) return TCBF_ERROR_INVALID_VALUE;
        if (d->a_batch_stride > ((int64_t)1 << 60) / d->batch / eb) return TCBF_ERROR_NOT_SUPPORTED;
    }
    if (d->b_k_contiguous != 0 && is_f16like(d->dtype) && !is_layout(d->b_layout)) return TCBF_ERROR_INVALID_VALUE;
    if (is_f16like(d->dtype)) {
        // every per-channel plane must be indexable with 32-bit element counts
        const int64_t kw = d->a_layout == TCBF_BLOCKED ? (d->K + 31) / 32 * 32 : d->K;
        if (2 * d->M * kw >= kMaxIndex || 2 * d->K * d->N >= kMaxIndex || 2 * d->M * d->N >= kMaxIndex)
            return TCBF_ERROR_NOT_SUPPORTED;
    } else if (d->dtype == TCBF_INT1) {
        if (d->a_layout != TCBF_PLANAR || d->b_layout != TCBF_PLANAR) return TCBF_ERROR_INVALID_VALUE;
        // int32 accumulators hold 4 * 2K: keep K well inside that range
        if (d->K > ((int64_t)1 << 26)) return TCBF_ERROR_NOT_SUPPORTED;
        if (2 * d->M * d->N >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;
    } else if (is_f8(d->dtype)) {
        const bool planar = d->a_layout == TCBF_PLANAR && d->b_layout == TCBF_PLANAR;
        const bool blocked = d->a_layout == TCBF_BLOCKED && d->b_layout == TCBF_BLOCKED;
        if (!planar && !blocked) return TCBF_ERROR_INVALID_VALUE;
        if (d->N % 4 != 0) return TCBF_ERROR_INVALID_VALUE;
        // byte offsets of every per-channel operand and output fit 31 bits
        // (blocked operands hold whole 64-receiver blocks)
        const int64_t kp = blocked ? (tcbf::f8_kp(d->K) + 63) / 64 * 64 : tcbf::f8_kp(d->K);
        if (2 * d->M * kp >= kMaxIndex || 2 * d->N * kp >= kMaxIndex || 8 * d->M * d->N >= kMaxIndex)
            return TCBF_ERROR_NOT_SUPPORTED;
    } else {
        return TCBF_ERROR_INVALID_VALUE;
    }
    return TCBF_SUCCESS;
}

}  // namespace

extern "C" {

const char *tcbf_status_string(tcbf_status s) {
    switch (s) {
    case TCBF_SUCCESS: return "TCBF_SUCCESS";
    case TCBF_ERROR_INVALID_VALUE: return "TCBF_ERROR_INVALID_VALUE";
    case TCBF_ERROR_NOT_SUPPORTED: return "TCBF_ERROR_NOT_SUPPORTED";
    case TCBF_ERROR_OUT_OF_MEMORY: return "TCBF_ERROR_OUT_OF_MEMORY";
    case TCBF_ERROR_DEVICE: return "TCBF_ERROR_DEVICE";
    case TCBF_ERROR_INTERNAL: return "TCBF_ERROR_INTERNAL";
    }
    return "TCBF_UNKNOWN_STATUS";
}

int32_t tcbf_version(void) { return TCBF_VERSION; }

tcbf_status tcbf_plan(const tcbf_plan_desc *desc, tcbf_plan_t *plan) {
    if (desc == nullptr || plan == nullptr) return TCBF_ERROR_INVALID_VALUE;
    *plan = nullptr;
    tcbf_status st = validate_desc(desc);
    if (st != TCBF_SUCCESS) return st;

    const tcbf_plan_desc d = full_desc(desc);
    const int64_t dense = tcbf::w_entry_elems(d.dtype, d.a_layout, d.M, d.K);
    tcbf::Problem p{d.batch, d.M, d.N, d.K, d.a_layout, d.b_layout, d.c_layout, d.a_shared != 0, d.device,
                    d.a_shared != 0 ? 0 : d.a_batch_stride > 0 ? d.a_batch_stride : dense,
                    is_f16like(d.dtype) && d.b_k_contiguous != 0, d.dtype == TCBF_BF16};
    tcbf_plan_s tmp;
    memset(&tmp, 0, sizeof(tmp));
    tmp.desc = d;
    tmp.prob = p;
    int64_t wgs = 0;
    if (is_f16like(desc->dtype)) {
        if (!tcbf::f16_select(p, desc->variant, &tmp.f16)) return TCBF_ERROR_INVALID_VALUE;
        wgs = tcbf::f16_workgroups(p, tmp.f16);
    } else if (is_f8(desc->dtype)) {
        if (!tcbf::f8_select(p, d.dtype == TCBF_MXF8_E4M3, desc->variant, &tmp.f8)) return TCBF_ERROR_INVALID_VALUE;
        wgs = tcbf::f8_workgroups(p, tmp.f8);
    } else {
        if (!tcbf::int1_select(p, desc->variant, &tmp.int1)) return TCBF_ERROR_INVALID_VALUE;
        wgs = tcbf::int1_workgroups(p, tmp.int1);
    }
    if (wgs >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;

    st = device_check(desc->device);
    if (st != TCBF_SUCCESS) return st;

    tcbf_plan_s *out = new (std::nothrow) tcbf_plan_s(tmp);
    if (out == nullptr) return TCBF_ERROR_OUT_OF_MEMORY;
    *plan = out;
    return TCBF_SUCCESS;
}

tcbf_status tcbf_plan_destroy(tcbf_plan_t plan) {
    delete plan;
    return TCBF_SUCCESS;
}

tcbf_status tcbf_plan_query(tcbf_plan_t plan, tcbf_plan_info *info) {
    if (plan == nullptr || info == nullptr) return TCBF_ERROR_INVALID_VALUE;
    if (info->struct_size < sizeof(tcbf_plan_info)) return TCBF_ERROR_INVALID_VALUE;
    const tcbf::Problem &p = plan->prob;
    tcbf_plan_info r;
    memset(&r, 0, sizeof(r));
    r.struct_size = sizeof(tcbf_plan_info);
    const double cm = (double)p.batch * p.M * p.N * p.K;
    r.useful_ops = 8.0 * cm;
    const double nw = p.a_shared ? 1.0 : (double)p.batch;
    if (is_f16like(plan->desc.dtype)) {
        r.variant = plan->f16.variant;
        r.tile_m = plan->f16.tile_m;
        r.tile_n = plan->f16.tile_n;
        r.tile_k = plan->f16.tile_k;
        r.threads = plan->f16.threads;
        r.workgroups = tcbf::f16_workgroups(p, plan->f16);
        r.algorithmic_bytes = 4.0 * nw * p.M * p.K + 4.0 * p.batch * p.K * p.N + 8.0 * p.batch * p.M * p.N;
        snprintf(r.kernel_name, sizeof(r.kernel_name), "%s", tcbf::f16_kernel_name(plan->f16));
    } else if (is_f8(plan->desc.dtype)) {
        const double kp = (double)tcbf::f8_kp(p.K);
        r.variant = plan->f8.variant;
        r.tile_m = plan->f8.tile_m;
        r.tile_n = plan->f8.tile_n;
        r.tile_k = plan->f8.tile_k;
        r.threads = plan->f8.threads;
        r.workgroups = tcbf::f8_workgroups(p, plan->f8);
        // codes, scales (fp32 per row, or one byte per 32-receiver block), output
        const double sa = plan->desc.dtype == TCBF_F8_E4M3 ? 4.0 : kp / 32.0;
        r.algorithmic_bytes = (2.0 * kp + sa) * (nw * p.M + (double)p.batch * p.N) + 8.0 * p.batch * p.M * p.N;
        snprintf(r.kernel_name, sizeof(r.kernel_name), "%s", tcbf::f8_kernel_name(plan->f8));
    } else {
        const double kw = (double)((p.K + 31) / 32);
        r.variant = plan->int1.variant;
        r.tile_m = plan->int1.tile_m;
        r.tile_n = plan->int1.tile_n;
        r.tile_k = plan->int1.tile_kw * 32;
        r.threads = plan->int1.threads;
        r.workgroups = tcbf::int1_workgroups(p, plan->int1);
        r.algorithmic_bytes = 8.0 * nw * p.M * kw + 8.0 * p.batch * p.N * kw + 8.0 * p.batch * p.M * p.N;
        snprintf(r.kernel_name, sizeof(r.kernel_name), "%s", tcbf::int1_kernel_name(plan->int1));
    }
    memcpy(info, &r, sizeof(r));
    return TCBF_SUCCESS;
}

tcbf_status tcbf_execute(tcbf_plan_t plan, const void *A, const void *B, void *C, const void *a_scale,
                         const void *b_scale, void *stream) {
    if (plan == nullptr || A == nullptr || B == nullptr || C == nullptr) return TCBF_ERROR_INVALID_VALUE;
    const bool f8 = is_f8(plan->desc.dtype);
    if (f8) {
        if (a_scale == nullptr || b_scale == nullptr) return TCBF_ERROR_INVALID_VALUE;
        if (!aligned16(a_scale) || !aligned16(b_scale)) return TCBF_ERROR_INVALID_VALUE;
    } else if (a_scale != nullptr || b_scale != nullptr) {
        return TCBF_ERROR_INVALID_VALUE;
    }
    if (!aligned16(A) || !aligned16(B) || !aligned16(C)) return TCBF_ERROR_INVALID_VALUE;
    tcbf_status st = current_device_is(plan->desc.device);
    if (st != TCBF_SUCCESS) return st;
    hipError_t e;
    if (is_f16like(plan->desc.dtype)) {
        e = tcbf::f16_launch(plan->prob, plan->f16, A, B, C, (hipStream_t)stream);
    } else if (f8) {
        e = tcbf::f8_launch(plan->prob, plan->f8, plan->desc.dtype == TCBF_MXF8_E4M3, A, B, C, a_scale, b_scale,
                            (hipStream_t)stream);
    } else {
        e = tcbf::int1_launch(plan->prob, plan->int1, (const uint32_t *)A, (const uint32_t *)B, (int32_t *)C,
                              (hipStream_t)stream);
    }
    return from_hip(e);
}

tcbf_status tcbf_block_weights(const void *src, int32_t src_layout, int64_t batch, int64_t M, int64_t K, void *dst,
                               void *stream) {
    if (src == nullptr || dst == nullptr) return TCBF_ERROR_INVALID_VALUE;
    if (!is_layout(src_layout)) return TCBF_ERROR_INVALID_VALUE;
    if (batch < 1 || M < 1 || K < 1) return TCBF_ERROR_INVALID_VALUE;
    if (!aligned16(src) || !aligned16(dst)) return TCBF_ERROR_INVALID_VALUE;
    if ((double)batch * (double)M * (double)(K + 31) >= 0x1p62) return TCBF_ERROR_NOT_SUPPORTED;
    if (tcbf::block_weights_workgroups(batch, M, K) >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;
    hipError_t e = tcbf::block_weights_launch(src, src_layout, batch, M, K, dst, (hipStream_t)stream);
    return from_hip(e);
}

tcbf_status tcbf_pack1bit(const void *src, int32_t src_type, int32_t src_layout, int64_t batch, int64_t rows,
                          int64_t K, int32_t src_k_major, uint32_t *dst, void *stream) {
    if (src == nullptr || dst == nullptr) return TCBF_ERROR_INVALID_VALUE;
    if (!is_src_type(src_type)) return TCBF_ERROR_INVALID_VALUE;
    if (!is_layout(src_layout)) return TCBF_ERROR_INVALID_VALUE;
    if (batch < 1 || rows < 1 || K < 1) return TCBF_ERROR_INVALID_VALUE;
    if (!aligned16(src) || !aligned16(dst)) return TCBF_ERROR_INVALID_VALUE;
    // sizes whose products could overflow are refused before the workgroup count
    if ((double)batch * (double)rows * (double)K >= 0x1p62) return TCBF_ERROR_NOT_SUPPORTED;
    if (tcbf::pack1bit_workgroups(src_type, batch, rows, K, src_k_major != 0) >= kMaxIndex)
        return TCBF_ERROR_NOT_SUPPORTED;
    hipError_t e = tcbf::pack1bit_launch(src, src_type, src_layout, batch, rows, K, src_k_major != 0, dst,
                                         (hipStream_t)stream);
    return from_hip(e);
}

tcbf_status tcbf_quantize_e4m3(const void *src, int32_t src_type, int32_t src_layout, int64_t batch, int64_t rows,
                               int64_t K, int32_t src_k_major, int32_t block, int32_t dst_layout, uint8_t *dst,
                               void *scales, void *stream) {
    if (src == nullptr || dst == nullptr || scales == nullptr) return TCBF_ERROR_INVALID_VALUE;
    if (!is_src_type(src_type) || !is_layout(src_layout)) return TCBF_ERROR_INVALID_VALUE;
    if (dst_layout != TCBF_PLANAR && dst_layout != TCBF_BLOCKED) return TCBF_ERROR_INVALID_VALUE;
    if (block != 0 && block != 32) return TCBF_ERROR_INVALID_VALUE;
    if (batch < 1 || rows < 1 || K < 1) return TCBF_ERROR_INVALID_VALUE;
    if (!aligned16(src) || !aligned16(dst) || !aligned16(scales)) return TCBF_ERROR_INVALID_VALUE;
    if (tcbf::quantize_e4m3_tiles(batch, rows, K) >= kMaxIndex || batch * rows / 256 + 1 >= kMaxIndex)
        return TCBF_ERROR_NOT_SUPPORTED;
    hipError_t e = tcbf::quantize_e4m3_launch(src, src_type, src_layout, batch, rows, K, src_k_major != 0, block,
                                              dst_layout, dst, scales, (hipStream_t)stream);
    return from_hip(e);
}

tcbf_status tcbf_steering_weights(const double *positions, const double *directions, const double *frequencies,
                                  double wave_speed, int64_t batch, int64_t M, int64_t K, int32_t out_type,
                                  int32_t out_layout, void *W, void *stream) {
    if (positions == nullptr || directions == nullptr || frequencies == nullptr || W == nullptr)
        return TCBF_ERROR_INVALID_VALUE;
    if (out_type != TCBF_SRC_F16 && out_type != TCBF_SRC_F32) return TCBF_ERROR_INVALID_VALUE;
    // blocked output: fp16 weights only (the layout the fp16 product reads)
    if (out_layout != TCBF_PLANAR && !(out_layout == TCBF_BLOCKED && out_type == TCBF_SRC_F16))
        return TCBF_ERROR_INVALID_VALUE;
    if (batch < 1 || M < 1 || K < 1) return TCBF_ERROR_INVALID_VALUE;
    if (!(wave_speed > 0.0) || wave_speed > 1e300) return TCBF_ERROR_INVALID_VALUE;
    if (!aligned8(positions) || !aligned8(directions) || !aligned8(frequencies) || !aligned16(W))
        return TCBF_ERROR_INVALID_VALUE;
    if ((double)batch * (double)M * (double)(K + 31) >= 0x1p62) return TCBF_ERROR_NOT_SUPPORTED;
    if (tcbf::steering_blocks(batch, M, K, out_layout == TCBF_BLOCKED) >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;
    hipError_t e = tcbf::steering_launch(positions, directions, frequencies, wave_speed, batch, M, K, out_type,
                                         out_layout, W, (hipStream_t)stream);
    return from_hip(e);
}

tcbf_status tcbf_peak_probe(int32_t kind, int64_t blocks, int64_t iterations, uint32_t operand_bits,
                            int32_t operand_mode, void *sink, int64_t sink_bytes, double *ops, void *stream) {
    if (kind < TCBF_PROBE_F16 || kind > TCBF_PROBE_VALU_XOR_POPC) return TCBF_ERROR_INVALID_VALUE;
    if (operand_mode != TCBF_PROBE_UNIFORM && operand_mode != TCBF_PROBE_RANDOM) return TCBF_ERROR_INVALID_VALUE;
    if (blocks < 1 || iterations < 1 || sink == nullptr || !aligned16(sink)) return TCBF_ERROR_INVALID_VALUE;
    if (blocks >= kMaxIndex / 256 || iterations > ((int64_t)1 << 40)) return TCBF_ERROR_NOT_SUPPORTED;
    if (sink_bytes < tcbf::peak_probe_sink_bytes(blocks)) return TCBF_ERROR_INVALID_VALUE;
    if (ops != nullptr) *ops = tcbf::peak_probe_ops(kind, blocks, iterations);
    hipError_t e = tcbf::peak_probe_launch(kind, blocks, iterations, operand_bits, operand_mode == TCBF_PROBE_RANDOM,
                                           sink, (hipStream_t)stream);
    return from_hip(e);
}

}  // extern "C"

namespace {

// Scratch memory of tcbf_group_execute_noalloc: the grouped launch's tile
// counter, one copy per GPU, held until the process ends.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns with the device current (kept per device).
static __device__ __align__(256) unsigned char scratch[TCBF_GROUP_SCRATCH_BYTES];
static_assert(TCBF_GROUP_WORKSPACE_BYTES <= TCBF_GROUP_SCRATCH_BYTES, "the scratch array holds one workspace");

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// Device address of `device`'s scratch array (the device must be current),
// looked up on the first call on that device.
tcbf_status scratch_of(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return TCBF_ERROR_NOT_SUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device] == nullptr) {
        void *ptr = nullptr;
        if (from_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != TCBF_SUCCESS || ptr == nullptr)
            return TCBF_ERROR_DEVICE;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return TCBF_SUCCESS;
}

// The grouped launch behind both entry points: the device tile counter is in
// the caller's `workspace`, or with `use_scratch` in this device's scratch
// array (looked up after every argument check).
tcbf_status group_execute(int32_t device, int32_t dtype, int32_t c_layout, const tcbf_group_problem *problems,
                          int32_t count, void *workspace, bool use_scratch, void *stream) {
    if (problems == nullptr || (workspace == nullptr && !use_scratch)) return TCBF_ERROR_INVALID_VALUE;
    if ((dtype != TCBF_F16 && dtype != TCBF_INT1 && !is_f8(dtype)) || !is_layout(c_layout))
        return TCBF_ERROR_INVALID_VALUE;
    if (count < 1 || count > TCBF_GROUP_MAX) return TCBF_ERROR_INVALID_VALUE;
    if (!use_scratch && !aligned16(workspace)) return TCBF_ERROR_INVALID_VALUE;
    tcbf::Problem probs[TCBF_GROUP_MAX];
    const void *A[TCBF_GROUP_MAX];
    const void *B[TCBF_GROUP_MAX];
    void *C[TCBF_GROUP_MAX];
    const void *SA[TCBF_GROUP_MAX];
    const void *SB[TCBF_GROUP_MAX];
    int order[TCBF_GROUP_MAX];
    int variants[TCBF_GROUP_MAX];
    int64_t total = 0;
    // one operand layout per launch (it picks the kernel): planar, or blocked
    // fp16 weights / blocked FP8 codes
    const int32_t layout = problems[0].layout;
    if (layout != TCBF_PLANAR && !(layout == TCBF_BLOCKED && dtype != TCBF_INT1)) return TCBF_ERROR_INVALID_VALUE;
    const bool blocked = layout == TCBF_BLOCKED;
    for (int i = 0; i < count; ++i) {
        const tcbf_group_problem &g = problems[i];
        if (g.A == nullptr || g.B == nullptr || g.C == nullptr || g.layout != layout) return TCBF_ERROR_INVALID_VALUE;
        if (!aligned16(g.A) || !aligned16(g.B) || !aligned16(g.C)) return TCBF_ERROR_INVALID_VALUE;
        if (g.batch < 1 || g.M < 1 || g.N < 1 || g.K < 1) return TCBF_ERROR_INVALID_VALUE;
        probs[i] = tcbf::Problem{g.batch, g.M, g.N, g.K, layout, (blocked && is_f8(dtype)) ? TCBF_BLOCKED : TCBF_PLANAR,
                                 c_layout, g.a_shared != 0, device,
                                 g.a_shared != 0 ? 0 : tcbf::w_entry_elems(dtype, layout, g.M, g.K), 0, 0};
        if (g.reserved != 0 || g.variant < 0) return TCBF_ERROR_INVALID_VALUE;
        variants[i] = 0;
        if (dtype == TCBF_F16) {
            if ((!blocked && g.K % 8 != 0) || g.N % 8 != 0) return TCBF_ERROR_INVALID_VALUE;
            if (g.a_scale != nullptr || g.b_scale != nullptr) return TCBF_ERROR_INVALID_VALUE;
            if (!tcbf::f16_group_problem_ok(probs[i])) return TCBF_ERROR_NOT_SUPPORTED;
            // the problem's variant: given (a fast variant its plan accepts)
            // or the plan's default; it picks the grouped launch it joins
            tcbf::F16Config cfg;
            if (g.variant == 1 || !tcbf::f16_select(probs[i], g.variant, &cfg) || cfg.variant < 2)
                return TCBF_ERROR_INVALID_VALUE;
            variants[i] = cfg.variant;
            total += tcbf::f16_group_tiles(probs[i]);
        } else if (dtype == TCBF_INT1) {
            if (g.variant != 0) return TCBF_ERROR_INVALID_VALUE;
            if (g.a_scale != nullptr || g.b_scale != nullptr) return TCBF_ERROR_INVALID_VALUE;
            // the plan limits: int32 accumulators, 32-bit output indices
            if (g.K > ((int64_t)1 << 26) || 2 * g.M * g.N >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;
            total += tcbf::int1_group_tiles(probs[i]);
        } else {
            if (g.variant != 0) return TCBF_ERROR_INVALID_VALUE;
            if (g.N % 4 != 0) return TCBF_ERROR_INVALID_VALUE;
            if (g.a_scale == nullptr || g.b_scale == nullptr) return TCBF_ERROR_INVALID_VALUE;
            if (!aligned16(g.a_scale) || !aligned16(g.b_scale)) return TCBF_ERROR_INVALID_VALUE;
            // the plan limits: byte offsets of per-channel operands and output fit 31 bits
            const int64_t kp = blocked ? (tcbf::f8_kp(g.K) + 63) / 64 * 64 : tcbf::f8_kp(g.K);
            if (2 * g.M * kp >= kMaxIndex || 2 * g.N * kp >= kMaxIndex || 8 * g.M * g.N >= kMaxIndex)
                return TCBF_ERROR_NOT_SUPPORTED;
            total += tcbf::f8_group_tiles(probs[i]);
        }
        if (total >= kMaxIndex) return TCBF_ERROR_NOT_SUPPORTED;
        A[i] = g.A;
        B[i] = g.B;
        C[i] = g.C;
        SA[i] = g.a_scale;
        SB[i] = g.b_scale;
        order[i] = i;
    }
    // longest tiles (most receivers) first, so the list ends on short tiles
    std::stable_sort(order, order + count, [&](int a, int b) { return probs[a].K > probs[b].K; });
    tcbf_status st = device_check(device);
    if (st == TCBF_SUCCESS) st = current_device_is(device);
    if (st != TCBF_SUCCESS) return st;
    if (use_scratch) {
        st = scratch_of(device, &workspace);
        if (st != TCBF_SUCCESS) return st;
    }
    int cus = 0;
    if (from_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != TCBF_SUCCESS || cus < 1)
        return TCBF_ERROR_DEVICE;
    const int grid = (int)std::min<int64_t>(total, 2 * (int64_t)cus);
    unsigned int *counter = (unsigned int *)workspace;
    hipError_t e;
    if (dtype == TCBF_F16)
        e = tcbf::f16_group_launch(probs, A, B, C, order, variants, count, c_layout, cus, counter, (hipStream_t)stream);
    else if (dtype == TCBF_INT1)
        e = tcbf::int1_group_launch(probs, A, B, C, order, count, c_layout, grid, counter, (hipStream_t)stream);
    else
        e = tcbf::f8_group_launch(probs, A, B, C, SA, SB, order, count, dtype == TCBF_MXF8_E4M3, c_layout, grid,
                                  counter, (hipStream_t)stream);
    return from_hip(e);
}

}  // namespace

extern "C" {

tcbf_status tcbf_group_execute(int32_t device, int32_t dtype, int32_t c_layout, const tcbf_group_problem *problems,
                               int32_t count, void *workspace, void *stream) {
    return group_execute(device, dtype, c_layout, problems, count, workspace, false, stream);
}

tcbf_status tcbf_group_execute_noalloc(int32_t device, int32_t dtype, int32_t c_layout,
                                       const tcbf_group_problem *problems, int32_t count, void *stream) {
    return group_execute(device, dtype, c_layout, problems, count, nullptr, true, stream);
}

}  // extern "C"
