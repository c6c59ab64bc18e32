// Steering weights from array geometry: the step before the product, on the
// GPU and in FP64 (the only FP64 work in the library).
//
// Sec. II gives the far-field delay of sensor k as its distance along the
// wavefront normal divided by the wave speed (Eq. 2, a 1-D array); for sensor
// positions p_k = (x, y, z) and a beam direction u_m = (l, m, n) of direction
// cosines that is tau = (p_k . u_m) / c.  The weight of Eq. 3 that re-aligns
// the phase at frequency f is w = exp(+i 2 pi f tau).  Per element, exactly:
//   s = x l + y m + z n          (left to right, every product and sum rounded)
//   cycles = (f s) / c
//   phi = 2 pi (cycles - floor(cycles))
//   w = (cos phi, sin phi)
// The reduction to one turn happens before the multiplication by 2 pi, so the
// argument of cos/sin stays in [0, 2 pi) for any delay.  No operation is fused
// (contraction is switched off in this file) so the FP64 phase is the one the
// same formula gives on any IEEE machine; cos/sin come from the device math
// library (a few FP64 ulps).  Output: planar [batch][2][M][K] in fp32 (nearest)
// or fp16.  fp16 is rounded once from FP64: the value is first rounded to fp32
// with round-to-odd (truncate, then set the last bit if anything was dropped),
// then to fp16 nearest-even, which equals direct nearest-even rounding because
// fp32 carries more than two extra bits (Boldo and Melquiond, "Emulation of FMA
// and correctly rounded sums: proved algorithms using rounding to odd", IEEE
// Trans. Computers 57(4), 2008).
#include "tcbf_internal.h"

#pragma clang fp contract(off)

namespace tcbf {
namespace {

constexpr int NT = 256;
constexpr double kTwoPi = 6.283185307179586;

__device__ __forceinline__ float round_to_odd_f32(double v) {
    float f = (float)v;                                    // nearest
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1u;                // one step back toward zero: truncation
    if ((double)__uint_as_float(b) != v) b |= 1u;          // inexact: make it odd
    return __uint_as_float(b);
}

__device__ __forceinline__ uint16_t to_f16_bits(double v) {
    const _Float16 h = (_Float16)round_to_odd_f32(v);
    return __builtin_bit_cast(uint16_t, h);
}

// One thread per (channel, beam, receiver); receivers fastest so every store
// instruction writes consecutive elements of one row.
template <int F16>
__global__ __launch_bounds__(NT) void steering_kernel(const double *__restrict__ pos, const double *__restrict__ dir,
                                                      const double *__restrict__ freq, double speed, int64_t batch,
                                                      int64_t M, int64_t K, void *__restrict__ out) {
    const int64_t kb = (K + NT - 1) / NT;
    const int64_t bid = blockIdx.x;
    const int64_t k = (bid % kb) * NT + threadIdx.x;
    const int64_t m = (bid / kb) % M;
    const int64_t c = bid / (kb * M);
    if (k >= K) return;
    const double l = dir[3 * m], mm = dir[3 * m + 1], n = dir[3 * m + 2];
    double s = pos[3 * k] * l;
    s = s + pos[3 * k + 1] * mm;
    s = s + pos[3 * k + 2] * n;
    const double cycles = (freq[c] * s) / speed;
    const double phi = kTwoPi * (cycles - floor(cycles));
    double sn, cs;
    sincos(phi, &sn, &cs);
    const int64_t re = ((c * 2 + 0) * M + m) * K + k, im = ((c * 2 + 1) * M + m) * K + k;
    if (F16) {
        ((uint16_t *)out)[re] = to_f16_bits(cs);
        ((uint16_t *)out)[im] = to_f16_bits(sn);
    } else {
        ((float *)out)[re] = (float)cs;
        ((float *)out)[im] = (float)sn;
    }
}

}  // namespace

int64_t steering_blocks(int64_t batch, int64_t M, int64_t K) { return batch * M * ((K + NT - 1) / NT); }

hipError_t steering_launch(const double *pos, const double *dir, const double *freq, double speed, int64_t batch,
                           int64_t M, int64_t K, int out_type, void *out, hipStream_t stream) {
    const uint32_t blocks = (uint32_t)steering_blocks(batch, M, K);
    if (out_type == TCBF_SRC_F16)
        hipLaunchKernelGGL(steering_kernel<1>, dim3(blocks), dim3(NT), 0, stream, pos, dir, freq, speed, batch, M, K,
                           out);
    else
        hipLaunchKernelGGL(steering_kernel<0>, dim3(blocks), dim3(NT), 0, stream, pos, dir, freq, speed, batch, M, K,
                           out);
    return hipGetLastError();
}

}  // namespace tcbf
