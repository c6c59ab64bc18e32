// Steering weights from array geometry: the step before the product, on the
// GPU, with the phase in FP64 (the only FP64 work in the library).
//
// Sec. II gives the far-field delay of sensor k as its distance along the
// wavefront normal divided by the wave speed (Eq. 2, a 1-D array); for sensor
// positions p_k = (x, y, z) and a beam direction u_m = (l, m, n) of direction
// cosines that is tau = (p_k . u_m) / c.  The weight of Eq. 3 that re-aligns
// the phase at frequency f is w = exp(+i 2 pi f tau).  Per element, exactly:
//   s = x l + y m + z n          (left to right, every product and sum rounded)
//   cycles = (f s) / c
//   turn = cycles - floor(cycles)          (the phase as a fraction of a turn)
//   w = (cos 2 pi turn, sin 2 pi turn)
// The reduction to one turn happens in FP64 before any trigonometry, so the
// argument stays in [0, 1) turn for any delay, and no operation is fused
// (contraction is switched off in this file): the FP64 turn is the one the
// same formula gives on any IEEE machine.
//  * fp32 output: cos/sin of 2 pi turn in FP64 from the device math library
//    (a few FP64 ulps), each rounded once to fp32.
//  * fp16 output: the turn split exactly in FP64 into a quarter-turn count
//    and a remainder |t| <= 1/8, t rounded to fp32 (relative error 2^-24),
//    cos/sin of 2 pi t from the fp32 sincospi of the device math library (a
//    few fp32 ulps), the quadrant applied by exact swaps and sign changes,
//    then rounded to fp16 nearest-even.  The relative error before that last
//    rounding is about 2^-21 at every magnitude (small values included, as
//    the remainder keeps its relative precision), far below half an fp16 ulp,
//    so the result is the correctly rounded fp16 value except where the
//    exact value lies within that error of a rounding boundary.
// Output: planar [batch][2][M][K].
#include "tcbf_internal.h"

#pragma clang fp contract(off)

namespace tcbf {
namespace {

constexpr int NT = 256;
constexpr double kTwoPi = 6.283185307179586;

// One weight: its cos / sin at the output precision (see above).
template <int F16>
__device__ __forceinline__ void weight(double px, double py, double pz, double l, double mm, double n, double f,
                                       double speed, float &c, float &sv) {
    double s = px * l;
    s = s + py * mm;
    s = s + pz * n;
    const double cycles = (f * s) / speed;
    const double turn = cycles - floor(cycles);
    if (F16) {
        // quarter-turn reduction in FP64 (exact): turn = q/4 + t, |t| <= 1/8,
        // so t keeps full relative precision in fp32 and values near zero
        // keep theirs
        const double q4 = rint(4.0 * turn);
        const float t = (float)(turn - 0.25 * q4);
        float sn, cs;
        sincospif(2.0f * t, &sn, &cs);
        switch ((int)q4 & 3) {
        case 0: c = cs; sv = sn; break;
        case 1: c = -sn; sv = cs; break;
        case 2: c = -cs; sv = -sn; break;
        default: c = sn; sv = -cs; break;
        }
    } else {
        double sn, cs;
        sincos(kTwoPi * turn, &sn, &cs);
        c = (float)cs;
        sv = (float)sn;
    }
}

// One thread per (channel, beam, 8 consecutive receivers): the 8 weights of
// each plane go out as one 16-byte (fp16) or two 16-byte (fp32) stores when
// K is a multiple of 8; consecutive threads take consecutive receiver groups
// of a row, then the next row.  BL (fp16 only): the receiver-blocked layout
// [c][2][Kb][M][32]; consecutive threads take the four 8-receiver groups of
// a block row, then the next beam, so a wave writes 16 beams x 64 bytes in
// one run; groups past K (up to the end of the last block) are written as
// zeros.
template <int F16, int BL>
__global__ __launch_bounds__(NT) void steering_kernel(const double *__restrict__ pos, const double *__restrict__ dir,
                                                      const double *__restrict__ freq, double speed, int64_t batch,
                                                      int64_t M, int64_t K, void *__restrict__ out) {
    static_assert(!BL || F16, "blocked output is fp16");
    const int64_t nkc = BL ? (K + 31) / 32 * 4 : (K + 7) / 8;
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t total = batch * M * nkc;
    if (gid >= total) return;
    int64_t kc, m, c;  // row = c M + m
    if (BL) {
        // gid = ((c Kb + kb) M + m) 4 + q, kc = 4 kb + q
        const int64_t kb_count = nkc / 4;
        const int64_t q = gid & 3, r = gid >> 2;
        m = r % M;
        const int64_t r2 = r / M;
        c = r2 / kb_count;
        kc = (r2 - c * kb_count) * 4 + q;
    } else if (total <= 0xffffffffll) {
        // 32-bit divisions (a 64-bit division is a long software sequence)
        const uint32_t g = (uint32_t)gid, nk = (uint32_t)nkc, mm32 = (uint32_t)M;
        const uint32_t row = g / nk;
        kc = g - row * nk;
        c = row / mm32;
        m = row - (uint32_t)c * mm32;
    } else {
        const int64_t row = gid / nkc;
        kc = gid - row * nkc;
        c = row / M;
        m = row - c * M;
    }
    const double l = dir[3 * m], mm = dir[3 * m + 1], n = dir[3 * m + 2], f = freq[c];
    const int64_t k0 = kc * 8;
    const int cnt = K - k0 < 8 ? (K - k0 > 0 ? (int)(K - k0) : 0) : 8;
    float cv[8], sv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        cv[i] = sv[i] = 0.0f;
        if (i < cnt) {
            const double *p = pos + 3 * (k0 + i);
            weight<F16>(p[0], p[1], p[2], l, mm, n, f, speed, cv[i], sv[i]);
        }
    }
    const int64_t kbn = (K + 31) / 32;
    const int64_t re = BL ? (((c * 2 + 0) * kbn + k0 / 32) * M + m) * 32 + k0 % 32 : ((c * 2 + 0) * M + m) * K + k0;
    const int64_t im = BL ? (((c * 2 + 1) * kbn + k0 / 32) * M + m) * 32 + k0 % 32 : ((c * 2 + 1) * M + m) * K + k0;
    if (F16) {
        _Float16 *o = (_Float16 *)out;
        if (BL || K % 8 == 0) {
            typedef _Float16 h8 __attribute__((ext_vector_type(8)));
            h8 a, b;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[i] = (_Float16)cv[i];
                b[i] = (_Float16)sv[i];
            }
            *reinterpret_cast<h8 *>(o + re) = a;
            *reinterpret_cast<h8 *>(o + im) = b;
        } else {
            for (int i = 0; i < cnt; ++i) {
                o[re + i] = (_Float16)cv[i];
                o[im + i] = (_Float16)sv[i];
            }
        }
    } else {
        float *o = (float *)out;
        if (K % 8 == 0) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            *reinterpret_cast<f4 *>(o + re) = (f4){cv[0], cv[1], cv[2], cv[3]};
            *reinterpret_cast<f4 *>(o + re + 4) = (f4){cv[4], cv[5], cv[6], cv[7]};
            *reinterpret_cast<f4 *>(o + im) = (f4){sv[0], sv[1], sv[2], sv[3]};
            *reinterpret_cast<f4 *>(o + im + 4) = (f4){sv[4], sv[5], sv[6], sv[7]};
        } else {
            for (int i = 0; i < cnt; ++i) {
                o[re + i] = cv[i];
                o[im + i] = sv[i];
            }
        }
    }
}

}  // namespace

int64_t steering_blocks(int64_t batch, int64_t M, int64_t K, int blocked) {
    const int64_t groups = blocked ? (K + 31) / 32 * 4 : (K + 7) / 8;
    return (batch * M * groups + NT - 1) / NT;
}

hipError_t steering_launch(const double *pos, const double *dir, const double *freq, double speed, int64_t batch,
                           int64_t M, int64_t K, int out_type, int out_layout, void *out, hipStream_t stream) {
    const bool bl = out_layout == TCBF_BLOCKED;
    const uint32_t blocks = (uint32_t)steering_blocks(batch, M, K, bl);
    typedef void (*Fn)(const double *, const double *, const double *, double, int64_t, int64_t, int64_t, void *);
    const Fn fn = out_type == TCBF_SRC_F16 ? (bl ? steering_kernel<1, 1> : steering_kernel<1, 0>)
                                           : steering_kernel<0, 0>;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(NT), 0, stream, pos, dir, freq, speed, batch, M, K, out);
    return hipGetLastError();
}

}  // namespace tcbf
