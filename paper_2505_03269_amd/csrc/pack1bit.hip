// Sign packing for the 1-bit mode (Sec. III: 32 consecutive 1-bit samples per
// 32-bit word; Sec. III-D / Fig. 1: bit 1 = +1, bit 0 = -1 per component).
//
// Sign rule: a value whose sign bit is clear becomes 1 (so integer 0 and +0.0
// give +1, -0.0 gives -1).  For two's-complement int8 this is exactly x >= 0.
// Destination: [batch][2][rows][kw] uint32, sample k in bit k % 32 of word
// k / 32, bits past K zero.
//
// Both source orientations are memory-bound streaming kernels:
//  * K-major (W-like, rows of K contiguous samples): one thread builds one
//    word per plane from 32 consecutive samples of its row; consecutive
//    threads take consecutive words, so the word stores are contiguous.
//  * N-major (X-like, [K][rows] with rows contiguous): consecutive threads take
//    consecutive rows so every sample row is read coalesced; each thread
//    builds 4 consecutive words (128 samples along K) per plane and writes
//    them as one 16-byte store.  When the row count allows, a thread takes 8
//    bytes' worth of consecutive rows per plane, so each receiver step is one
//    16-byte (or two 8-byte) loads per lane.
#include "tcbf_internal.h"

namespace tcbf {
namespace {

template <typename T> struct Bits;
template <> struct Bits<uint8_t> { static __device__ uint32_t pos(uint8_t v) { return (v >> 7) ^ 1u; } };
template <> struct Bits<uint16_t> { static __device__ uint32_t pos(uint16_t v) { return (v >> 15) ^ 1u; } };
template <> struct Bits<uint32_t> { static __device__ uint32_t pos(uint32_t v) { return (v >> 31) ^ 1u; } };

constexpr int NT = 256;
constexpr int VW = 4;            // waves per workgroup of the vectorised N-major kernel
constexpr int VNT = 64 * VW;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// K-major.  Thread -> (c, row, word); planar sources give plane stride rows*K,
// interleaved sources hold (re, im) pairs.
template <typename T, int IL>
__global__ __launch_bounds__(NT) void pack_kmajor_kernel(const T *__restrict__ src, uint32_t *__restrict__ dst,
                                                         int64_t batch, int64_t rows, int64_t K, int64_t kw) {
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t total = batch * rows * kw;
    if (gid >= total) return;
    const int64_t w = gid % kw;
    const int64_t r = (gid / kw) % rows;
    const int64_t c = gid / (kw * rows);
    const int64_t k0 = w * 32;
    const int n = (int)((K - k0) < 32 ? (K - k0) : 32);
    uint32_t wr = 0, wi = 0;
    if (IL) {
        const T *p = src + ((c * rows + r) * K + k0) * 2;
        for (int e = 0; e < n; ++e) {
            wr |= Bits<T>::pos(p[2 * e]) << e;
            wi |= Bits<T>::pos(p[2 * e + 1]) << e;
        }
    } else {
        const T *pr = src + ((c * 2 + 0) * rows + r) * K + k0;
        const T *pi = src + ((c * 2 + 1) * rows + r) * K + k0;
        for (int e = 0; e < n; ++e) {
            wr |= Bits<T>::pos(pr[e]) << e;
            wi |= Bits<T>::pos(pi[e]) << e;
        }
    }
    dst[((c * 2 + 0) * rows + r) * kw + w] = wr;
    dst[((c * 2 + 1) * rows + r) * kw + w] = wi;
}

// N-major.  Thread -> (c, word group of 4, row); rows fastest.
template <typename T, int IL>
__global__ __launch_bounds__(NT) void pack_nmajor_kernel(const T *__restrict__ src, uint32_t *__restrict__ dst,
                                                         int64_t batch, int64_t rows, int64_t K, int64_t kw,
                                                         int vec_store) {
    const int64_t gid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t ngroups = (kw + 3) / 4;
    const int64_t total = batch * ngroups * rows;
    if (gid >= total) return;
    const int64_t r = gid % rows;
    const int64_t g = (gid / rows) % ngroups;
    const int64_t c = gid / (rows * ngroups);
    uint32_t wr[4] = {0u, 0u, 0u, 0u}, wi[4] = {0u, 0u, 0u, 0u};
    const int64_t k0 = g * 128;
    const int n = (int)((K - k0) < 128 ? (K - k0) : 128);
    if (IL) {
        const T *p = src + ((c * K + k0) * rows + r) * 2;
        for (int e = 0; e < n; ++e) {
            const T *q = p + (int64_t)e * rows * 2;
            wr[e >> 5] |= Bits<T>::pos(q[0]) << (e & 31);
            wi[e >> 5] |= Bits<T>::pos(q[1]) << (e & 31);
        }
    } else {
        const T *pr = src + (c * 2 * K + k0) * rows + r;
        const T *pi = pr + K * rows;
        for (int e = 0; e < n; ++e) {
            wr[e >> 5] |= Bits<T>::pos(pr[(int64_t)e * rows]) << (e & 31);
            wi[e >> 5] |= Bits<T>::pos(pi[(int64_t)e * rows]) << (e & 31);
        }
    }
    uint32_t *dr = dst + ((c * 2 + 0) * rows + r) * kw + g * 4;
    uint32_t *di = dst + ((c * 2 + 1) * rows + r) * kw + g * 4;
    if (vec_store && g * 4 + 4 <= kw) {
        *reinterpret_cast<uint4 *>(dr) = make_uint4(wr[0], wr[1], wr[2], wr[3]);
        *reinterpret_cast<uint4 *>(di) = make_uint4(wi[0], wi[1], wi[2], wi[3]);
    } else {
        for (int q = 0; q < 4 && g * 4 + q < kw; ++q) {
            dr[q] = wr[q];
            di[q] = wi[q];
        }
    }
}

// N-major, vectorised: each thread owns R consecutive rows (R * sizeof(T) =
// 8 bytes per plane), 128 receivers, both planes.  Per receiver it loads the
// R rows' 16 bytes (interleaved: one 16-byte load of (re, im) pairs; planar:
// 8 bytes of each plane); a wave load covers 64 * 8 consecutive row bytes per
// plane.  Needs rows % R == 0.
//
// Receivers go in rounds of 16 with all 16 loads issued before any is used,
// so every thread keeps 16 loads in flight (2% faster than rounds of 8 on
// int8 [16][8192][8192][2]; a 32-bit word's tail takes rounds of 8 and 1).
// The sign bits of each group of 8 receivers are gathered without
// per-element work: shifting receiver u's dword right by (element width - 1
// - u) puts each element's sign bit at bit u of that element's field, so
// OR-ing the 8 masked dwords collects, per element, its 8 receivers' signs
// in the low byte of its field; one complement turns sign bits into the +1
// bits, and each byte lands in its row's word at the group's bit offset.
template <int IL> struct RawRows;
template <> struct RawRows<1> {
    static __device__ __forceinline__ u32x4 load(const void *p, int64_t) {
        return *reinterpret_cast<const u32x4 *>(p);
    }
};
template <> struct RawRows<0> {
    static __device__ __forceinline__ u32x4 load(const void *p, int64_t plane_bytes) {
        const u32x2 a = *reinterpret_cast<const u32x2 *>(p);
        const u32x2 b = *reinterpret_cast<const u32x2 *>((const char *)p + plane_bytes);
        return (u32x4){a[0], a[1], b[0], b[1]};
    }
};

template <typename T, int IL>
__global__ __launch_bounds__(VNT) void pack_nmajor_vec_kernel(const T *__restrict__ src, uint32_t *__restrict__ dst,
                                                             int64_t batch, int64_t rows, int64_t K, int64_t kw) {
    constexpr int R = 8 / (int)sizeof(T);      // rows per thread
    constexpr int E = 2 * R;                   // elements in the 16 bytes of one receiver
    constexpr int W = 8 * (int)sizeof(T);      // element width in bits
    constexpr int EPD = 4 / (int)sizeof(T);    // elements per dword
    constexpr uint32_t LOW = sizeof(T) == 1 ? 0x01010101u : sizeof(T) == 2 ? 0x00010001u : 1u;
    // Workgroup -> (c, VW word groups, 64 row groups): wave w takes word group
    // VW gb + w of the workgroup's rows, so the VW waves write the VW 16-byte
    // pieces of each row's 16 VW output bytes together (whole 64-byte runs
    // instead of scattered pieces); consecutive workgroups take the next
    // rows, so the reads in flight spread along each receiver's row of
    // samples.
    const int64_t ngroups = (kw + 3) / 4;
    const int64_t rgroups = rows / R;
    const int64_t gblocks = (ngroups + VW - 1) / VW, rblocks = (rgroups + 63) / 64;
    const int64_t bid = blockIdx.x;
    const int64_t rb = bid % rblocks, gb = (bid / rblocks) % gblocks, c = bid / (gblocks * rblocks);
    const int64_t g = gb * VW + (threadIdx.x >> 6);
    const int64_t rg = rb * 64 + (threadIdx.x & 63);
    if (c >= batch || g >= ngroups || rg >= rgroups) return;
    const int64_t r0 = rg * R;
    uint32_t wr[R][4], wi[R][4];
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) wr[j][q] = wi[j][q] = 0u;
    const int64_t k0 = g * 128;
    const int n = (int)((K - k0) < 128 ? (K - k0) : 128);
    // element (k, row) of plane 0: interleaved ((c K + k) rows + row) * 2, planar (c 2 K + k) rows + row
    const T *base = IL ? src + ((c * K + k0) * rows + r0) * 2 : src + (c * 2 * K + k0) * rows + r0;
    const int64_t kstep = IL ? rows * 2 : rows, plane_bytes = K * rows * (int64_t)sizeof(T);
    // element e of a receiver's 16 bytes -> plane and row
    auto place = [](int e, int &pl, int &row) {
        pl = IL ? (e & 1) : (e >= R);
        row = IL ? (e >> 1) : (e % R);
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (32 * q >= n) break;
        const int m = n - 32 * q < 32 ? n - 32 * q : 32;
        int b = 0;
        // rounds of 16 receivers (16 loads in flight), gathered as two groups of 8
        for (; b + 16 <= m; b += 16) {
            u32x4 d[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) d[u] = RawRows<IL>::load(base + (int64_t)(32 * q + b + u) * kstep, plane_bytes);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                u32x4 t = (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
                for (int u = 0; u < 8; ++u) t |= (d[8 * h + u] >> (uint32_t)(W - 1 - u)) & (LOW << u);
                t = ~t;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    int pl, row;
                    place(e, pl, row);
                    const uint32_t byte = (t[e / EPD] >> (W * (e % EPD))) & 0xffu;
                    if (pl) wi[row][q] |= byte << (b + 8 * h);
                    else wr[row][q] |= byte << (b + 8 * h);
                }
            }
        }
        for (; b + 8 <= m; b += 8) {
            u32x4 d[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] = RawRows<IL>::load(base + (int64_t)(32 * q + b + u) * kstep, plane_bytes);
            u32x4 t = (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
            for (int u = 0; u < 8; ++u) t |= (d[u] >> (uint32_t)(W - 1 - u)) & (LOW << u);
            t = ~t;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                int pl, row;
                place(e, pl, row);
                const uint32_t byte = (t[e / EPD] >> (W * (e % EPD))) & 0xffu;
                if (pl) wi[row][q] |= byte << b;
                else wr[row][q] |= byte << b;
            }
        }
        for (; b < m; ++b) {
            const u32x4 t = ~RawRows<IL>::load(base + (int64_t)(32 * q + b) * kstep, plane_bytes);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                int pl, row;
                place(e, pl, row);
                const uint32_t bit = (t[e / EPD] >> (W * (e % EPD) + W - 1)) & 1u;
                if (pl) wi[row][q] |= bit << b;
                else wr[row][q] |= bit << b;
            }
        }
    }
    const bool full = g * 4 + 4 <= kw;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        uint32_t *dr = dst + ((c * 2 + 0) * rows + r0 + j) * kw + g * 4;
        uint32_t *di = dst + ((c * 2 + 1) * rows + r0 + j) * kw + g * 4;
        if (full && (kw % 4) == 0) {
            *reinterpret_cast<uint4 *>(dr) = make_uint4(wr[j][0], wr[j][1], wr[j][2], wr[j][3]);
            *reinterpret_cast<uint4 *>(di) = make_uint4(wi[j][0], wi[j][1], wi[j][2], wi[j][3]);
        } else {
            for (int q = 0; q < 4 && g * 4 + q < kw; ++q) {
                dr[q] = wr[j][q];
                di[q] = wi[j][q];
            }
        }
    }
}

// Workgroups of the kernel that takes (element size, rows, K, orientation).
int64_t pack_workgroups(int64_t elem_bytes, int64_t batch, int64_t rows, int64_t K, int kmajor) {
    const int64_t kw = (K + 31) / 32, ngroups = (kw + 3) / 4, R = 8 / elem_bytes;
    if (kmajor) return (batch * rows * kw + NT - 1) / NT;
    if (rows % R == 0) return batch * ((ngroups + VW - 1) / VW) * ((rows / R + 63) / 64);
    return (batch * ngroups * rows + NT - 1) / NT;
}

template <typename T>
hipError_t launch_typed(const void *src, int il, int64_t batch, int64_t rows, int64_t K, int kmajor,
                        uint32_t *dst, hipStream_t stream) {
    const int64_t kw = (K + 31) / 32;
    const T *s = (const T *)src;
    const dim3 grid((uint32_t)pack_workgroups(sizeof(T), batch, rows, K, kmajor));
    if (kmajor) {
        if (il) hipLaunchKernelGGL((pack_kmajor_kernel<T, 1>), grid, dim3(NT), 0, stream, s, dst, batch, rows, K, kw);
        else    hipLaunchKernelGGL((pack_kmajor_kernel<T, 0>), grid, dim3(NT), 0, stream, s, dst, batch, rows, K, kw);
    } else if (rows % (8 / (int64_t)sizeof(T)) == 0) {
        if (il) hipLaunchKernelGGL((pack_nmajor_vec_kernel<T, 1>), grid, dim3(VNT), 0, stream, s, dst, batch, rows, K, kw);
        else    hipLaunchKernelGGL((pack_nmajor_vec_kernel<T, 0>), grid, dim3(VNT), 0, stream, s, dst, batch, rows, K, kw);
    } else {
        const int vec = (kw % 4) == 0;
        if (il) hipLaunchKernelGGL((pack_nmajor_kernel<T, 1>), grid, dim3(NT), 0, stream, s, dst, batch, rows, K, kw, vec);
        else    hipLaunchKernelGGL((pack_nmajor_kernel<T, 0>), grid, dim3(NT), 0, stream, s, dst, batch, rows, K, kw, vec);
    }
    return hipGetLastError();
}

}  // namespace

int64_t pack1bit_workgroups(int src_type, int64_t batch, int64_t rows, int64_t K, int src_k_major) {
    const int64_t eb = src_type == TCBF_SRC_I8 ? 1 : src_type == TCBF_SRC_F16 ? 2 : 4;
    return pack_workgroups(eb, batch, rows, K, src_k_major);
}

hipError_t pack1bit_launch(const void *src, int src_type, int src_layout, int64_t batch, int64_t rows,
                           int64_t K, int src_k_major, uint32_t *dst, hipStream_t stream) {
    const int il = src_layout == TCBF_INTERLEAVED;
    switch (src_type) {
    case TCBF_SRC_I8: return launch_typed<uint8_t>(src, il, batch, rows, K, src_k_major, dst, stream);
    case TCBF_SRC_F16: return launch_typed<uint16_t>(src, il, batch, rows, K, src_k_major, dst, stream);
    case TCBF_SRC_F32: return launch_typed<uint32_t>(src, il, batch, rows, K, src_k_major, dst, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tcbf
