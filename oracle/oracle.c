/*
 * oracle.c -- plain CPU reference for the batched complex beamforming product.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may include,
 * link, load or call this file.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * helper with the GPU library: it has its own bit unpacking, its own sign rule,
 * its own FP8 decoding and its own loops.
 *
 * Everything here is written for readability, not speed: straight loops over
 * the definition, in FP64 for floating point and int64 for the 1-bit mode.
 * OpenMP only splits the outermost loops across threads; it does not change
 * the order of any sum.
 *
 * Conventions shared by all functions (plain C arrays, row-major):
 *   W  (weights)  [batch][M][K]   beams x receivers      (w_shared: one [M][K])
 *   X  (data)     [batch][K][N]   receivers x samples
 *   B  (output)   [batch][M][N]   beams x samples
 * Complex operands are passed as separate real and imaginary planes.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops below will use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORACLE_W_OFF(c, w_shared, M, K) ((w_shared) ? (int64_t)0 : (int64_t)(c) * (M) * (K))

/* ------------------------------------------------------------------------- */
/* Floating-point mode                                                        */
/* ------------------------------------------------------------------------- */

/*
 * One output entry of the beamformer, Eq. (3): y = sum_k w_k x_k over the K
 * receivers, with the complex product written out as in Sec. III-B
 * (Re = Re a Re b - Im a Im b, Im = Re a Im b + Im a Re b).  There is no
 * conjugation anywhere (Eq. (3) has none).  Sec. II maps many samples at once
 * to an M x K by K x N matrix product: M beams, N samples, K receivers.
 */
static void entry_f64(int64_t K, int64_t N, int64_t m, int64_t n,
                      const double *wr, const double *wi, /* this channel's W */
                      const double *xr, const double *xi, /* this channel's X */
                      double *out_re, double *out_im)
{
    double sr = 0.0, si = 0.0;
    for (int64_t k = 0; k < K; ++k) {
        double a_re = wr[m * K + k], a_im = wi[m * K + k];
        double b_re = xr[k * N + n], b_im = xi[k * N + n];
        sr += a_re * b_re - a_im * b_im;
        si += a_re * b_im + a_im * b_re;
    }
    *out_re = sr;
    *out_im = si;
}

/* Full product B[c] = W[c] X[c] for every c, m, n (Eq. (3), Sec. II). */
void oracle_cgemm_f64(int64_t batch, int64_t M, int64_t N, int64_t K, int w_shared,
                      const double *wr, const double *wi,
                      const double *xr, const double *xi,
                      double *br, double *bi)
{
    int64_t c, m;
#pragma omp parallel for collapse(2) schedule(static)
    for (c = 0; c < batch; ++c)
        for (m = 0; m < M; ++m) {
            const double *cwr = wr + ORACLE_W_OFF(c, w_shared, M, K);
            const double *cwi = wi + ORACLE_W_OFF(c, w_shared, M, K);
            const double *cxr = xr + c * K * N;
            const double *cxi = xi + c * K * N;
            for (int64_t n = 0; n < N; ++n) {
                int64_t o = (c * M + m) * N + n;
                entry_f64(K, N, m, n, cwr, cwi, cxr, cxi, &br[o], &bi[o]);
            }
        }
}

/* Selected entries (c[s], m[s], n[s]) of the same product, one by one. */
void oracle_cgemm_f64_entries(int64_t batch, int64_t M, int64_t N, int64_t K, int w_shared,
                              const double *wr, const double *wi,
                              const double *xr, const double *xi,
                              int64_t count, const int64_t *cs, const int64_t *ms,
                              const int64_t *ns, double *out_re, double *out_im)
{
    int64_t s;
    (void)batch;
#pragma omp parallel for schedule(static)
    for (s = 0; s < count; ++s) {
        int64_t c = cs[s];
        entry_f64(K, N, ms[s], ns[s],
                  wr + ORACLE_W_OFF(c, w_shared, M, K), wi + ORACLE_W_OFF(c, w_shared, M, K),
                  xr + c * K * N, xi + c * K * N, &out_re[s], &out_im[s]);
    }
}

/*
 * Sum of |w_k| |x_k| over k for each selected entry: the scale of the
 * floating-point summation error bound used by the tests (standard bound for
 * a recursive sum of 2K real products, each pair forming one complex term).
 */
void oracle_abs_dot_entries(int64_t M, int64_t N, int64_t K, int w_shared,
                            const double *wr, const double *wi,
                            const double *xr, const double *xi,
                            int64_t count, const int64_t *cs, const int64_t *ms,
                            const int64_t *ns, double *out)
{
    int64_t s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < count; ++s) {
        int64_t c = cs[s], m = ms[s], n = ns[s];
        const double *cwr = wr + ORACLE_W_OFF(c, w_shared, M, K);
        const double *cwi = wi + ORACLE_W_OFF(c, w_shared, M, K);
        const double *cxr = xr + c * K * N;
        const double *cxi = xi + c * K * N;
        double acc = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = hypot(cwr[m * K + k], cwi[m * K + k]);
            double b = hypot(cxr[k * N + n], cxi[k * N + n]);
            acc += a * b;
        }
        out[s] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* 1-bit mode                                                                 */
/* ------------------------------------------------------------------------- */

/*
 * Sign rule for packing (Sec. III-D: one bit per component keeps only the
 * sign; zero has no code).  A value whose sign bit is clear (including +0)
 * becomes bit 1 (+1); a value whose sign bit is set (including -0) becomes
 * bit 0 (-1).  Integer sources reach this function converted exactly to
 * double, so an integer 0 maps to +1 as well.
 */
static int sign_bit_code(double v)
{
    return signbit(v) ? 0 : 1;
}

/*
 * Packing (Sec. III, kernels paragraph): 32 consecutive 1-bit samples along K
 * go into one 32-bit word.  Sample k lands in bit (k mod 32) of word k/32
 * (least-significant bit first).  Bits past K in the last word stay 0, which
 * is the padding value of Sec. III-D (binary 0, i.e. -1).
 * vals: [rows][K] doubles;  words: [rows][kw] with kw >= ceil(K/32).
 */
void oracle_pack1bit(int64_t rows, int64_t K, int64_t kw, const double *vals, uint32_t *words)
{
    memset(words, 0, (size_t)(rows * kw) * sizeof(uint32_t));
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t k = 0; k < K; ++k)
            if (sign_bit_code(vals[r * K + k]))
                words[r * kw + k / 32] |= (uint32_t)1 << (k % 32);
}

/*
 * Inverse of the packing above.  Fig. 1: per component, bit 1 is +1 and bit 0
 * is -1 (codes 00 = -1-i, 01 = -1+i, 10 = 1-i, 11 = 1+i, real bit first).
 * vals: [rows][K] of +1/-1.
 */
void oracle_unpack1bit(int64_t rows, int64_t K, int64_t kw, const uint32_t *words, int8_t *vals)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t k = 0; k < K; ++k) {
            uint32_t bit = (words[r * kw + k / 32] >> (k % 32)) & 1u;
            vals[r * K + k] = bit ? (int8_t)1 : (int8_t)-1;
        }
}

/*
 * 1-bit product by its plain definition: the same Eq. (3) sum as the FP
 * mode, over values in {-1, +1} for each component, exact in int64.
 * W: [batch][M][K] (+-1), X: [batch][K][N] (+-1).
 */
void oracle_cgemm_1bit_def(int64_t batch, int64_t M, int64_t N, int64_t K, int w_shared,
                           const int8_t *wr, const int8_t *wi,
                           const int8_t *xr, const int8_t *xi,
                           int64_t *br, int64_t *bi)
{
    int64_t c, m;
#pragma omp parallel for collapse(2) schedule(static)
    for (c = 0; c < batch; ++c)
        for (m = 0; m < M; ++m) {
            const int8_t *cwr = wr + ORACLE_W_OFF(c, w_shared, M, K);
            const int8_t *cwi = wi + ORACLE_W_OFF(c, w_shared, M, K);
            const int8_t *cxr = xr + c * K * N;
            const int8_t *cxi = xi + c * K * N;
            for (int64_t n = 0; n < N; ++n) {
                int64_t sr = 0, si = 0;
                for (int64_t k = 0; k < K; ++k) {
                    int64_t a_re = cwr[m * K + k], a_im = cwi[m * K + k];
                    int64_t b_re = cxr[k * N + n], b_im = cxi[k * N + n];
                    sr += a_re * b_re - a_im * b_im;
                    si += a_re * b_im + a_im * b_re;
                }
                br[(c * M + m) * N + n] = sr;
                bi[(c * M + m) * N + n] = si;
            }
        }
}

/*
 * The paper's 1-bit algorithm (Sec. III-D), on packed words:
 *   real dot product of two sign vectors of length L:  L - 2 popc(A xor B)
 *   complex, with K_p = 32 * kw padded positions and K_pad = K_p - K:
 *     Re = 2 (K_p - (popc(Ar xor Br) + popc(Ai xor not Bi)))
 *     Im = 2 (K_p - K_pad - (popc(Ar xor Bi) + popc(Ai xor Br)))
 * The "K" printed in the two complex equations is read as the padded length
 * K_p (with that reading the equations reproduce the definition exactly; the
 * complement of Bi is taken over all K_p bits, pad bits included).
 * W: [batch][M][kw] words per plane, X: [batch][N][kw] words per plane
 * (X packed along K, i.e. one row of words per sample n).
 * A library popcount serves as the popc step.
 */
static void entry_1bit_popc(int64_t kw, int64_t K,
                            const uint32_t *ar, const uint32_t *ai,
                            const uint32_t *xr, const uint32_t *xi,
                            int64_t *out_re, int64_t *out_im)
{
    int64_t Kp = 32 * kw, Kpad = Kp - K;
    int64_t s_re = 0, s_im = 0;
    for (int64_t w = 0; w < kw; ++w) {
        s_re += __builtin_popcount(ar[w] ^ xr[w]) + __builtin_popcount(ai[w] ^ ~xi[w]);
        s_im += __builtin_popcount(ar[w] ^ xi[w]) + __builtin_popcount(ai[w] ^ xr[w]);
    }
    *out_re = 2 * (Kp - s_re);
    *out_im = 2 * (Kp - Kpad - s_im);
}

void oracle_cgemm_1bit_popc(int64_t batch, int64_t M, int64_t N, int64_t K, int64_t kw,
                            int w_shared,
                            const uint32_t *wr, const uint32_t *wi,
                            const uint32_t *xr, const uint32_t *xi,
                            int64_t *br, int64_t *bi)
{
    int64_t c, m;
#pragma omp parallel for collapse(2) schedule(static)
    for (c = 0; c < batch; ++c)
        for (m = 0; m < M; ++m) {
            int64_t wo = ORACLE_W_OFF(c, w_shared, M, kw) + m * kw;
            for (int64_t n = 0; n < N; ++n) {
                int64_t xo = (c * N + n) * kw;
                int64_t o = (c * M + m) * N + n;
                entry_1bit_popc(kw, K, wr + wo, wi + wo, xr + xo, xi + xo, &br[o], &bi[o]);
            }
        }
}

void oracle_cgemm_1bit_popc_entries(int64_t M, int64_t N, int64_t K, int64_t kw, int w_shared,
                                    const uint32_t *wr, const uint32_t *wi,
                                    const uint32_t *xr, const uint32_t *xi,
                                    int64_t count, const int64_t *cs, const int64_t *ms,
                                    const int64_t *ns, int64_t *out_re, int64_t *out_im)
{
    int64_t s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < count; ++s) {
        int64_t c = cs[s];
        int64_t wo = ORACLE_W_OFF(c, w_shared, M, kw) + ms[s] * kw;
        int64_t xo = (c * N + ns[s]) * kw;
        entry_1bit_popc(kw, K, wr + wo, wi + wo, xr + xo, xi + xo, &out_re[s], &out_im[s]);
    }
}

/*
 * Real 1-bit dot product of two packed sign vectors of length L (bits past L
 * are ignored by masking here), by the two forms of Sec. III-D/III-E:
 *   xor form: L - 2 popc(A xor B)
 *   and form: 2 (popc(A and B) + popc(not A and not B)) - L
 * Both must equal the sum of the +-1 products.
 */
int64_t oracle_dot1bit_xor(int64_t L, const uint32_t *a, const uint32_t *b)
{
    int64_t ones = 0;
    for (int64_t w = 0; w * 32 < L; ++w) {
        int64_t valid = L - 32 * w;
        uint32_t mask = valid >= 32 ? 0xffffffffu : (((uint32_t)1 << valid) - 1u);
        ones += __builtin_popcount((a[w] ^ b[w]) & mask);
    }
    return L - 2 * ones;
}

int64_t oracle_dot1bit_and(int64_t L, const uint32_t *a, const uint32_t *b)
{
    int64_t same = 0;
    for (int64_t w = 0; w * 32 < L; ++w) {
        int64_t valid = L - 32 * w;
        uint32_t mask = valid >= 32 ? 0xffffffffu : (((uint32_t)1 << valid) - 1u);
        same += __builtin_popcount(a[w] & b[w] & mask) + __builtin_popcount(~a[w] & ~b[w] & mask);
    }
    return 2 * same - L;
}

/* ------------------------------------------------------------------------- */
/* FP8 (e4m3) mode                                                             */
/* ------------------------------------------------------------------------- */

/*
 * OCP FP8 E4M3 (the "8-bit float" formats the paper expects to matter, Sec. VI):
 * 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; exponent 0 holds
 * subnormals m * 2^-9; exponent 15 with mantissa 7 is NaN; there are no
 * infinities and the largest finite magnitude is 448.
 */
double oracle_e4m3_decode_one(uint8_t b)
{
    int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v;
    if (e == 15 && m == 7)
        return NAN;
    v = (e == 0) ? ldexp((double)m, -9) : ldexp((double)(8 + m), e - 10);
    return s ? -v : v;
}

void oracle_e4m3_decode(int64_t n, const uint8_t *codes, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = oracle_e4m3_decode_one(codes[i]);
}

/*
 * Round a value to the nearest finite e4m3 magnitude by scanning every finite
 * code; a tie goes to the code with an even mantissa; beyond 448 it saturates.
 */
static uint8_t e4m3_round_nearest_even(float y)
{
    double a = fabs((double)y);
    int best = 0;
    double best_d = a;                       /* distance to code 0 (+0.0) */
    for (int c = 1; c <= 126; ++c) {
        double d = fabs(oracle_e4m3_decode_one((uint8_t)c) - a);
        if (d < best_d || (d == best_d && (c & 1) == 0)) {
            best = c;
            best_d = d;
        }
    }
    if (isnan(y))
        return 0x7f;
    return (uint8_t)(best | (signbit(y) ? 0x80 : 0));
}

/*
 * The library's per-row FP8 quantisation, step by step in fp32:
 *   amax  = max |x| over the row's real and imaginary parts
 *   scale = amax / 448           (1 when amax is 0)
 *   inv   = 448 / amax           (1 when amax is 0)
 *   q     = nearest-even e4m3 of (x * inv), saturating at 448
 * so that q * scale approximates x.  re, im: [rows][cols] fp32 values; one
 * scale per row.
 */
void oracle_quantize_e4m3_rows(int64_t rows, int64_t cols, const float *re, const float *im,
                               uint8_t *qre, uint8_t *qim, float *scales)
{
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < rows; ++r) {
        float amax = 0.0f, scale, inv;
        for (int64_t k = 0; k < cols; ++k) {
            float a = fabsf(re[r * cols + k]), b = fabsf(im[r * cols + k]);
            if (a > amax) amax = a;
            if (b > amax) amax = b;
        }
        scale = amax > 0.0f ? amax / 448.0f : 1.0f;
        inv = amax > 0.0f ? 448.0f / amax : 1.0f;
        scales[r] = scale;
        for (int64_t k = 0; k < cols; ++k) {
            float yr = re[r * cols + k] * inv;
            float yi = im[r * cols + k] * inv;
            qre[r * cols + k] = e4m3_round_nearest_even(yr);
            qim[r * cols + k] = e4m3_round_nearest_even(yi);
        }
    }
}

/*
 * Smallest integer e with amax <= 448 * 2^e (the power-of-two scale that
 * brings a block's largest magnitude inside the e4m3 range), found by plain
 * upward search from -127; 127 when no e up to 127 suffices (infinity), 0 for
 * an all-zero block.  E8M0 stores e + 127.
 */
static int mx_block_exponent(float amax)
{
    int e;
    if (!(amax > 0.0f))
        return 0;
    for (e = -127; e < 127; ++e)
        if ((double)amax <= 448.0 * ldexp(1.0, e))
            return e;
    return 127;
}

/*
 * The library's per-block FP8 quantisation (the OCP MX arrangement: one
 * power-of-two scale per 32 consecutive receivers of a row, shared by its real
 * and imaginary parts):
 *   amax  = max |x| over the block's real and imaginary parts (fp32, NaN ignored)
 *   e     = mx_block_exponent(amax)
 *   q     = nearest-even e4m3 of x * 2^-e (exact in double, then fp32)
 * re, im: [rows][cols]; codes: [rows][ceil(cols / 32)] holding e + 127.
 */
void oracle_quantize_e4m3_blocks(int64_t rows, int64_t cols, const float *re, const float *im,
                                 uint8_t *qre, uint8_t *qim, uint8_t *codes)
{
    const int64_t nb = (cols + 31) / 32;
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < rows; ++r) {
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t k0 = 32 * b, k1 = (k0 + 32 < cols) ? k0 + 32 : cols;
            float amax = 0.0f;
            int e;
            for (int64_t k = k0; k < k1; ++k) {
                float a = fabsf(re[r * cols + k]), c = fabsf(im[r * cols + k]);
                if (a > amax) amax = a;
                if (c > amax) amax = c;
            }
            e = mx_block_exponent(amax);
            codes[r * nb + b] = (uint8_t)(e + 127);
            for (int64_t k = k0; k < k1; ++k) {
                qre[r * cols + k] = e4m3_round_nearest_even((float)ldexp((double)re[r * cols + k], -e));
                qim[r * cols + k] = e4m3_round_nearest_even((float)ldexp((double)im[r * cols + k], -e));
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Steering weights from array geometry                                      */
/* ------------------------------------------------------------------------- */

/*
 * Far-field delay of Sec. II (Eq. 2, tau_k = d_k sin(theta) / c, written for a
 * 3-D array as the projection of the sensor position on the beam direction):
 *   s = x_k l_m + y_k m_m + z_k n_m        (metres, left to right, no fused ops)
 *   cycles = (f_c * s) / c
 * and the weight that re-aligns the phase of sensor k for beam m (Eq. 3):
 *   w = exp(+i 2 pi frac(cycles)),  frac(v) = v - floor(v)
 * positions [K][3] (x, y, z), directions [M][3] (l, m, n), freqs [batch];
 * re, im: [batch][M][K] FP64.
 */
void oracle_steering_weights(int64_t batch, int64_t M, int64_t K, const double *positions,
                             const double *directions, const double *freqs, double wave_speed,
                             double *re, double *im)
{
    int64_t cm;
    const double two_pi = 6.283185307179586;
#pragma omp parallel for schedule(static)
    for (cm = 0; cm < batch * M; ++cm) {
        const int64_t c = cm / M, m = cm % M;
        const double l = directions[3 * m], mm = directions[3 * m + 1], n = directions[3 * m + 2];
        for (int64_t k = 0; k < K; ++k) {
            double s = positions[3 * k] * l;
            double cycles, phi;
            s = s + positions[3 * k + 1] * mm;
            s = s + positions[3 * k + 2] * n;
            cycles = (freqs[c] * s) / wave_speed;
            phi = two_pi * (cycles - floor(cycles));
            re[cm * K + k] = cos(phi);
            im[cm * K + k] = sin(phi);
        }
    }
}
