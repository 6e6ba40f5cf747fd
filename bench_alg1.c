/*
 * bench_alg1.c -- host CPU context for the benchmark: the table method of
 * Sec. IV-A (Alg. 1) on one core with AVX-512BW byte shuffles.
 *
 * Not part of the GPU library and never called by it: bench.py times it next
 * to the plain oracle so the GPU figures can be read against the paper's own
 * CPU method on the host that runs them.
 *
 * The method: multiplying a byte of packed n-bit words by a constant c is
 * linear over GF(2) in the byte's bits, so c * b is the XOR of c times its low
 * nibble and c times its high nibble.  Two 16-entry tables per coefficient
 * hold those products for every nibble value, and a byte shuffle looks up 64
 * bytes of one table at once.
 *
 * Structure here (not the paper's loop): an encode walks the packets in
 * 64-byte columns and, for each column, keeps up to 16 coded rows in vector
 * registers while every source column is loaded once and multiplied into all
 * of them; the last partial column uses masked loads and stores.  Tables are
 * per coefficient value, so c = 0 and c = 1 go through the same lookups as
 * any other coefficient (their tables are the zero map and the identity).
 */
#define _POSIX_C_SOURCE 199309L
#include <immintrin.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

/* Reduction polynomials by word width (bit n is the x^n term). */
static const int poly_of[9] = {0, 0, 0x7, 0, 0x13, 0, 0, 0, 0x11D};

/* c * a in GF(2^n): walk the bits of c, doubling a (times x) as we go. */
static int field_mul(int n, int a, int c)
{
    if (n == 1)
        return a & c;
    int r = 0;
    for (int i = 0; i < n; i++) {
        if (c & (1 << i))
            r ^= a;
        a <<= 1;
        if (a & (1 << n))
            a ^= poly_of[n];
    }
    return r;
}

/* c applied to each n-bit word of the byte v. */
static uint8_t byte_mul(int n, int c, int v)
{
    const int mask = (1 << n) - 1;
    int out = 0;
    for (int s = 0; s < 8; s += n)
        out |= field_mul(n, (v >> s) & mask, c) << s;
    return (uint8_t)out;
}

int alg1_supported(void)
{
    __builtin_cpu_init();
    return __builtin_cpu_supports("avx512bw") ? 1 : 0;
}

/* The two lookup tables of one coefficient, each repeated in all four 128-bit
 * lanes (a byte shuffle indexes within its lane). */
typedef struct {
    __m512i low, high;
} coef_tables;

__attribute__((target("avx512f,avx512bw")))
static coef_tables tables_of(int n, int c)
{
    uint8_t lo[16], hi[16];
    for (int v = 0; v < 16; v++) {
        lo[v] = byte_mul(n, c, v);
        hi[v] = byte_mul(n, c, v << 4);
    }
    coef_tables t;
    t.low = _mm512_broadcast_i32x4(_mm_loadu_si128((const __m128i *)lo));
    t.high = _mm512_broadcast_i32x4(_mm_loadu_si128((const __m128i *)hi));
    return t;
}

/* c * v for 64 bytes: the low nibbles index one table, the high nibbles
 * (shifted down within each 32-bit word, then masked) the other. */
__attribute__((target("avx512f,avx512bw")))
static inline __m512i times(const coef_tables *t, __m512i v)
{
    const __m512i m = _mm512_set1_epi8(0x0F);
    const __m512i lo = _mm512_shuffle_epi8(t->low, _mm512_and_si512(v, m));
    const __m512i hi = _mm512_shuffle_epi8(t->high, _mm512_and_si512(_mm512_srli_epi32(v, 4), m));
    return _mm512_xor_si512(lo, hi);
}

/* Byte mask of the first `k` (<= 64) lanes. */
static inline __mmask64 first_bytes(size_t k) { return k >= 64 ? ~(__mmask64)0 : (((__mmask64)1 << k) - 1); }

/* Returns 0, or -1 for a bad field or coefficient, -2 without AVX-512BW.
 * y := y + c * x over len bytes; c = 0 touches nothing. */
__attribute__((target("avx512f,avx512bw")))
int alg1_region_madd(int n, uint8_t *y, const uint8_t *x, int c, size_t len)
{
    if (!(n == 1 || n == 2 || n == 4 || n == 8) || c < 0 || c >= (1 << n))
        return -1;
    if (!alg1_supported())
        return -2;
    if (c == 0 || len == 0)
        return 0;
    const coef_tables t = tables_of(n, c);
    size_t i = 0;
    for (; i + 128 <= len; i += 128) {   /* two independent vectors per step */
        const __m512i a0 = _mm512_loadu_si512((const void *)(x + i));
        const __m512i a1 = _mm512_loadu_si512((const void *)(x + i + 64));
        const __m512i p0 = times(&t, a0), p1 = times(&t, a1);
        _mm512_storeu_si512((void *)(y + i), _mm512_xor_si512(p0, _mm512_loadu_si512((const void *)(y + i))));
        _mm512_storeu_si512((void *)(y + i + 64),
                            _mm512_xor_si512(p1, _mm512_loadu_si512((const void *)(y + i + 64))));
    }
    for (; i < len; i += 64) {
        const __mmask64 k = first_bytes(len - i);
        const __m512i a = _mm512_maskz_loadu_epi8(k, x + i);
        const __m512i b = _mm512_maskz_loadu_epi8(k, y + i);
        _mm512_mask_storeu_epi8(y + i, k, _mm512_xor_si512(b, times(&t, a)));
    }
    return 0;
}

/* Rows k0 .. k0 + kn - 1 (kn <= 16) of Y = C S over the column [j, j + 64):
 * the accumulators stay in registers while each source column is read once. */
__attribute__((target("avx512f,avx512bw")))
static void encode_column(const coef_tables *tab, const uint8_t *C, int N, int k0, int kn, const uint8_t *S,
                          size_t ld_s, uint8_t *Y, size_t ld_y, size_t j, __mmask64 m)
{
    __m512i acc[16];
    for (int r = 0; r < 16; r++)
        acc[r] = _mm512_setzero_si512();
    const __m512i nib = _mm512_set1_epi8(0x0F);
    for (int i = 0; i < N; i++) {
        const __m512i v = _mm512_maskz_loadu_epi8(m, S + (size_t)i * ld_s + j);
        const __m512i lo = _mm512_and_si512(v, nib);                          /* shared by all rows */
        const __m512i hi = _mm512_and_si512(_mm512_srli_epi32(v, 4), nib);
        const uint8_t *ci = C + (size_t)k0 * N + i;
        for (int r = 0; r < kn; r++) {
            const coef_tables *t = &tab[ci[(size_t)r * N]];
            acc[r] = _mm512_ternarylogic_epi64(acc[r], _mm512_shuffle_epi8(t->low, lo),
                                               _mm512_shuffle_epi8(t->high, hi), 0x96);   /* a ^ b ^ c */
        }
    }
    for (int r = 0; r < kn; r++)
        _mm512_mask_storeu_epi8(Y + (size_t)(k0 + r) * ld_y + j, m, acc[r]);
}

/* Encode one generation on one core: Y (K rows of len bytes) = C S (Eq. 1).
 * The tables of every coefficient value are built once before the timed loop,
 * as a CPU library would keep them.  Returns the median seconds of `reps`
 * encodes, or < 0 on error. */
__attribute__((target("avx512f,avx512bw")))
double alg1_encode_seconds(int n, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s, uint8_t *Y,
                           size_t ld_y, size_t len, int reps)
{
    if (!(n == 1 || n == 2 || n == 4 || n == 8) || K < 1 || N < 1 || reps < 1 || reps > 64)
        return -1.0;
    if (!alg1_supported())
        return -2.0;
    for (size_t e = 0; e < (size_t)K * N; e++)
        if (C[e] >= (1 << n))
            return -1.0;
    static coef_tables tab[256];
    for (int c = 0; c < (1 << n); c++)
        tab[c] = tables_of(n, c);
    double t[64];
    for (int r = 0; r < reps; r++) {
        struct timespec a, b;
        clock_gettime(CLOCK_MONOTONIC, &a);
        for (size_t j = 0; j < len; j += 64) {
            const __mmask64 m = first_bytes(len - j);
            for (int k0 = 0; k0 < K; k0 += 16)
                encode_column(tab, C, N, k0, K - k0 < 16 ? K - k0 : 16, S, ld_s, Y, ld_y, j, m);
        }
        clock_gettime(CLOCK_MONOTONIC, &b);
        t[r] = (double)(b.tv_sec - a.tv_sec) + 1e-9 * (double)(b.tv_nsec - a.tv_nsec);
    }
    for (int i = 1; i < reps; i++)   /* insertion sort for the median */
        for (int j = i; j > 0 && t[j] < t[j - 1]; j--) {
            const double s = t[j];
            t[j] = t[j - 1];
            t[j - 1] = s;
        }
    return t[reps / 2];
}
