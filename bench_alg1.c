/*
 * bench_alg1.c -- host CPU context for the benchmark: the split-nibble
 * region madd of Sec. IV-A (Alg. 1) with AVX-512BW byte shuffles, on one core.
 *
 * Not part of the GPU library and never called by it: bench.py times it next
 * to the plain oracle so the GPU figures can be read against the paper's own
 * CPU method on the host that runs them.
 *
 * y := y + c * x word-wise over GF(2^n), n in {1, 2, 4, 8}.  Each byte is
 * split into its low and high nibble; two 16-entry tables per coefficient
 * hold c times every nibble value (c * v and c * (v << 4), whole bytes), and
 * one byte shuffle per nibble looks 64 of them up at once.  c = 0 does
 * nothing and c = 1 is a plain XOR, the trivial cases the paper catches first.
 */
#define _POSIX_C_SOURCE 199309L
#include <immintrin.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

static const int poly_of[9] = {0, 0, 0x7, 0, 0x13, 0, 0, 0, 0x11D};

/* c * a in GF(2^n) (shift-and-add, reduced as the top bit leaves the field). */
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

/* c applied to each n-bit word of byte v. */
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

__attribute__((target("avx512f,avx512bw")))
static void madd_shuffle(uint8_t *y, const uint8_t *x, size_t len, const uint8_t lo[16], const uint8_t hi[16])
{
    const __m512i tlo = _mm512_broadcast_i32x4(_mm_loadu_si128((const __m128i *)lo));
    const __m512i thi = _mm512_broadcast_i32x4(_mm_loadu_si128((const __m128i *)hi));
    const __m512i nib = _mm512_set1_epi8(0x0F);
    size_t i = 0;
    for (; i + 64 <= len; i += 64) {
        const __m512i v = _mm512_loadu_si512((const void *)(x + i));
        const __m512i pl = _mm512_shuffle_epi8(tlo, _mm512_and_si512(v, nib));
        const __m512i ph = _mm512_shuffle_epi8(thi, _mm512_and_si512(_mm512_srli_epi16(v, 4), nib));
        const __m512i acc = _mm512_loadu_si512((const void *)(y + i));
        _mm512_storeu_si512((void *)(y + i), _mm512_ternarylogic_epi64(acc, pl, ph, 0x96));
    }
    for (; i < len; i++)
        y[i] ^= (uint8_t)(lo[x[i] & 15] ^ hi[x[i] >> 4]);
}

__attribute__((target("avx512f,avx512bw")))
static void xor_rows(uint8_t *y, const uint8_t *x, size_t len)
{
    size_t i = 0;
    for (; i + 64 <= len; i += 64)
        _mm512_storeu_si512((void *)(y + i), _mm512_xor_si512(_mm512_loadu_si512((const void *)(y + i)),
                                                              _mm512_loadu_si512((const void *)(x + i))));
    for (; i < len; i++)
        y[i] ^= x[i];
}

/* Nibble tables of c: lo[v] = c * v, hi[v] = c * (v << 4), as whole bytes. */
static void nibble_tables(int n, int c, uint8_t lo[16], uint8_t hi[16])
{
    for (int v = 0; v < 16; v++) {
        lo[v] = byte_mul(n, c, v);
        hi[v] = byte_mul(n, c, v << 4);
    }
}

/* Returns 0, or -1 for a bad field or coefficient, -2 without AVX-512BW. */
int alg1_region_madd(int n, uint8_t *y, const uint8_t *x, int c, size_t len)
{
    if (!(n == 1 || n == 2 || n == 4 || n == 8) || c < 0 || c >= (1 << n))
        return -1;
    if (!alg1_supported())
        return -2;
    if (c == 0)
        return 0;
    if (c == 1) {
        xor_rows(y, x, len);
        return 0;
    }
    uint8_t lo[16], hi[16];
    nibble_tables(n, c, lo, hi);
    madd_shuffle(y, x, len, lo, hi);
    return 0;
}

/* Encode one generation on one core with the region madd: Y (K rows) = C S,
 * every row of Y zeroed first, then K * N madds (Eq. 1).  Tables are built
 * once per coefficient value before the timed loop, as a CPU library would
 * keep them.  Returns the median seconds of `reps` encodes, or < 0 on error. */
double alg1_encode_seconds(int n, const uint8_t *C, int K, int N, const uint8_t *S, size_t ld_s, uint8_t *Y,
                           size_t ld_y, size_t len, int reps)
{
    if (!(n == 1 || n == 2 || n == 4 || n == 8) || K < 1 || N < 1 || reps < 1 || reps > 64)
        return -1.0;
    if (!alg1_supported())
        return -2.0;
    static uint8_t lo[256][16], hi[256][16];
    for (int c = 0; c < (1 << n); c++)
        nibble_tables(n, c, lo[c], hi[c]);
    double t[64];
    for (int r = 0; r < reps; r++) {
        struct timespec a, b;
        clock_gettime(CLOCK_MONOTONIC, &a);
        for (int k = 0; k < K; k++) {
            uint8_t *yk = Y + (size_t)k * ld_y;
            memset(yk, 0, len);
            for (int i = 0; i < N; i++) {
                const int c = C[(size_t)k * N + i];
                if (c == 1)
                    xor_rows(yk, S + (size_t)i * ld_s, len);
                else if (c > 1)
                    madd_shuffle(yk, S + (size_t)i * ld_s, len, lo[c], hi[c]);
            }
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
