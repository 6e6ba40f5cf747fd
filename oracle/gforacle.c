/*
 * gforacle.c -- plain CPU reference for GF(2^n) network-coding arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Everything here is written for clarity, not speed: each operation is its
 * textbook definition, evaluated element by element.
 *
 * Paper: Guenther, Appel, Carle, "Galois Field Arithmetics for Linear Network
 * Coding using AVX 512 Instruction Set Extensions" (arXiv 1909.02871).
 *   Sec. II      packets as vectors of n-bit words over F_q, q = 2^n; the
 *                generation matrix; encoding b = A c (Eq. 1); addition is
 *                XOR and multiplication is reduction by a field polynomial.
 *   Sec. IV-A    the madd primitive b := b + c * a and its split-nibble
 *                (shuffle) formulation, Algorithm 1.
 *   Sec. IV-B    the bit-decomposition (imul) formulation, Algorithm 2.
 *
 * The paper names no reduction polynomial.  This oracle uses
 *   GF(4):   x^2 + x + 1                     (0x7)
 *   GF(16):  x^4 + x + 1                     (0x13)
 *   GF(256): x^8 + x^4 + x^3 + x^2 + 1       (0x11D)
 * and GF(2) multiplication is logical AND.
 *
 * Packing: a byte holds 8/n words; word k occupies bits [n*k, n*k + n).
 * Decoding is not spelled out in the paper (Sec. I only says a generation may
 * fail to decode after loss); it is Gauss-Jordan elimination with the lowest
 * nonzero row as pivot.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include "gforacle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ field */

int gfo_valid_field(int n) { return n == 1 || n == 2 || n == 4 || n == 8; }

int gfo_poly(int n)
{
    switch (n) {
    case 2: return 0x7;
    case 4: return 0x13;
    case 8: return 0x11D;
    default: return 0;       /* GF(2) has no reduction step */
    }
}

/* Product of two field elements (Sec. II): the carry-less (XOR) product of
 * the two bit polynomials, then reduction by the field polynomial, cancelling
 * the highest set bit first. */
int gfo_mul(int n, int a, int b)
{
    int q = 1 << n;
    if (a < 0 || a >= q || b < 0 || b >= q)
        return -1;
    if (n == 1)
        return a & b;
    int r = 0;
    for (int i = 0; i < n; i++)
        if ((b >> i) & 1)
            r ^= a << i;
    int p = gfo_poly(n);
    for (int d = 2 * n - 2; d >= n; d--)
        if ((r >> d) & 1)
            r ^= p << (d - n);
    return r;
}

/* Second, independent multiplier ("Russian peasant"): walk the bits of b,
 * doubling a (multiplying by x and reducing immediately) at each step. */
int gfo_mul_peasant(int n, int a, int b)
{
    int q = 1 << n;
    if (a < 0 || a >= q || b < 0 || b >= q)
        return -1;
    if (n == 1)
        return a & b;
    int p = gfo_poly(n);
    int r = 0;
    while (b) {
        if (b & 1)
            r ^= a;
        a <<= 1;
        if (a & q)
            a ^= p;
        b >>= 1;
    }
    return r;
}

/* Multiplicative inverse by exhaustive search; 0 has none (returns 0). */
int gfo_inv(int n, int a)
{
    int q = 1 << n;
    if (a <= 0 || a >= q)
        return 0;
    for (int x = 1; x < q; x++)
        if (gfo_mul(n, a, x) == 1)
            return x;
    return 0;
}

/* a^e by repeated multiplication (e >= 0). */
int gfo_pow(int n, int a, int e)
{
    int r = 1;
    for (int i = 0; i < e; i++)
        r = gfo_mul(n, r, a);
    return r;
}

/* Multiply every n-bit word of byte b by the field element c (Sec. II: a
 * packet is a sequence of words; the madd primitive acts word by word). */
int gfo_mulbyte(int n, int c, int b)
{
    int mask = (1 << n) - 1, r = 0;
    for (int k = 0; k < 8 / n; k++) {
        int w = (b >> (n * k)) & mask;
        r |= gfo_mul(n, c, w) << (n * k);
    }
    return r;
}

/* ------------------------------------------------- the paper's two kernels,
 * emulated one byte at a time.  They are independent derivations of the
 * product and serve only as checks of the definition above. */

/* Sec. IV-A: low/high nibble product tables for coefficient c.  tl[x] is the
 * product of c with the byte whose low nibble is x, th[x] with the byte whose
 * high nibble is x; a byte's product is the XOR of its two lookups. */
void gfo_shuffle_tables(int n, int c, uint8_t tl[16], uint8_t th[16])
{
    for (int x = 0; x < 16; x++) {
        tl[x] = (uint8_t)gfo_mulbyte(n, c, x);
        th[x] = (uint8_t)gfo_mulbyte(n, c, x << 4);
    }
}

int gfo_shuffle_byte(int n, int c, int a)
{
    uint8_t tl[16], th[16];
    gfo_shuffle_tables(n, c, tl, th);
    return tl[a & 0x0f] ^ th[(a & 0xf0) >> 4];
}

/* Sec. IV-B: c times the i-th basis element x^i, for i < n. */
void gfo_imul_powers(int n, int c, int p[8])
{
    for (int i = 0; i < n; i++)
        p[i] = gfo_mul(n, c, 1 << i);
}

/* Sec. IV-B on one 32-bit lane: isolate bit i of every word with a mask,
 * shift it to the word's lowest bit, multiply the lane as an integer by
 * c * x^i (the words are far enough apart that no product overlaps the next
 * word), and XOR the n partial products. */
uint32_t gfo_imul_word(int n, int c, uint32_t v)
{
    int p[8];
    uint32_t unit = 0;                   /* bit 0 of every word in the lane */
    for (int k = 0; k < 32 / n; k++)
        unit |= 1u << (n * k);
    gfo_imul_powers(n, c, p);
    uint32_t r = 0;
    for (int i = 0; i < n; i++) {
        uint32_t bits = (v & (unit << i)) >> i;
        r ^= bits * (uint32_t)p[i];
    }
    return r;
}

/* ------------------------------------------------------------ region ops */

/* madd (Sec. II, Sec. IV): y := y + c * x over len bytes. */
int gfo_region_madd(int n, uint8_t *y, const uint8_t *x, int c, size_t len)
{
    if (!gfo_valid_field(n) || c < 0 || c >= (1 << n))
        return -1;
    for (size_t j = 0; j < len; j++)
        y[j] ^= (uint8_t)gfo_mulbyte(n, c, x[j]);
    return 0;
}

/* y := c * x over len bytes. */
int gfo_region_mul(int n, uint8_t *y, const uint8_t *x, int c, size_t len)
{
    if (!gfo_valid_field(n) || c < 0 || c >= (1 << n))
        return -1;
    for (size_t j = 0; j < len; j++)
        y[j] = (uint8_t)gfo_mulbyte(n, c, x[j]);
    return 0;
}

/* ---------------------------------------------------------------- encode */

/* Eq. (1) for K coding vectors at once: coded packet k is the sum over the
 * N source packets of C[k][i] times source packet i, byte by byte.
 * C is K x N row-major; S rows are ld_s bytes apart; Y rows ld_y apart. */
int gfo_encode(int n, const uint8_t *C, int K, int N,
               const uint8_t *S, size_t ld_s, uint8_t *Y, size_t ld_y, size_t len)
{
    if (!gfo_valid_field(n) || K < 0 || N < 0)
        return -1;
    for (int k = 0; k < K; k++)
        for (size_t j = 0; j < len; j++) {
            int acc = 0;
            for (int i = 0; i < N; i++)
                acc ^= gfo_mulbyte(n, C[(size_t)k * N + i], S[(size_t)i * ld_s + j]);
            Y[(size_t)k * ld_y + j] = (uint8_t)acc;
        }
    return 0;
}

/* Eq. (1) for many generations at once: generation g is gfo_encode of its
 * own coefficient matrix and sources, found through desc[8 g .. 8 g + 7] =
 * {C offset, S offset, Y offset, ld_s, ld_y, len, K, N} (byte offsets into
 * the C, S and Y blobs).  Generations are independent, so they are dealt to
 * `threads` OpenMP threads one at a time; each is the plain loop above.
 * Returns the number of threads that ran, or -1 on a bad argument. */
int gfo_encode_batch(int n, int count, const int64_t *desc, const uint8_t *C, const uint8_t *S, uint8_t *Y,
                     int threads)
{
    if (!gfo_valid_field(n) || count < 0 || threads < 1)
        return -1;
    int used = 1, bad = 0;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1) reduction(| : bad)
    for (int g = 0; g < count; g++) {
        const int64_t *d = desc + 8 * (size_t)g;
#ifdef _OPENMP
        if (g == 0)
            used = omp_get_num_threads();
#endif
        bad |= gfo_encode(n, C + d[0], (int)d[6], (int)d[7], S + d[1], (size_t)d[3], Y + d[2], (size_t)d[4],
                          (size_t)d[5]) != 0;
    }
    return bad ? -1 : used;
}

/* Matrix product over the field: R (a x c) = P (a x b) * Q (b x c). */
int gfo_matmul(int n, const uint8_t *P, const uint8_t *Q, uint8_t *R, int a, int b, int c)
{
    if (!gfo_valid_field(n))
        return -1;
    for (int i = 0; i < a; i++)
        for (int j = 0; j < c; j++) {
            int acc = 0;
            for (int t = 0; t < b; t++)
                acc ^= gfo_mul(n, P[(size_t)i * b + t], Q[(size_t)t * c + j]);
            R[(size_t)i * c + j] = (uint8_t)acc;
        }
    return 0;
}

/* Recoding (Sec. I): a node combines M coded packets it received -- each a
 * coefficient vector over the N source packets plus a payload -- with a
 * local Kout x M matrix R.  The new coefficient vectors are the element
 * product Cout = R * Cin; the new payloads are Eq. (1) applied to the
 * received payloads, Yout = R * Bin. */
int gfo_recode(int n, const uint8_t *R, int Kout, int M, int N, const uint8_t *Cin,
               const uint8_t *Bin, size_t ld_b, uint8_t *Cout, uint8_t *Yout, size_t ld_y, size_t len)
{
    if (!gfo_valid_field(n) || Kout < 0 || M < 0 || N < 0)
        return -1;
    if (gfo_matmul(n, R, Cin, Cout, Kout, M, N) != 0)
        return -1;
    return gfo_encode(n, R, Kout, M, Bin, ld_b, Yout, ld_y, len);
}

/* ------------------------------------------------------ Gauss-Jordan core */

/* Row-reduce the rows x cols matrix M in place, applying every row operation
 * to the rows x w payload D as well (D may be NULL).  Each column in turn
 * takes as pivot the lowest not-yet-used row with a nonzero entry there; the
 * pivot row is swapped up, scaled to a leading 1, and cleared from every
 * other row.  Returns the rank.  The coefficient columns cover the whole
 * field element; payload bytes are combined with the word-wise product. */
static int gauss_jordan(int n, uint8_t *M, int rows, int cols, uint8_t *D, size_t w)
{
    int prow = 0;
    for (int j = 0; j < cols && prow < rows; j++) {
        int r = -1;
        for (int i = prow; i < rows; i++)
            if (M[(size_t)i * cols + j] != 0) { r = i; break; }
        if (r < 0)
            continue;
        if (r != prow) {
            for (int t = 0; t < cols; t++) {
                uint8_t s = M[(size_t)r * cols + t];
                M[(size_t)r * cols + t] = M[(size_t)prow * cols + t];
                M[(size_t)prow * cols + t] = s;
            }
            if (D)
                for (size_t t = 0; t < w; t++) {
                    uint8_t s = D[(size_t)r * w + t];
                    D[(size_t)r * w + t] = D[(size_t)prow * w + t];
                    D[(size_t)prow * w + t] = s;
                }
        }
        int s = gfo_inv(n, M[(size_t)prow * cols + j]);
        for (int t = 0; t < cols; t++)
            M[(size_t)prow * cols + t] = (uint8_t)gfo_mul(n, s, M[(size_t)prow * cols + t]);
        if (D)
            for (size_t t = 0; t < w; t++)
                D[(size_t)prow * w + t] = (uint8_t)gfo_mulbyte(n, s, D[(size_t)prow * w + t]);
        for (int i = 0; i < rows; i++) {
            if (i == prow)
                continue;
            int f = M[(size_t)i * cols + j];
            if (f == 0)
                continue;
            for (int t = 0; t < cols; t++)
                M[(size_t)i * cols + t] ^= (uint8_t)gfo_mul(n, f, M[(size_t)prow * cols + t]);
            if (D)
                for (size_t t = 0; t < w; t++)
                    D[(size_t)i * w + t] ^= (uint8_t)gfo_mulbyte(n, f, D[(size_t)prow * w + t]);
        }
        prow++;
    }
    return prow;
}

int gfo_rank(int n, const uint8_t *M, int rows, int cols)
{
    if (!gfo_valid_field(n) || rows < 0 || cols < 0)
        return -1;
    uint8_t *W = malloc((size_t)rows * cols + 1);
    if (!W)
        return -1;
    memcpy(W, M, (size_t)rows * cols);
    int r = gauss_jordan(n, W, rows, cols, NULL, 0);
    free(W);
    return r;
}

/* Inverse of the N x N matrix C via Gauss-Jordan on [C | I].  Writes Cinv
 * only when C is invertible; returns the rank of C. */
int gfo_invert(int n, const uint8_t *C, int N, uint8_t *Cinv)
{
    if (!gfo_valid_field(n) || N < 0)
        return -1;
    uint8_t *W = malloc((size_t)N * N + 1), *I = malloc((size_t)N * N + 1);
    if (!W || !I) { free(W); free(I); return -1; }
    memcpy(W, C, (size_t)N * N);
    memset(I, 0, (size_t)N * N);
    for (int i = 0; i < N; i++)
        I[(size_t)i * N + i] = 1;
    int r = gauss_jordan(n, W, N, N, I, (size_t)N);
    if (r == N)
        memcpy(Cinv, I, (size_t)N * N);
    free(W);
    free(I);
    return r;
}

/* Decode: Gauss-Jordan on the augmented [C | B], where B holds N coded
 * packets of len bytes (rows ld_b apart).  When C has full rank the payload
 * part is the source generation and is written to S (rows ld_s apart);
 * otherwise S is left untouched.  Returns the rank of C. */
int gfo_decode(int n, const uint8_t *C, const uint8_t *B, size_t ld_b, int N,
               uint8_t *S, size_t ld_s, size_t len)
{
    if (!gfo_valid_field(n) || N < 0)
        return -1;
    uint8_t *W = malloc((size_t)N * N + 1), *D = malloc((size_t)N * len + 1);
    if (!W || !D) { free(W); free(D); return -1; }
    memcpy(W, C, (size_t)N * N);
    for (int i = 0; i < N; i++)
        memcpy(D + (size_t)i * len, B + (size_t)i * ld_b, len);
    int r = gauss_jordan(n, W, N, N, D, len);
    if (r == N)
        for (int i = 0; i < N; i++)
            memcpy(S + (size_t)i * ld_s, D + (size_t)i * len, len);
    free(W);
    free(D);
    return r;
}

/* Number of invertible N x N matrices over GF(2^n), by enumerating every
 * matrix (tiny N only: q^(N*N) matrices). Returns -1 if too large. */
long long gfo_count_invertible(int n, int N)
{
    int q = 1 << n;
    double total = 1.0;
    for (int i = 0; i < N * N; i++)
        total *= q;
    if (total > 1e8 || N < 1)
        return -1;
    long long count = 0, m = (long long)total;
    uint8_t M[64];
    for (long long code = 0; code < m; code++) {
        long long c = code;
        for (int i = 0; i < N * N; i++) {
            M[i] = (uint8_t)(c % q);
            c /= q;
        }
        if (gfo_rank(n, M, N, N) == N)
            count++;
    }
    return count;
}

/* ------------------------------------------------------ progressive decode
 * Received packets are kept in reduced row echelon form over
 * [coefficients | payload].  A new packet is first cleared against every
 * existing pivot column; if nothing is left it carries no new information.
 * Otherwise it is scaled to a leading 1, its pivot column is cleared from the
 * older rows, and it is stored.  With N pivots the payload rows, ordered by
 * pivot column, are the source packets. */
struct gfo_prog {
    int n, N;
    size_t len;
    int rank;
    int *pivot_row;      /* pivot_row[col] = stored row with pivot col, or -1 */
    uint8_t *coef;       /* N rows of N coefficients */
    uint8_t *pay;        /* N rows of len bytes */
};

gfo_prog *gfo_prog_new(int n, int N, size_t len)
{
    if (!gfo_valid_field(n) || N <= 0)
        return NULL;
    gfo_prog *p = calloc(1, sizeof *p);
    if (!p)
        return NULL;
    p->n = n; p->N = N; p->len = len; p->rank = 0;
    p->pivot_row = malloc(sizeof(int) * N);
    p->coef = calloc((size_t)N * N, 1);
    p->pay = calloc((size_t)N * len + 1, 1);
    if (!p->pivot_row || !p->coef || !p->pay) {
        gfo_prog_free(p);
        return NULL;
    }
    for (int j = 0; j < N; j++)
        p->pivot_row[j] = -1;
    return p;
}

void gfo_prog_free(gfo_prog *p)
{
    if (!p)
        return;
    free(p->pivot_row);
    free(p->coef);
    free(p->pay);
    free(p);
}

int gfo_prog_rank(const gfo_prog *p) { return p->rank; }

/* Returns 1 if the packet raised the rank, 0 if it was not innovative. */
int gfo_prog_add(gfo_prog *p, const uint8_t *c_in, const uint8_t *b_in)
{
    int n = p->n, N = p->N;
    size_t len = p->len;
    uint8_t *c = malloc((size_t)N), *b = malloc(len + 1);
    if (!c || !b) { free(c); free(b); return -1; }
    memcpy(c, c_in, (size_t)N);
    memcpy(b, b_in, len);
    for (int j = 0; j < N; j++) {
        int r = p->pivot_row[j];
        if (r < 0 || c[j] == 0)
            continue;
        int f = c[j];
        for (int t = 0; t < N; t++)
            c[t] ^= (uint8_t)gfo_mul(n, f, p->coef[(size_t)r * N + t]);
        for (size_t t = 0; t < len; t++)
            b[t] ^= (uint8_t)gfo_mulbyte(n, f, p->pay[(size_t)r * len + t]);
    }
    int lead = -1;
    for (int j = 0; j < N; j++)
        if (c[j] != 0) { lead = j; break; }
    if (lead < 0) {
        free(c); free(b);
        return 0;
    }
    int s = gfo_inv(n, c[lead]);
    for (int t = 0; t < N; t++)
        c[t] = (uint8_t)gfo_mul(n, s, c[t]);
    for (size_t t = 0; t < len; t++)
        b[t] = (uint8_t)gfo_mulbyte(n, s, b[t]);
    for (int j = 0; j < N; j++) {
        int r = p->pivot_row[j];
        if (r < 0)
            continue;
        int f = p->coef[(size_t)r * N + lead];
        if (f == 0)
            continue;
        for (int t = 0; t < N; t++)
            p->coef[(size_t)r * N + t] ^= (uint8_t)gfo_mul(n, f, c[t]);
        for (size_t t = 0; t < len; t++)
            p->pay[(size_t)r * len + t] ^= (uint8_t)gfo_mulbyte(n, f, b[t]);
    }
    int slot = p->rank;
    memcpy(p->coef + (size_t)slot * N, c, (size_t)N);
    memcpy(p->pay + (size_t)slot * len, b, len);
    p->pivot_row[lead] = slot;
    p->rank++;
    free(c); free(b);
    return 1;
}

/* When the rank is N, write the source packets (row j = pivot column j) to S
 * and return N; otherwise leave S untouched and return the rank. */
int gfo_prog_solve(const gfo_prog *p, uint8_t *S, size_t ld_s)
{
    if (p->rank < p->N)
        return p->rank;
    for (int j = 0; j < p->N; j++)
        memcpy(S + (size_t)j * ld_s, p->pay + (size_t)p->pivot_row[j] * p->len, p->len);
    return p->N;
}
