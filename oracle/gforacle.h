/*
 * gforacle.h -- plain CPU reference for GF(2^n) network-coding arithmetic.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline; never by the GPU library.  n is the number of
 * bits per field word (1, 2, 4 or 8); every byte holds 8/n words.
 */
#ifndef GFORACLE_H
#define GFORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int gfo_valid_field(int n);
int gfo_poly(int n);
int gfo_mul(int n, int a, int b);
int gfo_mul_peasant(int n, int a, int b);
int gfo_inv(int n, int a);
int gfo_pow(int n, int a, int e);
int gfo_mulbyte(int n, int c, int b);

void gfo_shuffle_tables(int n, int c, uint8_t tl[16], uint8_t th[16]);
int gfo_shuffle_byte(int n, int c, int a);
void gfo_imul_powers(int n, int c, int p[8]);
uint32_t gfo_imul_word(int n, int c, uint32_t v);

int gfo_region_madd(int n, uint8_t *y, const uint8_t *x, int c, size_t len);
int gfo_region_mul(int n, uint8_t *y, const uint8_t *x, int c, size_t len);
int gfo_encode(int n, const uint8_t *C, int K, int N,
               const uint8_t *S, size_t ld_s, uint8_t *Y, size_t ld_y, size_t len);
int gfo_encode_batch(int n, int count, const int64_t *desc, const uint8_t *C, const uint8_t *S, uint8_t *Y,
                     int threads);
int gfo_matmul(int n, const uint8_t *P, const uint8_t *Q, uint8_t *R, int a, int b, int c);
int gfo_recode(int n, const uint8_t *R, int Kout, int M, int N, const uint8_t *Cin,
               const uint8_t *Bin, size_t ld_b, uint8_t *Cout, uint8_t *Yout, size_t ld_y, size_t len);
int gfo_rank(int n, const uint8_t *M, int rows, int cols);
int gfo_invert(int n, const uint8_t *C, int N, uint8_t *Cinv);
int gfo_decode(int n, const uint8_t *C, const uint8_t *B, size_t ld_b, int N,
               uint8_t *S, size_t ld_s, size_t len);
long long gfo_count_invertible(int n, int N);

typedef struct gfo_prog gfo_prog;
gfo_prog *gfo_prog_new(int n, int N, size_t len);
void gfo_prog_free(gfo_prog *p);
int gfo_prog_rank(const gfo_prog *p);
int gfo_prog_add(gfo_prog *p, const uint8_t *c, const uint8_t *b);
int gfo_prog_solve(const gfo_prog *p, uint8_t *S, size_t ld_s);

#ifdef __cplusplus
}
#endif
#endif
