/*
 * phgrms_oracle.h -- CPU oracle for P-HGRMS salt-and-pepper denoising.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product library
 * (include/phgrms.h) shares no source, header or table with it, and never
 * calls it.
 *
 * What it computes (P-HGRMS, Section 2 of the paper):
 *   one pass  = Algorithm 1 (cardinality matrix C of the current image I)
 *               followed by Algorithm 2 (noise test and root-mean-square
 *               replacement written into a temporary image I'), then I := I';
 *   denoise   = repeat passes until a pass changes no pixel, or k passes ran.
 *
 * Images are single-channel uint8, row-major, pitch == cols, caller-owned,
 * host memory.  Everything is integer arithmetic; single-threaded.
 *
 * Return value of every call: 0 on success, -1 on an invalid argument
 * (nothing is written in that case).
 */
#ifndef PHGRMS_ORACLE_H
#define PHGRMS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Algorithm 1: cardinality matrix.
 * card[p] = number of in-image pixels q in the (2*beta+1)^2 window centred on
 * p with  I[p]-alpha < I[q] < I[p]+alpha  (strict band, p itself included).
 * scatter_form != 0 follows the printed algorithm (each pixel p adds one to
 * every neighbour q that lies in p's band); scatter_form == 0 gathers at p.
 * Both must agree because the band relation is symmetric.
 * Domain: rows, cols >= 0; rows*cols < 2^31; 0 <= alpha <= 255; beta >= 1. */
int phgrms_oracle_cardinality(const uint8_t* img, int32_t rows, int32_t cols,
                              int32_t alpha, int32_t beta, int32_t scatter_form,
                              uint16_t* card);

/* One pass (Algorithm 1 in scatter form, then Algorithm 2).  in and out must
 * not overlap.  Returns the number of pixels whose value changed, or -1. */
int64_t phgrms_oracle_pass(const uint8_t* in, uint8_t* out, int32_t rows,
                           int32_t cols, int32_t alpha, int32_t beta);

/* Full method: passes until one changes nothing or k passes have run.
 * in == out is allowed.  changed (length >= k, may be NULL) receives the
 * per-pass changed-pixel counts; *iterations (may be NULL) the number of
 * passes executed.  Domain as above plus 0 <= k <= 1024. */
int phgrms_oracle_denoise(const uint8_t* in, uint8_t* out, int32_t rows,
                          int32_t cols, int32_t alpha, int32_t beta, int32_t k,
                          int64_t* changed, int32_t* iterations);

/* The pass loop with an opt-in extra stop rule: also stop after a pass
 * t >= 2 whose image equals the image two passes before (I_t == I_{t-2}, a
 * cycle of period 2).  Arguments and results as phgrms_oracle_denoise. */
int phgrms_oracle_denoise_cycle(const uint8_t* in, uint8_t* out, int32_t rows,
                                int32_t cols, int32_t alpha, int32_t beta, int32_t k,
                                int64_t* changed, int32_t* iterations);

/* floor(sqrt(q)) by counting up: the plain definition. */
uint32_t phgrms_oracle_isqrt(uint32_t q);

/* ---- the experiments' noise and quality measure (Section 3) ------------- */

/* The first n outputs of the SplitMix64 generator seeded with `seed`, in
 * order (state += 0x9e3779b97f4a7c15, then the output function). */
void phgrms_oracle_splitmix64(uint64_t seed, int64_t n, uint64_t* out);

/* Salt-and-pepper noise over n pixels: pixel i becomes 0 if u_i < t_pepper,
 * 255 if t_pepper <= u_i < t_salt, else keeps its value; u_i is the top 32
 * bits of output i of the generator above.  in == out is allowed. */
int phgrms_oracle_salt_pepper(const uint8_t* in, uint8_t* out, int64_t n, uint64_t seed,
                              uint32_t t_pepper, uint32_t t_salt);

/* Sum over i < n of (a[i] - b[i])^2; -1 if n < 0. */
int64_t phgrms_oracle_sq_diff_sum(const uint8_t* a, const uint8_t* b, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* PHGRMS_ORACLE_H */
