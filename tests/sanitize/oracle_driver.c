/*
 * Runs every function of the CPU oracle on small random and edge-case
 * images under AddressSanitizer and UndefinedBehaviorSanitizer (built and
 * run by tests/test_sanitizers.py).  It checks only what needs no second
 * implementation: results stay in [0, 255], counts are consistent, the
 * scatter and gather cardinalities agree, and a pass never changes a pixel
 * within beta of the border.  Exit status 0 when every check holds.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "phgrms_oracle.h"

static uint64_t rng_state = 0x2545F4914F6CDD1Dull;
static uint32_t next_u32(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (uint32_t)(rng_state >> 11);
}

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      failures++;                                                  \
    }                                                              \
  } while (0)

static void one_case(int rows, int cols, int alpha, int beta, int k, int mode) {
  const size_t n = (size_t)rows * (size_t)cols;
  uint8_t* img = (uint8_t*)malloc(n ? n : 1);
  uint8_t* out = (uint8_t*)malloc(n ? n : 1);
  uint8_t* one = (uint8_t*)malloc(n ? n : 1);
  uint16_t* cs = (uint16_t*)malloc((n ? n : 1) * sizeof(uint16_t));
  uint16_t* cg = (uint16_t*)malloc((n ? n : 1) * sizeof(uint16_t));
  int64_t changed[40];
  int32_t it = -1;
  for (size_t i = 0; i < n; ++i) {
    const uint32_t u = next_u32();
    img[i] = mode == 0 ? (uint8_t)u : (uint8_t)((u % 8 == 0) ? 255 * (u & 1) : 100 + (u >> 8) % 9);
  }
  CHECK(phgrms_oracle_cardinality(img, rows, cols, alpha, beta, 1, cs) == 0);
  CHECK(phgrms_oracle_cardinality(img, rows, cols, alpha, beta, 0, cg) == 0);
  CHECK(n == 0 || memcmp(cs, cg, n * sizeof(uint16_t)) == 0);
  const int64_t c1 = phgrms_oracle_pass(img, one, rows, cols, alpha, beta);
  CHECK(c1 >= 0 && (size_t)c1 <= n);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c)
      if (r < beta || c < beta || r >= rows - beta || c >= cols - beta)
        CHECK(one[(size_t)r * cols + c] == img[(size_t)r * cols + c]);
  CHECK(phgrms_oracle_denoise(img, out, rows, cols, alpha, beta, k, changed, &it) == 0);
  CHECK(it >= 0 && it <= k);
  if (k >= 1 && it >= 1) CHECK(changed[0] == c1);
  for (int t = 0; t + 1 < it; ++t) CHECK(changed[t] > 0);
  CHECK(phgrms_oracle_denoise_cycle(img, out, rows, cols, alpha, beta, k, changed, &it) == 0);
  CHECK(it >= 0 && it <= k);
  memcpy(out, img, n);
  CHECK(phgrms_oracle_denoise(out, out, rows, cols, alpha, beta, k, NULL, NULL) == 0);
  free(img);
  free(out);
  free(one);
  free(cs);
  free(cg);
}

int main(void) {
  static const int sizes[][2] = {{0, 0}, {0, 7}, {7, 0}, {1, 1}, {1, 40}, {40, 1}, {2, 2},
                                 {3, 3}, {5, 5}, {9, 13}, {17, 31}, {33, 64}};
  static const int alphas[] = {0, 1, 20, 255};
  for (size_t s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s)
    for (int beta = 1; beta <= 4; ++beta)
      for (size_t a = 0; a < sizeof(alphas) / sizeof(alphas[0]); ++a)
        for (int mode = 0; mode < 2; ++mode)
          one_case(sizes[s][0], sizes[s][1], alphas[a], beta, (int)(next_u32() % 12), mode);
  /* invalid arguments are refused and write nothing */
  uint8_t px[4] = {1, 2, 3, 4}, o[4] = {9, 9, 9, 9};
  CHECK(phgrms_oracle_denoise(px, o, 2, 2, 300, 1, 3, NULL, NULL) == -1);
  CHECK(phgrms_oracle_denoise(px, o, 2, 2, 20, 0, 3, NULL, NULL) == -1);
  CHECK(phgrms_oracle_denoise(px, o, 2, 2, 20, 1, 2000, NULL, NULL) == -1);
  CHECK(o[0] == 9 && o[3] == 9);
  CHECK(phgrms_oracle_isqrt(0) == 0 && phgrms_oracle_isqrt(65535) == 255);
  uint64_t draws[8];
  phgrms_oracle_splitmix64(1234567, 8, draws);
  uint8_t noisy[64], clean[64];
  for (int i = 0; i < 64; ++i) clean[i] = (uint8_t)(i * 3);
  CHECK(phgrms_oracle_salt_pepper(clean, noisy, 64, 99, 1u << 30, 1u << 31) == 0);
  CHECK(phgrms_oracle_sq_diff_sum(clean, noisy, 64) >= 0);
  CHECK(phgrms_oracle_sq_diff_sum(clean, noisy, -1) == -1);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle driver: all checks passed\n");
  return 0;
}
