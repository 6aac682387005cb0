/*
 * phgrms_oracle.c -- plain, slow, obviously correct CPU oracle for P-HGRMS.
 *
 * TEST INFRASTRUCTURE ONLY (see phgrms_oracle.h).  It follows the paper's two
 * algorithms step by step, in the paper's order and names, one pixel at a
 * time.  It shares nothing with the GPU library.
 *
 * Readings taken where the paper's text is silent or garbled (each one is
 * checked by a test that a different reading would fail):
 *   R1  windows are inclusive: rows r-beta..r+beta, cols c-beta..c+beta.
 *   R2  Algorithm 1 uses the strict band  x-alpha < y < x+alpha.
 *   R3  Algorithm 1 increments the neighbour's entry (scatter).
 *   R4  C is recomputed from zero at every pass.
 *   R5  all comparisons in int, no uint8 wrap-around of x+-alpha.
 *   R6  Algorithm 2's "outside" test is the printed one:
 *       not (y < x+alpha+1 and y > x-alpha), i.e. outside (x-alpha, x+alpha].
 *   R7  pix_count counts every window position, in the image or not.
 *   R8  the flag > pix_count-3 test follows both window loops.
 *   R9  the replacement is the root mean square: floor(sqrt(floor(sum/flag))).
 *   R10 I' starts each pass as a copy of I (unreplaced pixels carry over).
 *   R11 every read in a pass comes from the pre-pass image (Jacobi).
 *   R12 stop after the first pass that changes no pixel, or after k passes.
 */
#include "phgrms_oracle.h"

#include <stdlib.h>
#include <string.h>

static int valid_dims(int32_t rows, int32_t cols, int32_t alpha, int32_t beta) {
  if (rows < 0 || cols < 0) return 0;
  if ((int64_t)rows * (int64_t)cols >= ((int64_t)1 << 31)) return 0;
  if (alpha < 0 || alpha > 255) return 0;
  if (beta < 1 || beta > 127) return 0; /* keeps sum < 2^32 as in 32-bit C */
  return 1;
}

static int in_image(int64_t r, int64_t c, int64_t rows, int64_t cols) {
  return r >= 0 && r < rows && c >= 0 && c < cols;
}

uint32_t phgrms_oracle_isqrt(uint32_t q) {
  uint32_t n = 0;
  while ((uint64_t)(n + 1) * (uint64_t)(n + 1) <= (uint64_t)q) n++;
  return n;
}

/* Algorithm 1 (findIsolatedPixels).  For every pixel (r,c), scan its window;
 * for every in-image neighbour (i,j) whose value lies strictly inside the
 * alpha band of d_image[r][c], add one to d_card -- at the neighbour (the
 * printed scatter form) or at (r,c) (gather form). */
static void find_isolated_pixels(const uint8_t* d_image, uint16_t* d_card,
                                 int64_t col, int64_t row, int alpha, int beta,
                                 int scatter_form) {
  memset(d_card, 0, (size_t)(row * col) * sizeof(uint16_t)); /* R4 */
  for (int64_t r = 0; r < row; r++) {
    for (int64_t c = 0; c < col; c++) {
      int x = d_image[r * col + c];
      for (int64_t i = r - beta; i < r + beta + 1; i++) {   /* R1 */
        for (int64_t j = c - beta; j < c + beta + 1; j++) {
          if (!in_image(i, j, row, col)) continue;
          int y = d_image[i * col + j];
          if (y < x + alpha && y > x - alpha) {              /* R2, R5 */
            if (scatter_form)
              d_card[i * col + j] += 1;                      /* R3 */
            else
              d_card[r * col + c] += 1;
          }
        }
      }
    }
  }
}

/* Algorithm 2 (removeNoise).  Reads d_image and d_card, writes
 * d_tempImage, which the caller has initialised to a copy of d_image. */
static void remove_noise(const uint8_t* d_image, uint8_t* d_tempImage,
                         const uint16_t* d_card, int64_t col, int64_t row,
                         int alpha, int beta) {
  for (int64_t i = 0; i < row; i++) {
    for (int64_t j = 0; j < col; j++) {
      uint64_t sum = 0;
      int64_t pix_count = 0;
      int64_t flag = 0;
      if (d_card[i * col + j] <= 2) {
        int x = d_image[i * col + j];
        for (int64_t i1 = i - beta; i1 < i + beta + 1; i1++) {
          for (int64_t j1 = j - beta; j1 < j + beta + 1; j1++) {
            pix_count = pix_count + 1;                       /* R7 */
            if (in_image(i1, j1, row, col)) {
              int y = d_image[i1 * col + j1];                /* R11 */
              if (!(y < x + alpha + 1 && y > x - alpha)) {   /* R6 */
                sum = sum + (uint64_t)(y * y);
                flag = flag + 1;
              }
            }
          }
        }
        if (flag > pix_count - 3)                            /* R8 */
          d_tempImage[i * col + j] =
              (uint8_t)phgrms_oracle_isqrt((uint32_t)(sum / (uint64_t)flag)); /* R9 */
      }
    }
  }
}

int phgrms_oracle_cardinality(const uint8_t* img, int32_t rows, int32_t cols,
                              int32_t alpha, int32_t beta, int32_t scatter_form,
                              uint16_t* card) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  if ((int64_t)rows * cols > 0 && (img == NULL || card == NULL)) return -1;
  find_isolated_pixels(img, card, cols, rows, alpha, beta, scatter_form);
  return 0;
}

int64_t phgrms_oracle_pass(const uint8_t* in, uint8_t* out, int32_t rows,
                           int32_t cols, int32_t alpha, int32_t beta) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  int64_t n = (int64_t)rows * cols;
  if (n == 0) return 0;
  if (in == NULL || out == NULL) return -1;
  uint16_t* d_card = (uint16_t*)malloc((size_t)n * sizeof(uint16_t));
  if (d_card == NULL) return -1;
  find_isolated_pixels(in, d_card, cols, rows, alpha, beta, 1);
  memcpy(out, in, (size_t)n);                                /* R10 */
  remove_noise(in, out, d_card, cols, rows, alpha, beta);
  free(d_card);
  int64_t changed = 0;
  for (int64_t p = 0; p < n; p++) changed += (out[p] != in[p]);
  return changed;
}

int phgrms_oracle_denoise(const uint8_t* in, uint8_t* out, int32_t rows,
                          int32_t cols, int32_t alpha, int32_t beta, int32_t k,
                          int64_t* changed, int32_t* iterations) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  if (k < 0 || k > 1024) return -1;
  int64_t n = (int64_t)rows * cols;
  if (n > 0 && (in == NULL || out == NULL)) return -1;
  size_t bytes = (size_t)(n > 0 ? n : 1);
  uint8_t* cur = (uint8_t*)malloc(bytes);
  uint8_t* nxt = (uint8_t*)malloc(bytes);
  if (cur == NULL || nxt == NULL) {
    free(cur);
    free(nxt);
    return -1;
  }
  if (n > 0) memcpy(cur, in, (size_t)n);
  int32_t it = 0;
  for (int32_t t = 0; t < k; t++) {
    int64_t ch = phgrms_oracle_pass(cur, nxt, rows, cols, alpha, beta);
    if (ch < 0) {
      free(cur);
      free(nxt);
      return -1;
    }
    if (changed != NULL) changed[t] = ch;
    uint8_t* tmp = cur; /* the temporary image becomes the image */
    cur = nxt;
    nxt = tmp;
    it = t + 1;
    if (ch == 0) break; /* R12 */
  }
  if (n > 0) memcpy(out, cur, (size_t)n);
  if (iterations != NULL) *iterations = it;
  free(cur);
  free(nxt);
  return 0;
}

/* The pass loop with an opt-in extra stop (a self-chosen iteration count,
 * which the paper's conclusion names as future work): besides a pass that
 * changes nothing and the cap k, stop after a pass t >= 2 whose image
 * equals the image from before pass t-1, i.e. I_t == I_{t-2}: the method has
 * entered a cycle of period 2 and every later pass alternates between the
 * two images. */
int phgrms_oracle_denoise_cycle(const uint8_t* in, uint8_t* out, int32_t rows,
                                int32_t cols, int32_t alpha, int32_t beta, int32_t k,
                                int64_t* changed, int32_t* iterations) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  if (k < 0 || k > 1024) return -1;
  int64_t n = (int64_t)rows * cols;
  if (n > 0 && (in == NULL || out == NULL)) return -1;
  size_t bytes = (size_t)(n > 0 ? n : 1);
  uint8_t* older = (uint8_t*)malloc(bytes);  /* I_{t-2} */
  uint8_t* cur = (uint8_t*)malloc(bytes);    /* I_{t-1} */
  uint8_t* nxt = (uint8_t*)malloc(bytes);    /* I_t */
  if (older == NULL || cur == NULL || nxt == NULL) {
    free(older);
    free(cur);
    free(nxt);
    return -1;
  }
  if (n > 0) memcpy(cur, in, (size_t)n);
  int32_t it = 0;
  for (int32_t t = 1; t <= k; t++) {
    int64_t ch = phgrms_oracle_pass(cur, nxt, rows, cols, alpha, beta);
    if (ch < 0) {
      free(older);
      free(cur);
      free(nxt);
      return -1;
    }
    if (changed != NULL) changed[t - 1] = ch;
    it = t;
    int same_as_older = 0;
    if (t >= 2) same_as_older = (n == 0) || memcmp(nxt, older, (size_t)n) == 0;
    uint8_t* tmp = older; /* rotate: I_{t-1} -> older, I_t -> cur */
    older = cur;
    cur = nxt;
    nxt = tmp;
    if (ch == 0 || same_as_older) break;
  }
  if (n > 0) memcpy(out, cur, (size_t)n);
  if (iterations != NULL) *iterations = it;
  free(older);
  free(cur);
  free(nxt);
  return 0;
}

/* ---- noise and quality measure of the experiments (Section 3) ----------- */

/* SplitMix64, stepped in order: add the golden-ratio increment to the
 * state, then mix it (xor-shift 30, multiply, xor-shift 27, multiply,
 * xor-shift 31) -- the generator's published definition. */
void phgrms_oracle_splitmix64(uint64_t seed, int64_t n, uint64_t* out) {
  uint64_t state = seed;
  for (int64_t i = 0; i < n; ++i) {
    state += 0x9e3779b97f4a7c15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    out[i] = z ^ (z >> 31);
  }
}

int phgrms_oracle_salt_pepper(const uint8_t* in, uint8_t* out, int64_t n, uint64_t seed,
                              uint32_t t_pepper, uint32_t t_salt) {
  if (n < 0 || t_pepper > t_salt || (n > 0 && (in == NULL || out == NULL))) return -1;
  /* the generator advances one output per pixel, in pixel order */
  uint64_t state = seed;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t r;
    phgrms_oracle_splitmix64(state, 1, &r);        /* next output ... */
    state += 0x9e3779b97f4a7c15ull;                /* ... and the state it came from */
    const uint32_t u = (uint32_t)(r >> 32);
    uint8_t v = in[i];
    if (u < t_pepper)
      v = 0;
    else if (u < t_salt)
      v = 255;
    out[i] = v;
  }
  return 0;
}

int64_t phgrms_oracle_sq_diff_sum(const uint8_t* a, const uint8_t* b, int64_t n) {
  if (n < 0 || (n > 0 && (a == NULL || b == NULL))) return -1;
  int64_t s = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = (int64_t)a[i] - (int64_t)b[i];
    s += d * d;
  }
  return s;
}
