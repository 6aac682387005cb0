/*
 * phgrms_oracle.c -- plain, slow, obviously correct CPU oracle for P-HGRMS.
 *
 * TEST INFRASTRUCTURE ONLY (see phgrms_oracle.h).  It computes what Section 2
 * of the paper defines, one pixel at a time, with no blocking, fusion or
 * reordering, and shares nothing with the GPU library.
 *
 * The method, as this file reads it (each reading is checked by a test that
 * a different reading fails):
 *
 *   Window.  W(p) is the square of side 2*beta+1 centred on p, both ends
 *   included (R1); only its positions inside the image hold pixels.
 *
 *   Algorithm 1, the alpha-beta cardinality.  C(p) is the number of pixels q
 *   of W(p) (p itself included) whose grey level lies strictly inside
 *   (I(p) - alpha, I(p) + alpha) (R2), in int arithmetic with no 8-bit wrap
 *   (R5).  The paper fills C by scattering: every pixel p adds one to the
 *   entry of each neighbour in its band (R3); the band is symmetric, so the
 *   gather count at q is the same number.  C is rebuilt from zero for every
 *   pass (R4).
 *
 *   Algorithm 2, the noise test.  A pixel p with C(p) <= 2 is a candidate.
 *   For a candidate, the pixels q of W(p) whose level lies outside the
 *   half-open band (I(p) - alpha, I(p) + alpha] (R6, as printed; only
 *   d = +alpha is treated differently from the strict band) are the
 *   "outside" pixels; let F be their number and S the sum of their squared
 *   levels.  The window size M counts every position of W(p), inside the
 *   image or not (R7).  After the whole window is scanned (R8), if F > M - 3
 *   the pixel is replaced by the integer root mean square
 *   floor(sqrt(floor(S / F))) (R9); otherwise it keeps its value.
 *
 *   A pass writes the new image into a separate buffer that starts as a copy
 *   of the current one (R10), and every level it reads is a pre-pass level
 *   (R11).  Passes repeat until one changes no pixel or k passes have run
 *   (R12).
 */
#include "phgrms_oracle.h"

#include <stdlib.h>
#include <string.h>

static int valid_dims(int32_t rows, int32_t cols, int32_t alpha, int32_t beta) {
  if (rows < 0 || cols < 0) return 0;
  if ((int64_t)rows * (int64_t)cols >= ((int64_t)1 << 31)) return 0;
  if (alpha < 0 || alpha > 255) return 0;
  if (beta < 1 || beta > 127) return 0; /* keeps S < 2^32 as in 32-bit C */
  return 1;
}

/* A read-only view of one image. */
typedef struct {
  const uint8_t* level;
  int64_t rows, cols;
} image_view;

/* The grey level at (r, c) into *v; 0 if (r, c) lies outside the image. */
static int level_at(const image_view* im, int64_t r, int64_t c, int* v) {
  if (r < 0 || r >= im->rows || c < 0 || c >= im->cols) return 0;
  *v = im->level[r * im->cols + c];
  return 1;
}

uint32_t phgrms_oracle_isqrt(uint32_t q) {
  uint32_t n = 0;
  while ((uint64_t)(n + 1) * (uint64_t)(n + 1) <= (uint64_t)q) n++;
  return n;
}

/* y lies strictly inside x's alpha band (Algorithm 1). */
static int in_strict_band(int y, int x, int alpha) {
  return y > x - alpha && y < x + alpha;
}

/* y lies outside x's half-open band (x - alpha, x + alpha] (Algorithm 2). */
static int outside_band(int y, int x, int alpha) {
  return !(y > x - alpha && y <= x + alpha);
}

/* Algorithm 1: the cardinality matrix of one image.  With scatter_form, each
 * pixel p adds one to the entry of every window pixel q in p's strict band,
 * as the paper's kernel does; without it, p counts those q itself. */
static void cardinality_matrix(const image_view* im, int alpha, int beta, int scatter_form,
                               uint16_t* card) {
  memset(card, 0, (size_t)(im->rows * im->cols) * sizeof(uint16_t));
  for (int64_t r = 0; r < im->rows; r++) {
    for (int64_t c = 0; c < im->cols; c++) {
      const int x = im->level[r * im->cols + c];
      for (int di = -beta; di <= beta; di++) {
        for (int dj = -beta; dj <= beta; dj++) {
          int y;
          if (!level_at(im, r + di, c + dj, &y)) continue;
          if (!in_strict_band(y, x, alpha)) continue;
          if (scatter_form)
            card[(r + di) * im->cols + (c + dj)] += 1;
          else
            card[r * im->cols + c] += 1;
        }
      }
    }
  }
}

/* The outside pixels of the window of (r, c): their number F and the sum S
 * of their squared levels. */
typedef struct {
  int64_t count;
  uint64_t sq_sum;
} outside_pixels;

static outside_pixels scan_outside(const image_view* im, int64_t r, int64_t c, int alpha,
                                   int beta) {
  outside_pixels o = {0, 0};
  const int x = im->level[r * im->cols + c];
  for (int oy = -beta; oy <= beta; oy++) {
    for (int ox = -beta; ox <= beta; ox++) {
      int y;
      if (!level_at(im, r + oy, c + ox, &y)) continue;
      if (outside_band(y, x, alpha)) {
        o.count += 1;
        o.sq_sum += (uint64_t)y * (uint64_t)y;
      }
    }
  }
  return o;
}

/* Algorithm 2 for one pixel: its level after the pass, given C at it. */
static uint8_t noise_rule(const image_view* im, int64_t r, int64_t c, int alpha, int beta,
                          unsigned card) {
  const uint8_t x = im->level[r * im->cols + c];
  if (card > 2) return x;                      /* not a candidate */
  const int64_t side = 2 * (int64_t)beta + 1;
  const int64_t window_size = side * side;     /* every position (R7) */
  const outside_pixels o = scan_outside(im, r, c, alpha, beta);
  if (o.count <= window_size - 3) return x;
  return (uint8_t)phgrms_oracle_isqrt((uint32_t)(o.sq_sum / (uint64_t)o.count));
}

int phgrms_oracle_cardinality(const uint8_t* img, int32_t rows, int32_t cols,
                              int32_t alpha, int32_t beta, int32_t scatter_form,
                              uint16_t* card) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  if ((int64_t)rows * cols > 0 && (img == NULL || card == NULL)) return -1;
  const image_view im = {img, rows, cols};
  cardinality_matrix(&im, alpha, beta, scatter_form, card);
  return 0;
}

int64_t phgrms_oracle_pass(const uint8_t* in, uint8_t* out, int32_t rows,
                           int32_t cols, int32_t alpha, int32_t beta) {
  if (!valid_dims(rows, cols, alpha, beta)) return -1;
  int64_t n = (int64_t)rows * cols;
  if (n == 0) return 0;
  if (in == NULL || out == NULL) return -1;
  uint16_t* card = (uint16_t*)malloc((size_t)n * sizeof(uint16_t));
  if (card == NULL) return -1;
  const image_view before = {in, rows, cols};   /* every read of the pass (R11) */
  cardinality_matrix(&before, alpha, beta, 1, card);
  memcpy(out, in, (size_t)n);                   /* R10 */
  for (int64_t r = 0; r < rows; r++)
    for (int64_t c = 0; c < cols; c++)
      out[r * cols + c] = noise_rule(&before, r, c, alpha, beta, card[r * cols + c]);
  free(card);
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
  int32_t passes = 0;
  while (passes < k) {
    const int64_t moved = phgrms_oracle_pass(cur, nxt, rows, cols, alpha, beta);
    if (moved < 0) {
      free(cur);
      free(nxt);
      return -1;
    }
    if (changed != NULL) changed[passes] = moved;
    passes += 1;
    uint8_t* tmp = cur; /* the temporary image becomes the image */
    cur = nxt;
    nxt = tmp;
    if (moved == 0) break; /* R12 */
  }
  if (n > 0) memcpy(out, cur, (size_t)n);
  if (iterations != NULL) *iterations = passes;
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
