/*
 * phgrms.h -- C ABI of the MI355X (gfx950) P-HGRMS salt-and-pepper denoiser.
 *
 * The method (Agarwal, Jha, Kanna, "P-HGRMS: A Parallel Hypergraph Based Root
 * Mean Square Algorithm for Image Denoising", Section 2) repeats one pass over
 * a grey image I:
 *
 *   Algorithm 1  cardinality C(p) = number of image pixels q in the
 *                (2*beta+1) x (2*beta+1) window of p with
 *                I(p) - alpha < I(q) < I(p) + alpha;
 *   Algorithm 2  every pixel p with C(p) <= 2 whose window holds more than
 *                N - 3 positions (N = (2*beta+1)^2, all positions counted)
 *                with I(q) outside (I(p) - alpha, I(p) + alpha] is replaced,
 *                in a temporary image I', by the root mean square of those
 *                outside pixels, floor(sqrt(floor(sum I(q)^2 / count)));
 *   then I := I'.  The loop ends after the first pass that changes no pixel,
 *   or after k passes (the iteration factor of Section 2).
 *
 * Consequences used by the implementation (they are theorems of the rules
 * above): a pixel within beta of the image border is never replaced, and an
 * interior pixel is replaced exactly when at most 2 window pixels (itself
 * included) lie in (I(p) - alpha, I(p) + alpha].
 *
 * Conventions for every call:
 *   - images are single-channel uint8, row-major, row pitch == cols, any
 *     byte alignment; "d_" pointers are device (HBM) pointers, "h_" pointers
 *     host pointers; all memory is owned by the caller;
 *   - the library never allocates device memory; work buffers come in
 *     through a caller-provided workspace;
 *   - `stream` is a hipStream_t (NULL = the null stream); work is enqueued
 *     in order on that stream;
 *   - every call returns a phgrms_status; arguments are validated before any
 *     work is enqueued, and on PHGRMS_EINVAL / PHGRMS_ENOSPC /
 *     PHGRMS_EUNSUPPORTED nothing is written.  On PHGRMS_EDEVICE the
 *     contents of the outputs are unspecified.  phgrms_last_error() returns a
 *     thread-local message for the last failing call of that thread.
 *   - calls are thread-safe as long as no two calls share a workspace.
 */
#ifndef PHGRMS_H
#define PHGRMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PHGRMS_OK = 0,
  PHGRMS_EINVAL = -1,       /* an argument is outside its domain */
  PHGRMS_ENOSPC = -2,       /* workspace (or arena) too small */
  PHGRMS_EDEVICE = -3,      /* a HIP call failed */
  PHGRMS_EUNSUPPORTED = -4, /* valid for the method, not for this GPU path */
  PHGRMS_EBUSY = -5,        /* a bounded queue is full; retry later */
  PHGRMS_ENOTFOUND = -6,    /* unknown handle or request id */
  PHGRMS_EAGAIN = -7        /* result not ready yet */
} phgrms_status;

/* Largest window radius the GPU kernels are built for. */
#define PHGRMS_BETA_MAX 4
/* Largest iteration factor accepted. */
#define PHGRMS_K_MAX 1024

/* Parameters of one image (Section 2: alpha, beta, k; image rows x cols).
 * Domain: rows >= 0, cols >= 0, rows*cols < 2^31; 0 <= alpha <= 255;
 * 1 <= beta <= PHGRMS_BETA_MAX (a larger beta is valid for the method but
 * returns PHGRMS_EUNSUPPORTED); 0 <= k <= PHGRMS_K_MAX.
 * k = 0 copies the image (iterations = 0). */
typedef struct {
  int32_t rows;
  int32_t cols;
  int32_t alpha;
  int32_t beta;
  int32_t k;
} phgrms_params;

/* Human-readable name of a status code (static storage). */
const char* phgrms_status_str(int status);
/* Thread-local message of the last failing call on this thread ("" if none). */
const char* phgrms_last_error(void);
/* Library version: major*10000 + minor*100 + patch. */
int phgrms_version(void);

/* Bytes of device workspace one phgrms_denoise / _async / _plain call
 * with these parameters needs (0 when the parameters are invalid). */
size_t phgrms_workspace_bytes(phgrms_params p);

/* Denoise one image (the whole pass loop of Section 2).
 *   d_in, d_out  device images of p.rows x p.cols bytes; d_in == d_out is
 *                allowed, any other overlap is PHGRMS_EINVAL;
 *   d_ws         device workspace of ws_bytes >= phgrms_workspace_bytes(p)
 *                bytes, not overlapping the images; contents on entry are
 *                irrelevant;
 *   h_changed    host array of at least p.k entries (may be NULL): entry t
 *                receives the number of pixels pass t changed, for t <
 *                iterations; later entries are set to 0;
 *   h_iterations host int (may be NULL): passes executed;
 *   stream       hipStream_t.
 * Depending on the tuned kernel shape, several passes run per kernel launch
 * (temporal blocking) or, with a change-tracking shape, rows whose
 * neighbourhood did not change in the previous pass are copied through
 * untested (see phgrms_run_passes); convergence is detected on the device.
 * Returns after synchronising `stream`. */
int phgrms_denoise(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                   void* d_ws, size_t ws_bytes, int64_t* h_changed,
                   int32_t* h_iterations, void* stream);

/* As phgrms_denoise, but results stay on the device and nothing
 * synchronises: d_changed (device int64[k], may be NULL) and d_iterations
 * (device int32, may be NULL) are written by the last kernel of the call.
 * The enqueued work contains no host synchronisation and no memset nodes,
 * so it may be captured into a hipGraph. */
int phgrms_denoise_async(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                         void* d_ws, size_t ws_bytes, int64_t* d_changed,
                         int32_t* d_iterations, void* stream);

/* Bytes of the library's fixed device scratch used by
 * phgrms_denoise_noalloc (one array per GPU, held until the process ends). */
#define PHGRMS_NOALLOC_SCRATCH_BYTES (96u << 20)

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * phgrms_denoise_async, with the workspace taken from a fixed device array
 * inside the library instead of a caller buffer.  The caller still passes
 * the images and (optionally) d_changed / d_iterations.  The call allocates
 * nothing.  Parameters whose workspace (phgrms_workspace_bytes(p)) exceeds
 * PHGRMS_NOALLOC_SCRATCH_BYTES return PHGRMS_ENOSPC before any work (an
 * 8192 x 8192 image with k <= 1024 fits).  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams or
 * threads) race and give undefined results; calls in one stream are
 * ordered and safe.  Results are those of phgrms_denoise_async. */
int phgrms_denoise_noalloc(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                           int64_t* d_changed, int32_t* d_iterations, void* stream);

/* Flags of phgrms_denoise_ex. */
#define PHGRMS_STOP_ON_CYCLE 1

/* phgrms_denoise_async with a different stop rule, opt-in and never the
 * default.  The paper leaves choosing the number of passes from the image
 * itself to future work (Section 4); on real images the loop rarely reaches
 * a fixed point but settles into a cycle of period 2 (pixels alternating
 * between two values), so the plain rule runs all k passes.
 *   flags  0, or PHGRMS_STOP_ON_CYCLE: also stop after the first pass t
 *          (0-based, t >= 1) whose output image equals the image two passes
 *          before it (I_{t+1} == I_{t-1}); that pass is counted in
 *          *d_iterations and its output is the result.  The zero-change stop
 *          still applies.  Other bits: PHGRMS_EINVAL.
 * Every pass before the stop computes what phgrms_denoise computes, so the
 * result equals phgrms_denoise with k = the returned iteration count.  With
 * the flag, one pass runs per kernel launch (the cycle test compares each
 * stored pixel with the image two passes before it).  Other arguments,
 * workspace size and results as phgrms_denoise_async; flags = 0 is
 * phgrms_denoise_async. */
int phgrms_denoise_ex(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                      int32_t flags, void* d_ws, size_t ws_bytes,
                      int64_t* d_changed, int32_t* d_iterations, void* stream);

/* The plain per-image path: one kernel launch per pass and a host read-back
 * of the changed count after every pass, as the paper's host loop does
 * (Section 2).  Same arguments, results and kernel arithmetic as
 * phgrms_denoise.  Returns after synchronising `stream`. */
int phgrms_denoise_plain(const uint8_t* d_in, uint8_t* d_out, phgrms_params p,
                         void* d_ws, size_t ws_bytes, int64_t* h_changed,
                         int32_t* h_iterations, void* stream);

/* Changed counts of a pass are accumulated in PHGRMS_COUNT_SLOTS int64
 * slots: each workgroup adds its count to one of 32 slots, 16 entries (one
 * cache line) apart, so that the additions of a launch do not serialise on
 * one address.  A pass's count is the sum of slots[16*s], s = 0..31. */
#define PHGRMS_COUNT_SLOTS 512

/* Bytes of the change maps of one-pass launches over a p.rows x p.cols
 * image: two maps (one per pass parity) of one byte per (row, 256-column
 * tile column), each byte stamped with its pass, then the tile lists of the
 * skipping shapes (the tiles each launch runs, listed by the launch
 * before).  0 when the parameters are invalid. */
size_t phgrms_change_map_bytes(phgrms_params p);

/* One launch of the pass kernel: `p.k` passes (1 <= p.k <= the passes per
 * launch of `shape`) from d_src to d_dst.  d_counts is a device int64 array
 * of p.k * PHGRMS_COUNT_SLOTS entries, zeroed by the caller; pass t's
 * changed count is the sum of d_counts[t*PHGRMS_COUNT_SLOTS + 16*s] over
 * s = 0..31.  d_src and d_dst must not overlap.  No convergence test, no
 * synchronisation: the building block the pass loop is made of, exposed for
 * profiling and for callers that drive passes themselves.
 *   d_maps       NULL, or device memory of phgrms_change_map_bytes(p) bytes
 *                not overlapping the images, for a change-tracking shape
 *                (phgrms_shape_tracks_changes) with p.k == 1 (else
 *                PHGRMS_EINVAL); its contents before launch 0 are
 *                irrelevant (launch 0 reads no map and every launch writes
 *                its whole map).  In a sequence of launches
 *                over one image with pass_index 0, 1, 2, ..., each launch's
 *                d_src being the previous launch's d_dst, launch i writes
 *                which rows it changed into map i % 2 and (i > 0) reads map
 *                (i - 1) % 2 to copy through, untested, the rows whose
 *                neighbourhood did not change in the previous pass (such
 *                rows cannot change: Section 2's test and root mean square
 *                see the same window as in that pass).  Results are the same
 *                with and without maps.
 *                With a skipping shape (phgrms_shape_skips_unchanged) and
 *                pass_index >= 2, d_dst must hold the image launch
 *                pass_index - 1 read (two buffers used in turn, as the pass
 *                loop does): the tiles and rows that cannot change are then
 *                neither read nor written, since d_dst already holds them.
 *   pass_index   position of this launch in such a sequence (>= 0; ignored
 *                when d_maps is NULL). */
int phgrms_run_passes(const uint8_t* d_src, uint8_t* d_dst, phgrms_params p,
                      int32_t shape, int32_t pass_index, int64_t* d_counts,
                      uint8_t* d_maps, void* stream);

/* ---- the steps around the pass loop in the experiments (Section 3) -------
 * Salt-and-pepper noise at a chosen density (the input of Tables 1-2) and
 * the sum of squared differences behind PSNR (the restoration measure of
 * Table 2).  Both are plain streams over n bytes; enqueued on `stream`, no
 * synchronisation. */

/* Salt-and-pepper noise: d_out[i] = 0 if u_i < t_pepper, 255 if
 * t_pepper <= u_i < t_salt, else d_in[i], where u_i is the top 32 bits of
 * output i (0-based) of the SplitMix64 generator seeded with `seed` (its
 * state after i+1 steps is seed + (i+1) * 0x9e3779b97f4a7c15, mixed by the
 * generator's output function).  A density rho gives about rho*n noisy
 * pixels, half of each kind, with t_salt = round(rho * 2^32) (at most
 * 2^32-1) and t_pepper = t_salt / 2.  d_in == d_out is allowed, any other
 * overlap, n < 0, t_pepper > t_salt or a null pointer with n > 0 is
 * PHGRMS_EINVAL. */
int phgrms_salt_pepper(const uint8_t* d_in, uint8_t* d_out, int64_t n, uint64_t seed,
                       uint32_t t_pepper, uint32_t t_salt, void* stream);

/* *d_sum = sum over i < n of (d_a[i] - d_b[i])^2 (device int64, written by
 * the call; exact).  PSNR = 10 log10(255^2 * n / sum), infinite for equal
 * images.  n < 0 or a null pointer is PHGRMS_EINVAL. */
int phgrms_sq_diff_sum(const uint8_t* d_a, const uint8_t* d_b, int64_t n, int64_t* d_sum,
                       void* stream);

/* Self-test of the integer routines the kernels use for Algorithm 2's root
 * mean square: floor(S/F) for every S < 2^23 and 1 <= F <= 81, and
 * floor(sqrt(q)) for every q < 2^16, each a float estimate corrected with
 * exact integer arithmetic.  d_failures: device int64[2], receives the
 * number of wrong quotients and of wrong square roots.  Enqueued on
 * `stream`, no synchronisation. */
int phgrms_selftest(int64_t* d_failures, void* stream);

/* Algorithm 1 for one image: d_card[p] = C(p) as defined above, computed by
 * gathering at p (equal to the printed scatter form because the band
 * relation is symmetric).  d_card is a device uint16 array of rows*cols
 * entries.  alpha in [0,255], 1 <= beta <= PHGRMS_BETA_MAX.  Enqueued on
 * `stream`, no synchronisation.  Test and inspection use: the denoising
 * path never materialises C. */
int phgrms_cardinality(const uint8_t* d_img, int32_t rows, int32_t cols,
                       int32_t alpha, int32_t beta, uint16_t* d_card,
                       void* stream);

/* Algorithm 1 as printed (Section 2): every pixel p adds one to the
 * cardinality of each in-image pixel q of its (2*beta+1)^2 window whose grey
 * level lies in p's strict band (I(p) - alpha, I(p) + alpha).  The paper's
 * kernel increments without atomics; here the increments are atomic (LDS,
 * then one global atomic per touched cell), so the result is exact and,
 * the band relation being symmetric, equal to phgrms_cardinality's gather
 * form.  d_card: device uint32[rows*cols], overwritten.  Same domain and
 * errors as phgrms_cardinality; test and inspection only. */
int phgrms_cardinality_scatter(const uint8_t* d_img, int32_t rows, int32_t cols,
                               int32_t alpha, int32_t beta, uint32_t* d_card, void* stream);

/* ---- many images ---------------------------------------------------------
 * A batch denoises many images of different sizes, each with its own alpha,
 * beta and k, with one multi-image pass launch per (stream, launch index,
 * beta, kernel shape) instead of one launch sequence per image: the images
 * are spread over three streams by work, forked from the caller's stream
 * and joined back before the final kernel.  Images live in caller-owned
 * device arenas at byte offsets.  The plan is immutable after creation; the
 * first phgrms_batch_run with a given set of pointers captures the launch
 * sequence into a HIP graph that later runs with the same pointers replay.
 * The plan creates its three streams and their events (default priority)
 * at its first run, on the device current then, and frees them in
 * phgrms_plan_destroy.  With a change-tracking shape each image keeps its
 * change maps in the workspace; with a skipping shape the launches of a
 * group also keep one set of tile lists over all its images and, from the
 * fourth launch on, run only the listed tiles (as for one image, see
 * phgrms_run_passes); results are the same for every shape. */

/* One image of a batch: input at in_arena + in_off, output at
 * out_arena + out_off, p.rows * p.cols bytes each. */
typedef struct {
  uint64_t in_off;
  uint64_t out_off;
  phgrms_params p;
} phgrms_item;

typedef struct phgrms_plan phgrms_plan;

/* Build a plan for n >= 1 items (host memory, copied).  Every item's
 * parameters are validated (EINVAL / EUNSUPPORTED as for phgrms_denoise).
 * *ws_bytes receives the device workspace phgrms_batch_run needs.  The
 * plan uses the batch path's kernel shapes current at creation
 * (phgrms_set_batch_tuning_class, phgrms_load_tuning), or, with a non-NULL
 * tune_cache_path, those of that tuning cache (see phgrms_load_tuning) over
 * them, for this plan only: the process's tables do not change.  A missing
 * cache file is PHGRMS_ENOTFOUND, an unreadable or invalid one
 * PHGRMS_EINVAL; no plan is made then. */
int phgrms_batch_plan(const phgrms_item* items, int32_t n, const char* tune_cache_path,
                      phgrms_plan** out, size_t* ws_bytes);

/* Run a plan.  d_in_arena / d_out_arena of in_bytes / out_bytes bytes hold
 * the images (every item's range must fit); output ranges must be pairwise
 * disjoint, and each output range either equals its own input range (in
 * place) or overlaps no input range.  d_ws: plan workspace.  d_changed:
 * device int64 array of sum(k) entries (item i's passes start at the sum of
 * the k of items before it; may be NULL); d_iterations: device int32[n] (may
 * be NULL).  Enqueued on `stream`, no synchronisation.  PHGRMS_EINVAL if
 * the arenas are too small or ranges overlap as above. */
int phgrms_batch_run(phgrms_plan* plan, const uint8_t* d_in_arena, size_t in_bytes,
                     uint8_t* d_out_arena, size_t out_bytes, void* d_ws,
                     size_t ws_bytes, int64_t* d_changed, int32_t* d_iterations,
                     void* stream);

/* Number of kernel launches one phgrms_batch_run enqueues (for reports). */
int phgrms_batch_launches(const phgrms_plan* plan);

/* Free a plan (its cached graph, streams and events; waits for its
 * streams).  NULL is ignored. */
void phgrms_plan_destroy(phgrms_plan* plan);

/* ---- serving -------------------------------------------------------------
 * A server runs a continuous-batching loop on its own thread and stream.
 * Submitted requests wait in a FIFO until their device footprint
 * (2 * rows * cols bytes plus count slots) fits under the cap and a
 * contiguous block of the caller's arena is free; admitted requests then
 * advance `passes_per_step` passes per step, all active requests of a beta in
 * one multi-image launch.  Requests join and leave at step boundaries, so
 * requests that arrive while others run share the device with them.  A
 * request's result is bit-identical to phgrms_denoise on its image alone. */

typedef struct {
  int32_t device;            /* HIP device of the arena */
  int32_t max_active;        /* admitted requests at once (>= 1) */
  int32_t passes_per_step;   /* n > 0: a compiled shape with n passes per
                                launch (the tuned one if it has n, else
                                (1, 8, 4) for 1, else the first such; n other
                                than 1, 2, 4: the tuned shape);
                                0: the tuned kernel shape's passes per launch;
                                -1: adaptive (one pass per step while fewer than
                                8 requests are active, else the batch path's
                                shape for requests admitted then) */
  int32_t max_queue;         /* pending requests before submit returns EBUSY */
  uint64_t cap_bytes;        /* admission cap on device bytes (<= arena) */
} phgrms_server_cfg;

typedef struct phgrms_server phgrms_server;

/* Start a server on the caller's device arena (d_arena, arena_bytes; the
 * caller keeps it allocated until phgrms_server_destroy returns). */
int phgrms_server_create(const phgrms_server_cfg* cfg, void* d_arena, size_t arena_bytes,
                         phgrms_server** out);

/* Queue a request.  d_img (device, p.rows * p.cols bytes) must stay valid
 * and unchanged until the request is done.  Returns PHGRMS_EINVAL for bad
 * parameters or a footprint above the cap, PHGRMS_EBUSY when the queue is
 * full.  *req_id receives the request id. */
int phgrms_server_submit(phgrms_server* s, const uint8_t* d_img, phgrms_params p,
                         uint64_t* req_id);

/* As phgrms_server_submit, for an image in host memory (the end-to-end
 * form of serving, PCIe transfers included): h_img (p.rows * p.cols bytes)
 * is copied to the request's device block in the request's first step, and
 * the final image is copied to h_out (p.rows * p.cols bytes) after its last
 * step, both on the server's stream; the latency poll reports includes both
 * copies.  h_img must stay valid and unchanged, and h_out valid, until the
 * request is done; page-locked memory (hipHostMalloc) keeps the copies
 * asynchronous.  h_img and h_out must not overlap (PHGRMS_EINVAL).  poll's
 * *d_out still points at the device copy of the result. */
int phgrms_server_submit_host(phgrms_server* s, const uint8_t* h_img, uint8_t* h_out,
                              phgrms_params p, uint64_t* req_id);

/* PHGRMS_OK when done: *d_out points at the result (rows*cols bytes in the
 * arena, valid until release), *iterations and changed[0..k) as for
 * phgrms_denoise (changed may be NULL), *latency_s the time from submit to
 * completion on the device.  PHGRMS_EAGAIN while pending or running,
 * PHGRMS_ENOTFOUND for an unknown or released id.  Never blocks on the GPU. */
int phgrms_server_poll(phgrms_server* s, uint64_t req_id, uint8_t** d_out,
                       int32_t* iterations, int64_t* changed, double* latency_s);

/* Ids of requests completed since the last call, in completion order:
 * writes up to max ids and returns how many (>= 0), or a negative status. */
int phgrms_server_next_done(phgrms_server* s, uint64_t* ids, int32_t max);

/* Free a done request's arena memory.  PHGRMS_EAGAIN if not done yet. */
int phgrms_server_release(phgrms_server* s, uint64_t req_id);

/* Counters: requests submitted, completed, currently queued and active,
 * steps run, device bytes in use. */
typedef struct {
  uint64_t submitted, completed, queued, active, steps, bytes_in_use;
} phgrms_server_stats;
int phgrms_server_get_stats(phgrms_server* s, phgrms_server_stats* st);

/* Stop the loop (pending requests are dropped, running ones finish) and
 * free the server.  NULL is ignored. */
void phgrms_server_destroy(phgrms_server* s);

/* Test hook for failure isolation: when the environment variable
 * PHGRMS_FAULT_INJECT holds a positive integer n as a server is created,
 * that server's request with id n (ids count submits from 1) fails on the
 * host just before its first launch.  Nothing of it is enqueued; its arena
 * block is freed at once; next_done reports it and poll returns
 * PHGRMS_EDEVICE for it; release forgets it.  Every other request runs as
 * usual.  Not meant for production use. */

/* ---- tuning --------------------------------------------------------------
 * The fused path runs one of a few compiled kernel shapes: T passes per
 * launch (temporal blocking, Section 2's pass loop fused T times on an
 * LDS-resident tile), R rows per wave, W waves per workgroup; the tile is
 * 256 columns wide.  These calls list the shapes and choose the one the
 * fused path (phgrms_denoise, _async, the server) uses for a beta.
 * The choice is process-wide and never changes results, only speed. */

/* Number of compiled kernel shapes. */
int phgrms_num_shapes(void);
/* Shape `shape` (0 <= shape < phgrms_num_shapes()): passes per launch, rows
 * per wave, waves per workgroup.  Returns PHGRMS_EINVAL for a bad index. */
int phgrms_shape_info(int32_t shape, int32_t* passes_per_launch,
                      int32_t* rows_per_wave, int32_t* waves);
/* 1 if shape `shape` keeps change maps (one pass per launch; rows whose
 * neighbourhood did not change in the previous pass are copied through
 * untested, see phgrms_run_passes), 0 if not, PHGRMS_EINVAL for a bad
 * index.  Only such shapes accept change maps. */
int phgrms_shape_tracks_changes(int32_t shape);
/* 1 if shape `shape` is a change-tracking shape that, from the third pass of
 * a sequence on, leaves the tiles and rows that cannot change untouched: a
 * pass writes into the buffer that holds the image from two passes before,
 * and where no pixel within beta changed in the previous pass that image
 * already equals the new one (the pixels cannot change, as above, and did
 * not change in the previous pass).  The work of a pass then scales with
 * the pixels that changed in the pass before it.  0 if not, PHGRMS_EINVAL
 * for a bad index. */
int phgrms_shape_skips_unchanged(int32_t shape);
/* Use shape `shape` for beta in the fused path, for images of every size. */
int phgrms_set_tuning(int32_t beta, int32_t shape);
/* Shape used for beta at 2^22 pixels (negative status on a bad beta). */
int phgrms_get_tuning(int32_t beta);
/* Per image size class: 0 below 2^20 pixels, 1 below 2^24, 2 from 2^24. */
int phgrms_set_tuning_class(int32_t beta, int32_t size_class, int32_t shape);
int phgrms_get_tuning_class(int32_t beta, int32_t size_class);
/* The batch path (phgrms_batch_plan) keeps its own shape per beta and size
 * class: launches over many images favour other shapes than launches over
 * one.  size_class -1 sets every class.  Applies to plans made afterwards.
 * The getter returns the shape (negative status on a bad beta or class). */
int phgrms_set_batch_tuning_class(int32_t beta, int32_t size_class, int32_t shape);
int phgrms_get_batch_tuning_class(int32_t beta, int32_t size_class);
/* Device workspace phgrms_autotune needs for these parameters (an output
 * image plus one phgrms_denoise workspace); 0 when they are invalid. */
size_t phgrms_autotune_workspace_bytes(phgrms_params p);
/* Native autotuner for one size class: time the whole pass loop (as
 * phgrms_denoise_async runs it) on the device image d_img (p.rows x p.cols)
 * with every compiled shape, one run at a time on `stream` (one untimed
 * run, then `reps` timed runs between two events), and use the fastest for
 * p.beta and the size class of p.rows * p.cols (as phgrms_set_tuning_class).
 *   d_ws, ws_bytes  device workspace of phgrms_autotune_workspace_bytes(p)
 *                   bytes, not overlapping d_img; its contents are
 *                   overwritten;
 *   reps            1..1000;
 *   best_shape      out: the chosen shape;
 *   shape_us        out (may be NULL): phgrms_num_shapes() floats, the
 *                   microseconds of one run with each shape;
 *   cache_path      NULL, or a tuning cache file (see phgrms_load_tuning):
 *                   the choice is written into it, over the entries the
 *                   file already holds (created if missing).
 * An empty image or k = 0 is PHGRMS_EINVAL (nothing to time).  Returns
 * after synchronising `stream`.  Lone runs measure latency; the Python
 * module paper_1306_5390_amd.autotune times three concurrent runs
 * (throughput) and writes its choices, with the measured rates, into the
 * same kind of cache. */
int phgrms_autotune(phgrms_params p, const uint8_t* d_img, void* d_ws, size_t ws_bytes,
                    int32_t reps, int32_t* best_shape, float* shape_us,
                    const char* cache_path, void* stream);
/* Tuning cache: a JSON file naming the kernel shape of the fused path per
 * beta and size class and of the batch path per beta (and class):
 *   {"format": "phgrms-tuning-1", "shapes": [[T, rows, waves], ...],
 *    "choice": {"<beta>": {"<class>": {"shape": s}}},
 *    "batch_choice": {"<beta>": {"shape": s, "classes": {"<class>": s}}}}
 * (every field optional; "shapes" lists the compiled shapes the indices
 * refer to, and a file whose list differs from the library's is refused;
 * other keys, such as measured rates, are ignored and kept on rewriting).
 * phgrms_load_tuning applies a cache to the process-wide tables (entries
 * the file does not name keep their values); nothing changes on an error:
 * PHGRMS_ENOTFOUND for a missing file, PHGRMS_EINVAL for an unreadable,
 * malformed or out-of-range one.  phgrms_save_tuning writes the current
 * tables to `path` (through a temporary file renamed over it), keeping the
 * other keys of a valid existing file; a file that exists but is not a
 * valid cache is left alone (PHGRMS_EINVAL). */
int phgrms_load_tuning(const char* path);
int phgrms_save_tuning(const char* path);
/* Grid of a pass launch: 0 = one workgroup per tile (default), 1 =
 * persistent, about (CUs x resident workgroups) workgroups that each walk a
 * range of tiles.  Process-wide; never changes results. */
int phgrms_set_grid_mode(int32_t mode);
int phgrms_get_grid_mode(void);

/* ---- roofline calibration ------------------------------------------------
 * Two ceilings, measured on the device the pass kernels run on; no part of
 * the method uses them.  Both are enqueued on `stream` without
 * synchronisation; the caller times them (HIP events around the call).
 *
 * phgrms_calib_copy: copies `bytes` bytes from d_src to d_dst with 16-byte
 * non-temporal vector loads and stores.  Stream-copy bandwidth = 2 * bytes /
 * duration
 * (every byte read once and written once).  Both pointers and `bytes` must
 * be multiples of 16 and the regions must not overlap, else PHGRMS_EINVAL
 * (nothing launched); bytes = 0 does nothing.
 *
 * phgrms_calib_valu: `blocks` workgroups of 256 lanes; every lane issues
 * trips x 128 (kind 8: trips x 272) vector ALU instructions of one kind on
 * independent registers
 * (the integer instructions the pass kernels issue most: 0 v_add_u32,
 * 1 v_lerp_u8 (the band test), 2 v_xor_b32, 3 v_bitop3_b32 (the counter
 * tree), 4 v_add3_u32, 5 v_alignbyte_b32, 6 v_pk_add_u16, 7 v_dot4_u32_u8
 * (the sum of squares); 8 the band test's mix: per group of four neighbour
 * words, eight v_lerp_u8, four v_xor_b32 and five v_bitop3_b32, as the
 * kernels' inner loop), then writes one word to
 * d_out (device uint32[blocks * 256], overwritten, contents meaningless).
 * *h_valu_per_wave, if not NULL, receives that count, the instructions
 * each wave issues in its loop, so that the VALU issue rate is
 * blocks * 4 * *h_valu_per_wave / duration wave-instructions per second
 * (x 64 for lane operations).  blocks in [1, 2^20], trips in [1, 2^24],
 * kind in [0, 8], else PHGRMS_EINVAL. */
int phgrms_calib_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);
int phgrms_calib_valu(uint32_t* d_out, int32_t blocks, int32_t trips, int32_t kind,
                      uint64_t* h_valu_per_wave, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PHGRMS_H */
