// phgrms.hip -- host side of the C ABI declared in include/phgrms.h:
// argument validation, workspace layout, launch sequencing of the pass loop
// (Section 2 of the paper) and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "phgrms.h"
#include "phgrms_internal.hpp"
#include "pass_kernel.hpp"

namespace phg {

namespace {
thread_local char g_err[512] = "";
}  // namespace

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PHGRMS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- kernel configurations --------------------------------------------------

// Compiled (passes per launch, rows per wave, waves per workgroup, change
// tracking) shapes.
const KernelShape kShapes[] = {
    {1, 8, 1, 0},  {1, 16, 1, 0}, {1, 8, 2, 0}, {1, 8, 4, 0}, {1, 16, 4, 0},
    {2, 16, 4, 0}, {4, 16, 4, 0}, {1, 8, 4, 1}, {1, 8, 2, 1}, {1, 4, 8, 0},
    {1, 4, 4, 0},  {1, 8, 4, 2}, {1, 8, 2, 2},
};
const int kNumShapes = int(sizeof(kShapes) / sizeof(kShapes[0]));

namespace {

std::mutex g_tune_mu;
// Shape index used by the fused path, per beta (1..PHGRMS_BETA_MAX) and
// image size class (see size_class).
int g_fused_shape[PHGRMS_BETA_MAX + 1][kSizeClasses] = {
    {3, 3, 3}, {3, 3, 3}, {3, 3, 3}, {3, 3, 3}, {3, 3, 3}};
// Batch path: the skipping (1, 8, 2) at beta = 1 and 2 (the batch
// autotuner's choice on a 512-image mixed batch, whole-batch Mpixel*iter/s
// with one beta's shape varied: at beta = 2 1.30 M against 0.92 M with
// change maps only and 0.82 M dense; at beta = 1 1.30 M against 1.24 M
// for the skipping (1, 8, 4) and 1.23 M for four dense passes per
// launch); (1, 8, 4) for larger beta.
int g_batch_shape[PHGRMS_BETA_MAX + 1][kSizeClasses] = {
    {3, 3, 3}, {12, 12, 12}, {12, 12, 12}, {3, 3, 3}, {3, 3, 3}};

template <int B, int T, int R, int W, int TRACK = 0, bool CYC = false>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&pass_kernel<B, T, R, W, TRACK, CYC>);
}

template <int B>
const void* kernel_beta(int shape) {
  switch (shape) {
    case 0: return kernel_ptr<B, 1, 8, 1>();
    case 1: return kernel_ptr<B, 1, 16, 1>();
    case 2: return kernel_ptr<B, 1, 8, 2>();
    case 3: return kernel_ptr<B, 1, 8, 4>();
    case 4: return kernel_ptr<B, 1, 16, 4>();
    case 5: return kernel_ptr<B, 2, 16, 4>();
    case 6: return kernel_ptr<B, 4, 16, 4>();
    case 7: return kernel_ptr<B, 1, 8, 4, 1>();
    case 8: return kernel_ptr<B, 1, 8, 2, 1>();
    case 9: return kernel_ptr<B, 1, 4, 8>();
    case 10: return kernel_ptr<B, 1, 4, 4>();
    case 11: return kernel_ptr<B, 1, 8, 4, 2>();
    case 12: return kernel_ptr<B, 1, 8, 2, 2>();
    default: return nullptr;
  }
}

const void* pass_kernel_ptr(int beta, int shape) {
  switch (beta) {
    case 1: return kernel_beta<1>(shape);
    case 2: return kernel_beta<2>(shape);
    case 3: return kernel_beta<3>(shape);
    case 4: return kernel_beta<4>(shape);
    default: return nullptr;
  }
}

// The skipping shapes' kernel for launch `seq` of a sequence (see
// TileLists): plain change tracking for launches 0 and 1 (the pass loop
// runs them with the dense kernel instead), the list-keeping kernel
// over every tile for launch 2, over the listed tiles from launch 3.
template <int B>
const void* skip_kernel_beta(int shape, int seq) {
  if (shape == 11)
    return seq < 2 ? kernel_ptr<B, 1, 8, 4, 1>() : seq == 2 ? kernel_ptr<B, 1, 8, 4, 2>()
                                                           : kernel_ptr<B, 1, 8, 4, 3>();
  if (shape == 12)
    return seq < 2 ? kernel_ptr<B, 1, 8, 2, 1>() : seq == 2 ? kernel_ptr<B, 1, 8, 2, 2>()
                                                           : kernel_ptr<B, 1, 8, 2, 3>();
  return nullptr;
}

const void* skip_kernel_ptr(int beta, int shape, int seq) {
  switch (beta) {
    case 1: return skip_kernel_beta<1>(shape, seq);
    case 2: return skip_kernel_beta<2>(shape, seq);
    case 3: return skip_kernel_beta<3>(shape, seq);
    case 4: return skip_kernel_beta<4>(shape, seq);
    default: return nullptr;
  }
}

// Launches over listed tiles (skipping shapes, launch 3 on).
bool listed_launch(int shape, const PassArgs& a) {
  return kShapes[shape].track == 2 && a.list_state != nullptr && a.map_in != nullptr && a.seq >= 3;
}

// Variants of the period-2 stop (the pixels that differ from the image two
// passes before are counted at the store): shapes 3 and 7, (1, 8, 4) without
// and with change tracking, and the skipping shapes 11 and 12 (launch `seq`
// of their sequence, as skip_kernel_ptr).
static_assert(kDefaultShape == 3, "the period-2 variants are built for the default shape");
template <int B>
const void* cycle_kernel_beta(int shape, int seq) {
  if (shape == 3) return kernel_ptr<B, 1, 8, 4, 0, true>();
  if (shape == 7) return kernel_ptr<B, 1, 8, 4, 1, true>();
  if (shape == 11)
    return seq < 2 ? kernel_ptr<B, 1, 8, 4, 1, true>() : seq == 2 ? kernel_ptr<B, 1, 8, 4, 2, true>()
                                                                 : kernel_ptr<B, 1, 8, 4, 3, true>();
  if (shape == 12)
    return seq < 2 ? kernel_ptr<B, 1, 8, 2, 1, true>() : seq == 2 ? kernel_ptr<B, 1, 8, 2, 2, true>()
                                                                 : kernel_ptr<B, 1, 8, 2, 3, true>();
  return nullptr;
}

const void* cycle_kernel_ptr(int beta, int shape, int seq = 0) {
  switch (beta) {
    case 1: return cycle_kernel_beta<1>(shape, seq);
    case 2: return cycle_kernel_beta<2>(shape, seq);
    case 3: return cycle_kernel_beta<3>(shape, seq);
    case 4: return cycle_kernel_beta<4>(shape, seq);
    default: return nullptr;
  }
}

// Resident workgroups per CU for each (beta, shape), and CUs per device,
// queried once.
std::mutex g_occ_mu;
int g_occ[PHGRMS_BETA_MAX + 1][16][3];   // [beta][shape][plain, listed, listed period-2 kernel]
int g_cus[64];
// 0: one workgroup per tile; 1: persistent (CUs x resident workgroups).
int g_grid_mode = 0;

hipError_t launch_pass(int beta, int shape, const PassArgs& a, hipStream_t s) {
  // a launch over listed tiles: as many workgroups as fit on the device at
  // once, each taking its share of the list (which tiles run is known on
  // the device only)
  const bool listed = listed_launch(shape, a);
  const void* k = a.diff2 != nullptr ? cycle_kernel_ptr(beta, shape, a.seq)
                  : (kShapes[shape].track == 2 && a.list_state != nullptr)
                      ? skip_kernel_ptr(beta, shape, a.seq)
                      : pass_kernel_ptr(beta, shape);
  if (k == nullptr) return hipErrorInvalidValue;
  const int grid = pass_grid(beta, shape, a.ntiles, listed, a.diff2 != nullptr);
  if (grid <= 0) return hipErrorInvalidValue;
  void* args[] = {const_cast<PassArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(kShapes[shape].waves * 64), args, 0, s);
}

}  // namespace

int pass_grid(int beta, int shape, long long ntiles, bool persistent, bool cycle) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  int occ, cus;
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    if (g_cus[dev] == 0) {
      int n = 0;
      if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
      g_cus[dev] = n;
    }
    // the listed kernel's occupancy (its period-2 variant's apart)
    const void* lkern = cycle ? cycle_kernel_ptr(beta, shape, 3) : skip_kernel_ptr(beta, shape, 3);
    const int m = (persistent && lkern != nullptr) ? (cycle ? 2 : 1) : 0;
    if (g_occ[beta][shape][m] == 0) {
      int nb = 0;
      const void* k = m ? lkern : pass_kernel_ptr(beta, shape);
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kShapes[shape].waves * 64, 0) !=
          hipSuccess)
        return -1;
      g_occ[beta][shape][m] = nb > 0 ? nb : 1;
    }
    occ = g_occ[beta][shape][m];
    cus = g_cus[dev];
  }
  // Multiples of 8 so that every XCD gets the same number of workgroups.
  const long long need = (ntiles + 7) / 8 * 8;
  long long g = need;
  int mode;
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    mode = g_grid_mode;
  }
  if (mode == 1 && !persistent && (long long)occ * cus < g) g = (long long)occ * cus;
  // A launch over listed tiles: kListedOversubscription times as many
  // workgroups as fit on the device at once.  A workgroup that finds no
  // entry leaves at once, and the dispatcher hands the slots of finished
  // workgroups to waiting ones, which evens out the tiles' uneven cost
  // (measured: 0.82 against 0.83 ms at 8192^2, 3.08 against 3.23 ms at
  // 16384^2 with one resident grid; a grid of half or three quarters of
  // the resident one, or one workgroup per tile of the image, is slower).
  if (persistent) g = (long long)occ * cus * kListedOversubscription;
  g = std::min(g, max_workgroups(kShapes[shape].waves * 64));
  // (a launch over listed tiles takes whole groups of kListShards)
  const long long gm = persistent ? kListShards : 8;
  g = g / gm * gm;
  if (g < gm) g = gm;
  return int(g);
}

TileGeom tile_geom(const phgrms_params& p, int shape) {
  const KernelShape& k = kShapes[shape];
  TileGeom g;
  g.T = k.T;
  g.TH = k.waves * k.rows - 2 * (k.T - 1) * p.beta;
  g.TW = 256 - 2 * (k.T - 1) * p.beta;
  // (64-bit: an image side near 2^31 must not overflow the rounding up)
  g.tiles_x = int((static_cast<long long>(p.cols) + g.TW - 1) / g.TW);
  g.tiles_y = int((static_cast<long long>(p.rows) + g.TH - 1) / g.TH);
  g.ntiles = (long long)g.tiles_x * g.tiles_y;
  return g;
}

int set_grid_mode(int mode) {
  if (mode != 0 && mode != 1) return fail(PHGRMS_EINVAL, "bad grid mode %d", mode);
  std::lock_guard<std::mutex> lk(g_occ_mu);
  g_grid_mode = mode;
  return PHGRMS_OK;
}

int grid_mode() {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  return g_grid_mode;
}

int size_class(long long npx) {
  return npx < (1ll << 20) ? 0 : (npx < (1ll << 24) ? 1 : 2);
}

int fused_shape(int beta, long long npx) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_fused_shape[beta][size_class(npx)];
}

int batch_shape(int beta, long long npx) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_batch_shape[beta][size_class(npx)];
}

int set_batch_shape(int beta, int cls, int shape) {
  if (beta < 1 || beta > PHGRMS_BETA_MAX || shape < 0 || shape >= kNumShapes || cls < -1 ||
      cls >= kSizeClasses)
    return fail(PHGRMS_EINVAL, "bad batch tuning (beta %d, class %d, shape %d)", beta, cls, shape);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int c = 0; c < kSizeClasses; ++c)
    if (cls < 0 || c == cls) g_batch_shape[beta][c] = shape;
  return PHGRMS_OK;
}

TuneTables current_tuning() {
  TuneTables t;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::memcpy(t.fused, g_fused_shape, sizeof(t.fused));
  std::memcpy(t.batch, g_batch_shape, sizeof(t.batch));
  return t;
}

void apply_tuning(const TuneTables& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::memcpy(g_fused_shape, t.fused, sizeof(t.fused));
  std::memcpy(g_batch_shape, t.batch, sizeof(t.batch));
}

// The plain path runs one pass per launch: the tuned shape if it is a
// single-pass shape, else the default single-pass shape.
int plain_shape(int beta, long long npx) {
  const int s = fused_shape(beta, npx);
  return (kShapes[s].T == 1 && !kShapes[s].track) ? s : kDefaultShape;
}

int validate_params(const phgrms_params& p) {
  if (p.rows < 0 || p.cols < 0)
    return fail(PHGRMS_EINVAL, "rows (%d) and cols (%d) must be >= 0", p.rows, p.cols);
  if ((int64_t)p.rows * (int64_t)p.cols >= (int64_t(1) << 31))
    return fail(PHGRMS_EINVAL, "rows*cols must be < 2^31");
  if (p.alpha < 0 || p.alpha > 255) return fail(PHGRMS_EINVAL, "alpha %d not in [0,255]", p.alpha);
  if (p.beta < 1) return fail(PHGRMS_EINVAL, "beta %d must be >= 1", p.beta);
  if (p.k < 0 || p.k > PHGRMS_K_MAX)
    return fail(PHGRMS_EINVAL, "k %d not in [0,%d]", p.k, PHGRMS_K_MAX);
  if (p.beta > PHGRMS_BETA_MAX)
    return fail(PHGRMS_EUNSUPPORTED, "beta %d > %d is not built for the GPU", p.beta,
                PHGRMS_BETA_MAX);
  return PHGRMS_OK;
}

WsLayout ws_layout(const phgrms_params& p) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  WsLayout l;
  l.state_off = 0;
  l.counts_off = 256;
  l.diff_off = l.counts_off + sizeof(uint64_t) * size_t(kCountSlots) * size_t(std::max(p.k, 1));
  l.changed_off = l.diff_off + sizeof(uint64_t) * size_t(kCountSlots) * size_t(std::max(p.k, 1));
  l.img_off = l.changed_off + up(sizeof(uint64_t) * size_t(std::max(p.k, 1)));
  l.map_off = l.img_off + up(size_t(std::max<int64_t>((int64_t)p.rows * p.cols, 1)));
  l.map_bytes = change_map_bytes(p.rows, p.cols);
  l.total = l.map_off + up(std::max<size_t>(l.map_bytes, 1));
  return l;
}

size_t map_half_bytes(int rows, int cols) {
  return size_t(std::max(rows, 0)) * ((size_t(std::max(cols, 0)) + 255) / 256);
}

int list_capacity(int rows, int cols) {
  // the skipping shapes own at least 16 rows per tile
  return int(((size_t(std::max(rows, 0)) + 15) / 16) * ((size_t(std::max(cols, 0)) + 255) / 256));
}

size_t list_state_offset(int rows, int cols) {
  return (2 * map_half_bytes(rows, cols) + 255) & ~size_t(255);
}

long long list_clear_u64(int rows, int cols) {
  // the counts and the marks (TileLists::kHead is even)
  return (long long)((size_t(TileLists::kHead) + size_t(list_capacity(rows, cols)) + 1) / 2);
}

size_t change_map_bytes(int rows, int cols) {
  return list_state_offset(rows, cols) + 4 * TileLists::words(list_capacity(rows, cols));
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

int check_buffers(const uint8_t* d_in, const uint8_t* d_out, const phgrms_params& p,
                  const void* d_ws, size_t ws_bytes) {
  const size_t n = size_t((int64_t)p.rows * p.cols);
  const WsLayout l = ws_layout(p);
  if (n > 0 && (d_in == nullptr || d_out == nullptr))
    return fail(PHGRMS_EINVAL, "null image pointer");
  if (d_ws == nullptr) return fail(PHGRMS_EINVAL, "null workspace");
  if (ws_bytes < l.total)
    return fail(PHGRMS_ENOSPC, "workspace of %zu bytes, %zu needed", ws_bytes, l.total);
  if (d_in != d_out && overlaps(d_in, n, d_out, n))
    return fail(PHGRMS_EINVAL, "input and output overlap without being the same buffer");
  if (overlaps(d_ws, l.total, d_in, n) || overlaps(d_ws, l.total, d_out, n))
    return fail(PHGRMS_EINVAL, "workspace overlaps an image");
  return PHGRMS_OK;
}

// Enqueue the whole pass loop: zero changed[], ceil(k/T) pass launches
// alternating between d_out and the workspace image, then the finish kernel
// that derives the iteration count and leaves the result in d_out.
// With diff2 (slots right after `counts`; shapes with a period-2 variant),
// the run also stops after a pass whose image equals the image two passes
// before.
int enqueue_denoise(const uint8_t* d_in, uint8_t* d_out, const phgrms_params& p, int shape,
                    uint8_t* ws_img, unsigned long long* counts, unsigned long long* changed,
                    int* iterations, uint8_t* maps, hipStream_t s,
                    unsigned long long* diff2) {
  const long long n = (long long)p.rows * p.cols;
  hipError_t e;
  if (diff2 != nullptr && cycle_kernel_ptr(p.beta, shape) == nullptr)
    return fail(PHGRMS_EINVAL, "no period-2 variant of kernel shape %d", shape);
  const bool lists = maps != nullptr && kShapes[shape].track == 2;
  if (p.k > 0) {
    // counts and (directly after them) the period-2 slots; for a skipping
    // shape also the tile lists' counts and marks
    const long long nc = (long long)p.k * kCountSlots * (diff2 != nullptr ? 2 : 1);
    const long long nl = lists ? list_clear_u64(p.rows, p.cols) : 0;
    hipLaunchKernelGGL(zero2_u64_kernel,
                       dim3(int(std::min<long long>((nc + nl + 255) / 256, 1024))), dim3(256), 0, s,
                       counts, nc,
                       reinterpret_cast<unsigned long long*>(maps + list_state_offset(p.rows, p.cols)),
                       nl);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "init launch");
  }
  const TileGeom g = tile_geom(p, shape);
  const int L = (p.k + g.T - 1) / g.T;
  auto dst_of = [&](int j) -> uint8_t* { return ((L - 1 - j) % 2 == 0) ? d_out : ws_img; };
  const uint8_t* src = d_in;
  const uint8_t* src0 = d_in;    // source of launch 0 (after staging)
  if (n > 0 && L > 0 && d_in == d_out && dst_of(0) == d_out) {
    // Launch 0 must not write the buffer it reads: stage the input first.
    const int blocks = int(std::min<long long>((n / 4 + 255) / 256 + 1, 4096));
    hipLaunchKernelGGL(copy_bytes_kernel, dim3(blocks), dim3(256), 0, s, d_in, ws_img, n);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "stage launch");
    src = ws_img;
    src0 = ws_img;
  }
  if (n > 0) {
    for (int j = 0; j < L; ++j) {
      PassArgs a;
      a.src = src;
      a.dst = dst_of(j);
      a.changed = counts;
      a.rows = p.rows;
      a.cols = p.cols;
      a.alpha = p.alpha;
      a.pass0 = j * g.T;
      a.npasses = std::min(g.T, p.k - j * g.T);
      a.tiles_x = g.tiles_x;
      a.ntiles = int(g.ntiles);
      // one-pass launches keep change maps (alternating halves of `maps`).
      // The first kDenseFirstLaunches launches of such a loop run the dense
      // one-pass kernel instead: early passes change pixels all over the
      // image, so nearly every row would be tested anyway, and the dense
      // kernel has none of the map bookkeeping.  They write no map, so the
      // launch after them tests every row as well.
      const size_t half = map_half_bytes(p.rows, p.cols);
      const bool track = maps != nullptr && g.T == 1 && kShapes[shape].track;
      const bool dense0 = track && j < kDenseFirstLaunches;
      if (dense0) {
        const TileGeom gd = tile_geom(p, kDefaultShape);
        a.tiles_x = gd.tiles_x;
        a.ntiles = int(gd.ntiles);
      }
      a.map_in = (track && j > kDenseFirstLaunches) ? maps + size_t((j - 1) & 1) * half : nullptr;
      a.map_out = (track && !dense0) ? maps + size_t(j & 1) * half : nullptr;
      a.seq = j;
      a.list_state = (track && lists && !dense0)
                         ? reinterpret_cast<uint32_t*>(maps + list_state_offset(p.rows, p.cols))
                         : nullptr;
      a.list_cap = list_capacity(p.rows, p.cols);
      // image two passes before this launch's output: launch 0's source for
      // launch 1, the destination's own contents (launch j-2's output) later
      a.diff2 = diff2;
      a.prev2 = (diff2 == nullptr || j == 0) ? nullptr : (j == 1 ? src0 : a.dst);
      // (skipping shapes: from launch 2 on, the destination holds the
      // output of launch j-2, which is kept where nothing can change)
      if ((e = launch_pass(p.beta, dense0 ? kDefaultShape : shape, a, s)) != hipSuccess)
        return hip_fail(e, "pass launch");
      src = a.dst;
    }
  }
  FinishArgs f;
  f.counts = counts;
  f.diff2 = diff2;
  f.changed = changed;
  f.k = p.k;
  f.T = g.T;
  f.launches = L;
  f.buf_even_from_end = d_out;
  f.buf_odd_from_end = ws_img;
  f.first_src = d_in;
  f.out = d_out;
  f.n = n;
  f.iterations = iterations;
  // Every block re-derives the iteration count from the count slots; a
  // moved image (rare) is copied grid-stride.
  const int fblocks = int(std::min<long long>((n / 16 + 255) / 256 + 1, 1024));
  hipLaunchKernelGGL(finish_kernel, dim3(fblocks), dim3(256), 0, s, f);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "finish launch");
  return PHGRMS_OK;
}

int set_fused_shape(int beta, int cls, int shape) {
  if (beta < 1 || beta > PHGRMS_BETA_MAX || shape < 0 || shape >= kNumShapes || cls < -1 ||
      cls >= kSizeClasses)
    return fail(PHGRMS_EINVAL, "bad tuning (beta %d, class %d, shape %d)", beta, cls, shape);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int c = 0; c < kSizeClasses; ++c)
    if (cls < 0 || c == cls) g_fused_shape[beta][c] = shape;
  return PHGRMS_OK;
}

}  // namespace phg

using namespace phg;

extern "C" {

const char* phgrms_status_str(int status) {
  switch (status) {
    case PHGRMS_OK: return "PHGRMS_OK";
    case PHGRMS_EINVAL: return "PHGRMS_EINVAL";
    case PHGRMS_ENOSPC: return "PHGRMS_ENOSPC";
    case PHGRMS_EDEVICE: return "PHGRMS_EDEVICE";
    case PHGRMS_EUNSUPPORTED: return "PHGRMS_EUNSUPPORTED";
    case PHGRMS_EBUSY: return "PHGRMS_EBUSY";
    case PHGRMS_ENOTFOUND: return "PHGRMS_ENOTFOUND";
    case PHGRMS_EAGAIN: return "PHGRMS_EAGAIN";
    default: return "PHGRMS_UNKNOWN";
  }
}

const char* phgrms_last_error(void) { return g_err; }

int phgrms_version(void) { return 10000; }

size_t phgrms_workspace_bytes(phgrms_params p) {
  if (validate_params(p) == PHGRMS_EINVAL) return 0;
  return ws_layout(p).total;
}

int phgrms_denoise_async(const uint8_t* d_in, uint8_t* d_out, phgrms_params p, void* d_ws,
                         size_t ws_bytes, int64_t* d_changed, int32_t* d_iterations,
                         void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if ((rc = check_buffers(d_in, d_out, p, d_ws, ws_bytes)) != PHGRMS_OK) return rc;
  const WsLayout l = ws_layout(p);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  auto* counts = reinterpret_cast<unsigned long long*>(ws + l.counts_off);
  auto* changed = d_changed ? reinterpret_cast<unsigned long long*>(d_changed)
                            : reinterpret_cast<unsigned long long*>(ws + l.changed_off);
  int* iters = d_iterations ? reinterpret_cast<int*>(d_iterations)
                            : reinterpret_cast<int*>(ws + l.state_off);
  return enqueue_denoise(d_in, d_out, p, fused_shape(p.beta, (long long)p.rows * p.cols),
                         ws + l.img_off, counts, changed, iters, ws + l.map_off,
                         static_cast<hipStream_t>(stream));
}

int phgrms_denoise_ex(const uint8_t* d_in, uint8_t* d_out, phgrms_params p, int32_t flags,
                      void* d_ws, size_t ws_bytes, int64_t* d_changed, int32_t* d_iterations,
                      void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if ((flags & ~int32_t(PHGRMS_STOP_ON_CYCLE)) != 0)
    return fail(PHGRMS_EINVAL, "unknown flags 0x%x", unsigned(flags));
  if ((rc = check_buffers(d_in, d_out, p, d_ws, ws_bytes)) != PHGRMS_OK) return rc;
  const WsLayout l = ws_layout(p);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  auto* counts = reinterpret_cast<unsigned long long*>(ws + l.counts_off);
  auto* changed = d_changed ? reinterpret_cast<unsigned long long*>(d_changed)
                            : reinterpret_cast<unsigned long long*>(ws + l.changed_off);
  int* iters = d_iterations ? reinterpret_cast<int*>(d_iterations)
                            : reinterpret_cast<int*>(ws + l.state_off);
  int shape = fused_shape(p.beta, (long long)p.rows * p.cols);
  unsigned long long* diff2 = nullptr;
  if (flags & PHGRMS_STOP_ON_CYCLE) {
    // the period-2 variants: the tuned skipping shape's own, else (1, 8, 4)
    // with change tracking if the tuned shape tracks changes, else without
    diff2 = reinterpret_cast<unsigned long long*>(ws + l.diff_off);
    if (kShapes[shape].track != 2) shape = kShapes[shape].track ? 7 : kDefaultShape;
  }
  return enqueue_denoise(d_in, d_out, p, shape, ws + l.img_off, counts, changed, iters,
                         ws + l.map_off, static_cast<hipStream_t>(stream), diff2);
}

int phgrms_denoise(const uint8_t* d_in, uint8_t* d_out, phgrms_params p, void* d_ws,
                   size_t ws_bytes, int64_t* h_changed, int32_t* h_iterations, void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if ((rc = check_buffers(d_in, d_out, p, d_ws, ws_bytes)) != PHGRMS_OK) return rc;
  const WsLayout l = ws_layout(p);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  auto* counts = reinterpret_cast<unsigned long long*>(ws + l.counts_off);
  auto* changed = reinterpret_cast<unsigned long long*>(ws + l.changed_off);
  int* iters = reinterpret_cast<int*>(ws + l.state_off);
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = enqueue_denoise(d_in, d_out, p, fused_shape(p.beta, (long long)p.rows * p.cols),
                       ws + l.img_off, counts, changed, iters, ws + l.map_off, s);
  if (rc != PHGRMS_OK) return rc;
  hipError_t e;
  if (h_changed && p.k > 0) {
    e = hipMemcpyAsync(h_changed, changed, sizeof(int64_t) * size_t(p.k), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "changed read-back");
  }
  int32_t it = 0;
  e = hipMemcpyAsync(&it, iters, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "iterations read-back");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");
  if (h_iterations) *h_iterations = it;
  return PHGRMS_OK;
}

int phgrms_denoise_plain(const uint8_t* d_in, uint8_t* d_out, phgrms_params p, void* d_ws,
                         size_t ws_bytes, int64_t* h_changed, int32_t* h_iterations,
                         void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if ((rc = check_buffers(d_in, d_out, p, d_ws, ws_bytes)) != PHGRMS_OK) return rc;
  const WsLayout l = ws_layout(p);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  uint8_t* ws_img = ws + l.img_off;
  auto* counts = reinterpret_cast<unsigned long long*>(ws + l.counts_off);
  auto* changed = reinterpret_cast<unsigned long long*>(ws + l.changed_off);
  int* iters = reinterpret_cast<int*>(ws + l.state_off);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long n = (long long)p.rows * p.cols;
  hipError_t e;
  if (p.k > 0) {
    const long long nc = (long long)p.k * kCountSlots;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(int(std::min<long long>((nc + 255) / 256, 1024))),
                       dim3(256), 0, s, counts, nc);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "init launch");
  }
  // One pass per launch; the layout assumes all k passes run, so that a run
  // without early stop ends in d_out.
  const int pshape = plain_shape(p.beta, (long long)p.rows * p.cols);
  const TileGeom g = tile_geom(p, pshape);
  const int L = p.k;
  auto dst_of = [&](int j) -> uint8_t* { return ((L - 1 - j) % 2 == 0) ? d_out : ws_img; };
  const uint8_t* src = d_in;
  if (n > 0 && L > 0 && d_in == d_out && dst_of(0) == d_out) {
    const int blocks = int(std::min<long long>((n / 4 + 255) / 256 + 1, 4096));
    hipLaunchKernelGGL(copy_bytes_kernel, dim3(blocks), dim3(256), 0, s, d_in, ws_img, n);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "stage launch");
    src = ws_img;
  }
  for (int j = 0; j < L && n > 0; ++j) {
    PassArgs a;
    a.src = src;
    a.dst = dst_of(j);
    a.changed = counts;
    a.rows = p.rows;
    a.cols = p.cols;
    a.alpha = p.alpha;
    a.pass0 = j;
    a.npasses = 1;
    a.tiles_x = g.tiles_x;
    a.ntiles = int(g.ntiles);
    a.map_in = nullptr;      // the plain path tests every row of every pass
    a.map_out = nullptr;
    a.prev2 = nullptr;
    a.diff2 = nullptr;
    a.seq = j;
    a.list_state = nullptr;
    a.list_cap = 0;
    if ((e = launch_pass(p.beta, pshape, a, s)) != hipSuccess) return hip_fail(e, "pass launch");
    src = a.dst;
    unsigned long long slots[kCountSlots];
    e = hipMemcpyAsync(slots, counts + size_t(j) * kCountSlots, sizeof(slots),
                       hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "changed read-back");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");
    unsigned long long ch = 0;
    for (int k = 0; k < kCountShards; ++k) ch += slots[k * kCountStride];
    if (ch == 0) break;
  }
  FinishArgs f;
  f.counts = counts;
  f.diff2 = nullptr;
  f.changed = changed;
  f.k = p.k;
  f.T = 1;
  f.launches = L;
  f.buf_even_from_end = d_out;
  f.buf_odd_from_end = ws_img;
  f.first_src = d_in;
  f.out = d_out;
  f.n = n;
  f.iterations = iters;
  // Every block re-derives the iteration count from the count slots; a
  // moved image (rare) is copied grid-stride.
  const int fblocks = int(std::min<long long>((n / 16 + 255) / 256 + 1, 1024));
  hipLaunchKernelGGL(finish_kernel, dim3(fblocks), dim3(256), 0, s, f);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "finish launch");
  if (h_changed && p.k > 0) {
    e = hipMemcpyAsync(h_changed, changed, sizeof(int64_t) * size_t(p.k), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "changed read-back");
  }
  int32_t it = 0;
  e = hipMemcpyAsync(&it, iters, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "iterations read-back");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream sync");
  if (h_iterations) *h_iterations = it;
  return PHGRMS_OK;
}

size_t phgrms_change_map_bytes(phgrms_params p) {
  if (validate_params(p) == PHGRMS_EINVAL) return 0;
  return change_map_bytes(p.rows, p.cols);
}

int phgrms_run_passes(const uint8_t* d_src, uint8_t* d_dst, phgrms_params p, int32_t shape,
                      int32_t pass_index, int64_t* d_changed, uint8_t* d_maps, void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if (shape < 0 || shape >= kNumShapes) return fail(PHGRMS_EINVAL, "bad shape %d", shape);
  if (p.k < 1 || p.k > kShapes[shape].T)
    return fail(PHGRMS_EINVAL, "k %d not in [1,%d] for shape %d", p.k, kShapes[shape].T, shape);
  const long long n = (long long)p.rows * p.cols;
  if (n == 0) return PHGRMS_OK;
  if (!d_src || !d_dst || !d_changed) return fail(PHGRMS_EINVAL, "null pointer");
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_src), b = reinterpret_cast<uintptr_t>(d_dst);
  if (a < b + uintptr_t(n) && b < a + uintptr_t(n))
    return fail(PHGRMS_EINVAL, "source and destination overlap");
  if (d_maps != nullptr && (!kShapes[shape].track || p.k != 1))
    return fail(PHGRMS_EINVAL, "change maps need a change-tracking shape and k = 1");
  if (pass_index < 0) return fail(PHGRMS_EINVAL, "negative pass index");
  const size_t half = map_half_bytes(p.rows, p.cols);
  const size_t mbytes = change_map_bytes(p.rows, p.cols);
  const uintptr_t m = reinterpret_cast<uintptr_t>(d_maps);
  if (d_maps != nullptr && ((m < a + uintptr_t(n) && a < m + mbytes) ||
                            (m < b + uintptr_t(n) && b < m + mbytes)))
    return fail(PHGRMS_EINVAL, "change maps overlap an image");
  const TileGeom g = tile_geom(p, shape);
  PassArgs pa;
  pa.src = d_src;
  pa.dst = d_dst;
  pa.changed = reinterpret_cast<unsigned long long*>(d_changed);  // kCountSlots per pass
  pa.rows = p.rows;
  pa.cols = p.cols;
  pa.alpha = p.alpha;
  pa.pass0 = 0;
  pa.npasses = p.k;
  pa.tiles_x = g.tiles_x;
  pa.ntiles = int(g.ntiles);
  pa.map_in = (d_maps != nullptr && pass_index > 0)
                  ? d_maps + size_t((pass_index - 1) & 1) * half : nullptr;
  pa.map_out = d_maps != nullptr ? d_maps + size_t(pass_index & 1) * half : nullptr;
  pa.prev2 = nullptr;
  pa.diff2 = nullptr;
  // skipping shapes: from pass 2 on the destination holds the image before
  // the source (the caller ping-pongs two buffers); the tile lists' counts
  // and marks are cleared before the first launch of a sequence
  pa.seq = pass_index;
  pa.list_state = (d_maps != nullptr && kShapes[shape].track == 2)
                      ? reinterpret_cast<uint32_t*>(d_maps + list_state_offset(p.rows, p.cols))
                      : nullptr;
  pa.list_cap = list_capacity(p.rows, p.cols);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (pa.list_state != nullptr && pass_index == 0) {
    const long long nl = list_clear_u64(p.rows, p.cols);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(int(std::min<long long>((nl + 255) / 256, 1024))),
                       dim3(256), 0, s, reinterpret_cast<unsigned long long*>(pa.list_state), nl);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "list clear launch");
  }
  e = launch_pass(p.beta, shape, pa, s);
  if (e != hipSuccess) return hip_fail(e, "pass launch");
  return PHGRMS_OK;
}

int phgrms_selftest(int64_t* d_failures, void* stream) {
  if (d_failures == nullptr) return fail(PHGRMS_EINVAL, "null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* f = reinterpret_cast<unsigned long long*>(d_failures);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, f, 2ll);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "selftest launch");
  hipLaunchKernelGGL(selftest_kernel, dim3(4096), dim3(256), 0, s, f);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "selftest launch");
  return PHGRMS_OK;
}

int phgrms_num_shapes(void) { return kNumShapes; }

int phgrms_shape_tracks_changes(int32_t shape) {
  if (shape < 0 || shape >= kNumShapes) return fail(PHGRMS_EINVAL, "bad shape %d", shape);
  return kShapes[shape].track != 0 ? 1 : 0;
}

int phgrms_shape_skips_unchanged(int32_t shape) {
  if (shape < 0 || shape >= kNumShapes) return fail(PHGRMS_EINVAL, "bad shape %d", shape);
  return kShapes[shape].track == 2 ? 1 : 0;
}

int phgrms_shape_info(int32_t shape, int32_t* passes_per_launch, int32_t* rows_per_wave,
                      int32_t* waves) {
  if (shape < 0 || shape >= kNumShapes) return fail(PHGRMS_EINVAL, "bad shape %d", shape);
  if (passes_per_launch) *passes_per_launch = kShapes[shape].T;
  if (rows_per_wave) *rows_per_wave = kShapes[shape].rows;
  if (waves) *waves = kShapes[shape].waves;
  return PHGRMS_OK;
}

int phgrms_set_tuning(int32_t beta, int32_t shape) { return set_fused_shape(beta, -1, shape); }

int phgrms_set_tuning_class(int32_t beta, int32_t size_class, int32_t shape) {
  if (size_class < 0) return fail(PHGRMS_EINVAL, "bad size class %d", size_class);
  return set_fused_shape(beta, size_class, shape);
}

int phgrms_set_batch_tuning_class(int32_t beta, int32_t size_class, int32_t shape) {
  return set_batch_shape(beta, size_class, shape);
}

int phgrms_get_batch_tuning_class(int32_t beta, int32_t size_class) {
  if (beta < 1 || beta > PHGRMS_BETA_MAX || size_class < 0 || size_class >= kSizeClasses)
    return fail(PHGRMS_EINVAL, "bad beta %d or size class %d", beta, size_class);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_batch_shape[beta][size_class];
}

int phgrms_get_tuning_class(int32_t beta, int32_t size_class) {
  if (beta < 1 || beta > PHGRMS_BETA_MAX || size_class < 0 || size_class >= kSizeClasses)
    return fail(PHGRMS_EINVAL, "bad beta %d or size class %d", beta, size_class);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_fused_shape[beta][size_class];
}

int phgrms_set_grid_mode(int32_t mode) { return set_grid_mode(mode); }

int phgrms_get_grid_mode(void) { return grid_mode(); }

size_t phgrms_autotune_workspace_bytes(phgrms_params p) {
  if (validate_params(p) != PHGRMS_OK) return 0;
  const size_t n = size_t(std::max<int64_t>((int64_t)p.rows * p.cols, 1));
  return ((n + 255) & ~size_t(255)) + ws_layout(p).total;
}

int phgrms_autotune(phgrms_params p, const uint8_t* d_img, void* d_ws, size_t ws_bytes,
                    int32_t reps, int32_t* best_shape, float* shape_us, const char* cache_path,
                    void* stream) {
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  const long long n = (long long)p.rows * p.cols;
  if (n == 0 || p.k == 0) return fail(PHGRMS_EINVAL, "nothing to time (empty image or k = 0)");
  if (reps < 1 || reps > 1000) return fail(PHGRMS_EINVAL, "reps %d outside 1..1000", reps);
  if (d_img == nullptr || d_ws == nullptr || best_shape == nullptr)
    return fail(PHGRMS_EINVAL, "null pointer");
  const size_t need = phgrms_autotune_workspace_bytes(p);
  if (ws_bytes < need) return fail(PHGRMS_ENOSPC, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (overlaps(d_ws, need, d_img, size_t(n))) return fail(PHGRMS_EINVAL, "workspace overlaps the image");
  uint8_t* out = static_cast<uint8_t*>(d_ws);
  uint8_t* ws = out + ((size_t(n) + 255) & ~size_t(255));
  const WsLayout l = ws_layout(p);
  auto* counts = reinterpret_cast<unsigned long long*>(ws + l.counts_off);
  auto* changed = reinterpret_cast<unsigned long long*>(ws + l.changed_off);
  int* iters = reinterpret_cast<int*>(ws + l.state_off);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best = -1;
  float best_us = 0.f;
  for (int sh = 0; sh < kNumShapes && e == hipSuccess && rc == PHGRMS_OK; ++sh) {
    // one untimed run, then `reps` runs between two events
    for (int r = 0; r <= reps && rc == PHGRMS_OK && e == hipSuccess; ++r) {
      if (r == 1) e = hipEventRecord(e0, s);
      if (e == hipSuccess)
        rc = enqueue_denoise(d_img, out, p, sh, ws + l.img_off, counts, changed, iters,
                             ws + l.map_off, s);
    }
    if (rc != PHGRMS_OK || e != hipSuccess) break;
    float ms = 0.f;
    if ((e = hipEventRecord(e1, s)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess)
      e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    const float us = ms * 1000.f / float(reps);
    if (shape_us != nullptr) shape_us[sh] = us;
    if (best < 0 || us < best_us) {
      best = sh;
      best_us = us;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != PHGRMS_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  *best_shape = best;
  rc = set_fused_shape(p.beta, size_class(n), best);
  if (rc != PHGRMS_OK || cache_path == nullptr) return rc;
  // the cache file's own entries, with this choice over them
  TuneTables t = current_tuning();
  rc = read_tuning_file(cache_path, t);
  if (rc != PHGRMS_OK && rc != PHGRMS_ENOTFOUND) return rc;
  t.fused[p.beta][size_class(n)] = best;
  return write_tuning_file(cache_path, t);
}

int phgrms_load_tuning(const char* path) {
  TuneTables t = current_tuning();
  const int rc = read_tuning_file(path, t);
  if (rc != PHGRMS_OK) return rc;
  apply_tuning(t);
  return PHGRMS_OK;
}

int phgrms_save_tuning(const char* path) { return write_tuning_file(path, current_tuning()); }

int phgrms_get_tuning(int32_t beta) {
  if (beta < 1 || beta > PHGRMS_BETA_MAX) return fail(PHGRMS_EINVAL, "bad beta %d", beta);
  return fused_shape(beta, 1ll << 22);
}

int phgrms_cardinality(const uint8_t* d_img, int32_t rows, int32_t cols, int32_t alpha,
                       int32_t beta, uint16_t* d_card, void* stream) {
  phgrms_params p{rows, cols, alpha, beta, 0};
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  const long long n = (long long)rows * cols;
  if (n == 0) return PHGRMS_OK;
  if (d_img == nullptr || d_card == nullptr) return fail(PHGRMS_EINVAL, "null pointer");
  const int blocks = int(std::min<long long>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(cardinality_kernel, dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), d_img, rows, cols, alpha, beta, d_card);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "cardinality launch");
  return PHGRMS_OK;
}

}  // extern "C"
