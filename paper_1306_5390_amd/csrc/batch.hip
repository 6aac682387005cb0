// batch.hip -- many images per launch (C ABI phgrms_batch_*).
//
// Each image of a batch runs the pass loop of Section 2 with its own size,
// alpha, beta and k.  Instead of one launch sequence per image, the images
// are spread over three streams (balanced by work) and, per stream, launch j
// of every image with the same beta and kernel shape goes into one
// multi_pass_kernel launch over a static table of all their tiles.  The plan
// precomputes, per group, the tile table and the image descriptors of every
// launch index; a run uploads them once per set of pointers and replays the
// whole sequence (forked to the streams and joined) as a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "phgrms.h"
#include "phgrms_internal.hpp"
#include "pass_kernel.hpp"

using namespace phg;

namespace {

template <int B, int T, int R, int W, int TRACK = 0>
const void* multi_ptr() {
  return reinterpret_cast<const void*>(&multi_pass_kernel<B, T, R, W, TRACK>);
}

// With maps, the change-tracking shapes (7, 8, 11, 12) keep change maps
// per image; otherwise every shape runs dense.  The skipping shapes' list
// kernels are multi_skip_ptr's.
template <int B>
const void* multi_beta(int shape, bool maps) {
  switch (shape) {
    case 0: return multi_ptr<B, 1, 8, 1>();
    case 1: return multi_ptr<B, 1, 16, 1>();
    case 2: return multi_ptr<B, 1, 8, 2>();
    case 3: return multi_ptr<B, 1, 8, 4>();
    case 4: return multi_ptr<B, 1, 16, 4>();
    case 5: return multi_ptr<B, 2, 16, 4>();
    case 6: return multi_ptr<B, 4, 16, 4>();
    case 7:
    case 11: return maps ? multi_ptr<B, 1, 8, 4, 1>() : multi_ptr<B, 1, 8, 4>();
    case 8:
    case 12: return maps ? multi_ptr<B, 1, 8, 2, 1>() : multi_ptr<B, 1, 8, 2>();
    case 9: return multi_ptr<B, 1, 4, 8>();
    case 10: return multi_ptr<B, 1, 4, 4>();
    default: return nullptr;
  }
}

// The skipping shapes 11 and 12 over many images: launch `seq` of the
// sequence (as for one image: the dense kernel of the same tile geometry
// for the first kDenseFirstLaunches launches, lists from launch 2, listed
// tiles only from launch 3), with one set of tile lists for the launch.
template <int B>
const void* multi_skip_beta(int shape, int seq) {
  static_assert(kDenseFirstLaunches == 2, "launch 2 builds the first lists");
  if (shape == 11)
    return seq < 2 ? multi_ptr<B, 1, 8, 4>() : seq == 2 ? multi_ptr<B, 1, 8, 4, 2>()
                                                       : multi_ptr<B, 1, 8, 4, 3>();
  if (shape == 12)
    return seq < 2 ? multi_ptr<B, 1, 8, 2>() : seq == 2 ? multi_ptr<B, 1, 8, 2, 2>()
                                                       : multi_ptr<B, 1, 8, 2, 3>();
  return nullptr;
}

const void* multi_skip_ptr(int beta, int shape, int seq) {
  switch (beta) {
    case 1: return multi_skip_beta<1>(shape, seq);
    case 2: return multi_skip_beta<2>(shape, seq);
    case 3: return multi_skip_beta<3>(shape, seq);
    case 4: return multi_skip_beta<4>(shape, seq);
    default: return nullptr;
  }
}

// Workgroups of a listed launch: kListedOversubscription times as many as
// fit on the device at once (a multiple of kListShards), the occupancy
// queried once per (beta, shape).
int listed_grid(int beta, int shape) {
  static std::mutex mu;
  static int occ[PHGRMS_BETA_MAX + 1][16] = {};
  static int cus = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    cus = n;
  }
  if (occ[beta][shape] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, multi_skip_ptr(beta, shape, 3),
                                                     kShapes[shape].waves * 64, 0) != hipSuccess)
      return -1;
    occ[beta][shape] = nb > 0 ? nb : 1;
  }
  const long long g =
      (long long)occ[beta][shape] * cus * kListedOversubscription / kListShards * kListShards;
  return int(std::max<long long>(g, kListShards));
}

}  // namespace

const void* phg::multi_kernel_ptr(int beta, int shape, bool maps) {
  switch (beta) {
    case 1: return multi_beta<1>(shape, maps);
    case 2: return multi_beta<2>(shape, maps);
    case 3: return multi_beta<3>(shape, maps);
    case 4: return multi_beta<4>(shape, maps);
    default: return nullptr;
  }
}

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Streams the groups of a batch are spread over: the groups hold different
// images, so their launches are independent, and kernels of different
// groups running side by side overlap one group's tile loads and stores
// with another's arithmetic.
constexpr int kSideStreams = 3;

struct Group {
  int beta = 0;
  int shape = 0;
  int T = 1;
  bool maps = false;                // change maps per image (tracking shapes)
  bool lists = false;               // tile lists (skipping shapes): lists_off, capacity tiles.size()
  size_t lists_off = 0;
  int launches = 0;                 // max over its images of ceil(k/T)
  std::vector<int> images;          // item indices
  std::vector<TileRef> tiles;       // tile table (image = index into `images`)
  size_t tiles_off = 0;             // workspace offsets
  size_t descs_off = 0;             // launches x images.size() ImageDesc
};

}  // namespace

struct phgrms_plan {
  std::vector<phgrms_item> items;
  std::vector<size_t> counts_off;   // per item, in the workspace
  std::vector<size_t> img_off;      // per item, ping-pong image in the workspace
  std::vector<size_t> map_off;      // per item, its two change maps (tracking groups), or 0
  std::vector<size_t> map_half;     // per item, bytes of one change map
  std::vector<int> tile_base;       // per item, index of its first tile in its group's table
  std::vector<int64_t> k_off;       // per item, offset in d_changed
  std::vector<int> launches;        // per item, ceil(k/T)
  std::vector<int> T;               // per item
  std::vector<Group> groups;
  size_t stage_off = 0;             // CopyDesc[n]
  size_t finish_off = 0;            // BatchFinishDesc[n]
  size_t ws_bytes = 0;
  int total_launches = 0;
  std::mutex mu;
  // uploaded descriptors / captured graph, keyed by the run's pointers
  std::tuple<const void*, void*, void*, void*, void*> key{nullptr, nullptr, nullptr, nullptr, nullptr};
  bool uploaded = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // groups run on side streams forked from the caller's stream (created at
  // the first run, on the device current then)
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  std::vector<int> group_stream;    // per group: its side stream
};

namespace {

struct Host {
  std::vector<uint8_t> bytes;
  template <class X>
  void put(size_t off, const X* p, size_t count) {
    std::memcpy(bytes.data() + off, p, sizeof(X) * count);
  }
};

// Enqueue the kernels of one run (no uploads, no synchronisation).
int enqueue_run(phgrms_plan* pl, uint8_t* ws, hipStream_t s) {
  hipError_t e;
  const int n = int(pl->items.size());
  // 1. zero all count slots
  {
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += size_t(std::max(pl->items[i].p.k, 1)) * kCountSlots;
    auto* c = reinterpret_cast<unsigned long long*>(ws + pl->counts_off[0]);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(int(std::min<size_t>((total + 255) / 256, 4096))),
                       dim3(256), 0, s, c, (long long)total);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "batch zero launch");
    // and the counts and marks of the groups' tile lists
    for (auto& g : pl->groups) {
      if (!g.lists || g.tiles.empty()) continue;
      const long long nl = (long long)((size_t(TileLists::kHead) + g.tiles.size() + 1) / 2);
      hipLaunchKernelGGL(zero_u64_kernel, dim3(int(std::min<long long>((nl + 255) / 256, 1024))),
                         dim3(256), 0, s, reinterpret_cast<unsigned long long*>(ws + g.lists_off), nl);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "batch list clear launch");
    }
  }
  // 2. stage in-place inputs whose first launch writes the output buffer
  hipLaunchKernelGGL(multi_copy_kernel, dim3(32, std::min(n, 65535)), dim3(256), 0, s,
                     reinterpret_cast<const CopyDesc*>(ws + pl->stage_off), n);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "batch stage launch");
  // 3. launch j of every group; with several groups, each group on its side
  //    stream (forked from s after the staging, joined before the finish)
  int maxL = 0;
  unsigned used = 0;   // bit k: side stream k has a group with tiles
  for (auto& g : pl->groups) maxL = std::max(maxL, g.launches);
  for (size_t gi = 0; gi < pl->groups.size(); ++gi)
    if (!pl->groups[gi].tiles.empty()) used |= 1u << pl->group_stream[gi];
  const bool fork = (used & (used - 1)) != 0 && pl->fork != nullptr;
  if (fork) {
    if ((e = hipEventRecord(pl->fork, s)) != hipSuccess) return hip_fail(e, "batch fork");
    for (int k = 0; k < kSideStreams; ++k)
      if ((e = hipStreamWaitEvent(pl->side[k], pl->fork, 0)) != hipSuccess)
        return hip_fail(e, "batch fork wait");
  }
  for (int j = 0; j < maxL; ++j) {
    for (size_t gi = 0; gi < pl->groups.size(); ++gi) {
      auto& g = pl->groups[gi];
      if (j >= g.launches || g.tiles.empty()) continue;
      const hipStream_t gs = fork ? pl->side[pl->group_stream[gi]] : s;
      MultiArgs a;
      a.images = reinterpret_cast<const ImageDesc*>(ws + g.descs_off) + size_t(j) * g.images.size();
      a.tiles = reinterpret_cast<const TileRef*>(ws + g.tiles_off);
      a.ntiles = int(g.tiles.size());
      a.seq = j;
      a.list_state = g.lists ? reinterpret_cast<uint32_t*>(ws + g.lists_off) : nullptr;
      a.list_cap = a.ntiles;
      int grid = int(std::min<long long>((a.ntiles + 7) / 8 * 8,
                                         max_workgroups(kShapes[g.shape].waves * 64)));
      if (g.lists && j >= 3 && (grid = listed_grid(g.beta, g.shape)) <= 0)
        return fail(PHGRMS_EDEVICE, "occupancy query of the listed batch kernel failed");
      // (change-tracking groups: the dense kernel for the first launches)
      const void* k = g.lists ? multi_skip_ptr(g.beta, g.shape, j)
                              : multi_kernel_ptr(g.beta, g.shape, g.maps && j >= kDenseFirstLaunches);
      void* args[] = {&a};
      e = hipLaunchKernel(k, dim3(grid), dim3(kShapes[g.shape].waves * 64), args, 0, gs);
      if (e != hipSuccess) return hip_fail(e, "batch pass launch");
    }
  }
  if (fork) {
    for (int k = 0; k < kSideStreams; ++k) {
      if ((e = hipEventRecord(pl->join[k], pl->side[k])) != hipSuccess) return hip_fail(e, "batch join");
      if ((e = hipStreamWaitEvent(s, pl->join[k], 0)) != hipSuccess) return hip_fail(e, "batch join wait");
    }
  }
  // 4. totals, iteration counts, final images
  hipLaunchKernelGGL(batch_finish_kernel, dim3(32, std::min(n, 65535)), dim3(256), 0, s,
                     reinterpret_cast<const BatchFinishDesc*>(ws + pl->finish_off), n);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "batch finish launch");
  return PHGRMS_OK;
}

// Destroy a plan's side streams and events (after synchronising them).
void release_streams(phgrms_plan* pl) {
  for (int k = 0; k < kSideStreams; ++k) {
    if (pl->side[k]) {
      (void)hipStreamSynchronize(pl->side[k]);
      (void)hipStreamDestroy(pl->side[k]);
      pl->side[k] = nullptr;
    }
    if (pl->join[k]) {
      (void)hipEventDestroy(pl->join[k]);
      pl->join[k] = nullptr;
    }
  }
  if (pl->fork) {
    (void)hipEventDestroy(pl->fork);
    pl->fork = nullptr;
  }
}

bool ranges_overlap(uintptr_t a, size_t na, uintptr_t b, size_t nb) {
  return na > 0 && nb > 0 && a < b + nb && b < a + na;
}

}  // namespace

extern "C" {

int phgrms_batch_plan(const phgrms_item* items, int32_t n, const char* tune_cache_path,
                      phgrms_plan** out, size_t* ws_bytes) {
  if (out == nullptr || items == nullptr || n < 1) return fail(PHGRMS_EINVAL, "bad batch arguments");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    const int rc = validate_params(items[i].p);
    if (rc != PHGRMS_OK) {
      char msg[512];
      std::snprintf(msg, sizeof(msg), "%s", phgrms_last_error());
      return fail(rc, "item %d: %s", i, msg);
    }
  }
  // The batch shapes: the process's table, or the cache file's entries over it
  // (read here, for this plan only).
  TuneTables tune = current_tuning();
  if (tune_cache_path != nullptr) {
    const int rc = read_tuning_file(tune_cache_path, tune);
    if (rc != PHGRMS_OK) return rc;
  }
  auto batch_shape = [&](int beta, long long npx) { return tune.batch[beta][size_class(npx)]; };
  phgrms_plan* pl = new phgrms_plan();
  pl->items.assign(items, items + n);
  pl->counts_off.resize(n);
  pl->img_off.resize(n);
  pl->map_off.assign(n, 0);
  pl->map_half.assign(n, 0);
  pl->tile_base.assign(n, 0);
  pl->k_off.resize(n);
  pl->launches.resize(n);
  pl->T.resize(n);
  // workspace: count slots of every item, then ping-pong images
  size_t off = 0;
  int64_t koff = 0;
  for (int i = 0; i < n; ++i) {
    pl->counts_off[i] = off;
    off += sizeof(uint64_t) * size_t(kCountSlots) * size_t(std::max(items[i].p.k, 1));
    pl->k_off[i] = koff;
    koff += items[i].p.k;
  }
  off = up256(off);
  for (int i = 0; i < n; ++i) {
    pl->img_off[i] = off;
    off = up256(off + size_t(std::max<int64_t>((int64_t)items[i].p.rows * items[i].p.cols, 1)));
  }
  // Images are spread over kSideStreams streams, largest work (tiles x
  // launches) first, each to the stream with the least work so far; a group
  // is the images of one stream that share (beta, kernel shape), one
  // multi-image launch per launch index.
  std::vector<int> order(n), stream_of(n, 0);
  std::vector<double> work(n, 0.0), load(kSideStreams, 0.0);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    const int shp = batch_shape(items[i].p.beta, (long long)items[i].p.rows * items[i].p.cols);
    const int T = kShapes[shp].T;
    if ((int64_t)items[i].p.rows * items[i].p.cols > 0)
      work[i] = double(tile_geom(items[i].p, shp).ntiles) * double((items[i].p.k + T - 1) / T);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  for (int i : order) {
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    stream_of[i] = k;
    load[k] += work[i];
  }
  std::map<std::tuple<int, int, int>, int> gidx;
  for (int i = 0; i < n; ++i) {
    const int b = items[i].p.beta;
    const int shp = batch_shape(b, (long long)items[i].p.rows * items[i].p.cols);
    const auto key = std::make_tuple(stream_of[i], b, shp);
    if (!gidx.count(key)) {
      gidx[key] = int(pl->groups.size());
      Group g;
      g.beta = b;
      g.shape = shp;
      g.T = kShapes[g.shape].T;
      g.maps = kShapes[g.shape].track != 0 && g.T == 1;
      g.lists = kShapes[g.shape].track == 2 && g.T == 1;
      pl->groups.push_back(g);
      pl->group_stream.push_back(stream_of[i]);
    }
    Group& g = pl->groups[gidx[key]];
    const int local = int(g.images.size());
    g.images.push_back(i);
    pl->T[i] = g.T;
    pl->launches[i] = (items[i].p.k + g.T - 1) / g.T;
    g.launches = std::max(g.launches, pl->launches[i]);
    const TileGeom tg = tile_geom(items[i].p, g.shape);
    pl->tile_base[i] = int(g.tiles.size());
    if ((int64_t)items[i].p.rows * items[i].p.cols > 0)
      for (long long t = 0; t < tg.ntiles; ++t) g.tiles.push_back(TileRef{local, int(t)});
    if (g.maps && (int64_t)items[i].p.rows * items[i].p.cols > 0) {
      // one byte per (row, tile column), two maps alternating by launch
      // (never cleared: each byte carries its launch's stamp)
      pl->map_half[i] = size_t(items[i].p.rows) * size_t(tg.tiles_x);
      pl->map_off[i] = off;
      off = up256(off + 2 * pl->map_half[i]);
    }
  }
  for (auto& g : pl->groups) {
    if (g.tiles.size() > size_t(1) << 30) {
      delete pl;
      return fail(PHGRMS_EINVAL, "batch too large (%zu tiles)", g.tiles.size());
    }
    if (g.lists) {
      // tile lists over the group's tile table (cleared at every run)
      g.lists_off = off;
      off = up256(off + 4 * TileLists::words(int(g.tiles.size())));
    }
    g.tiles_off = off;
    off = up256(off + sizeof(TileRef) * g.tiles.size());
    g.descs_off = off;
    off = up256(off + sizeof(ImageDesc) * size_t(std::max(g.launches, 1)) * g.images.size());
    pl->total_launches += g.launches + ((g.lists && !g.tiles.empty()) ? 1 : 0);
  }
  pl->stage_off = off;
  off = up256(off + sizeof(CopyDesc) * size_t(n));
  pl->finish_off = off;
  off = up256(off + sizeof(BatchFinishDesc) * size_t(n));
  pl->ws_bytes = off;
  pl->total_launches += 3;
  *out = pl;
  if (ws_bytes) *ws_bytes = pl->ws_bytes;
  return PHGRMS_OK;
}

int phgrms_batch_launches(const phgrms_plan* plan) {
  if (plan == nullptr) return fail(PHGRMS_EINVAL, "null plan");
  return plan->total_launches;
}

int phgrms_batch_run(phgrms_plan* pl, const uint8_t* d_in, size_t in_bytes, uint8_t* d_out,
                     size_t out_bytes, void* d_ws, size_t ws_bytes, int64_t* d_changed,
                     int32_t* d_iterations, void* stream) {
  if (pl == nullptr) return fail(PHGRMS_EINVAL, "null plan");
  if (d_ws == nullptr || ws_bytes < pl->ws_bytes)
    return fail(PHGRMS_ENOSPC, "batch workspace of %zu bytes, %zu needed", ws_bytes, pl->ws_bytes);
  const int n = int(pl->items.size());
  // ranges: inside the arenas; outputs disjoint; an output equals its own
  // input or overlaps no input; nothing overlaps the workspace
  std::vector<std::pair<uintptr_t, size_t>> ins(n), outs(n);
  for (int i = 0; i < n; ++i) {
    const phgrms_item& it = pl->items[i];
    const size_t nb = size_t((int64_t)it.p.rows * it.p.cols);
    if (nb > 0 && (it.in_off + nb > in_bytes || it.out_off + nb > out_bytes || !d_in || !d_out))
      return fail(PHGRMS_EINVAL, "item %d does not fit its arena", i);
    ins[i] = {reinterpret_cast<uintptr_t>(d_in) + it.in_off, nb};
    outs[i] = {reinterpret_cast<uintptr_t>(d_out) + it.out_off, nb};
    if (ranges_overlap(reinterpret_cast<uintptr_t>(d_ws), pl->ws_bytes, ins[i].first, nb) ||
        ranges_overlap(reinterpret_cast<uintptr_t>(d_ws), pl->ws_bytes, outs[i].first, nb))
      return fail(PHGRMS_EINVAL, "item %d overlaps the workspace", i);
  }
  {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return outs[a].first < outs[b].first; });
    for (int i = 1; i < n; ++i) {
      const auto& a = outs[order[i - 1]];
      const auto& b = outs[order[i]];
      if (ranges_overlap(a.first, a.second, b.first, b.second))
        return fail(PHGRMS_EINVAL, "output ranges of items %d and %d overlap", order[i - 1], order[i]);
    }
    // outputs vs inputs of other items: sweep over sorted inputs
    std::vector<int> iord(n);
    for (int i = 0; i < n; ++i) iord[i] = i;
    std::sort(iord.begin(), iord.end(), [&](int a, int b) { return ins[a].first < ins[b].first; });
    for (int i = 0; i < n; ++i) {
      const auto& o = outs[i];
      if (o.second == 0) continue;
      // first input starting at or after o.first - max input size could overlap; linear
      // scan bounded by sorted order
      auto it = std::lower_bound(iord.begin(), iord.end(), o.first + o.second,
                                 [&](int a, uintptr_t v) { return ins[a].first < v; });
      for (auto jt = iord.begin(); jt != it; ++jt) {
        const int j = *jt;
        if (!ranges_overlap(o.first, o.second, ins[j].first, ins[j].second)) continue;
        if (j == i && ins[j].first == o.first) continue;   // in place
        return fail(PHGRMS_EINVAL, "output of item %d overlaps the input of item %d", i, j);
      }
    }
  }
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(pl->mu);
  const auto key = std::make_tuple(static_cast<const void*>(d_in), static_cast<void*>(d_out), d_ws,
                                   static_cast<void*>(d_changed), static_cast<void*>(d_iterations));
  hipError_t e;
  if (!pl->uploaded || key != pl->key) {
    // descriptors for these pointers
    Host h;
    h.bytes.assign(pl->ws_bytes, 0);
    std::vector<CopyDesc> stage(n);
    std::vector<BatchFinishDesc> fin(n);
    for (auto& g : pl->groups) {
      h.put(g.tiles_off, g.tiles.data(), g.tiles.size());
      std::vector<ImageDesc> d(size_t(std::max(g.launches, 1)) * g.images.size());
      for (size_t li = 0; li < g.images.size(); ++li) {
        const int i = g.images[li];
        const phgrms_item& it = pl->items[i];
        const phgrms_params& p = it.p;
        const int L = pl->launches[i];
        const uint8_t* in = d_in + it.in_off;
        uint8_t* outp = d_out + it.out_off;
        uint8_t* wimg = ws + pl->img_off[i];
        auto dst_of = [&](int j) -> uint8_t* { return ((L - 1 - j) % 2 == 0) ? outp : wimg; };
        const long long nb = (long long)p.rows * p.cols;
        const uint8_t* src0 = in;
        stage[i] = CopyDesc{in, wimg, 0};
        if (nb > 0 && L > 0 && in == outp && dst_of(0) == outp) {
          stage[i].n = nb;
          src0 = wimg;
        }
        const TileGeom tg = tile_geom(p, g.shape);
        for (int j = 0; j < g.launches; ++j) {
          ImageDesc x;
          std::memset(&x, 0, sizeof(x));
          x.src = (j == 0) ? src0 : dst_of(j - 1);
          x.dst = dst_of(j);
          x.counts = reinterpret_cast<unsigned long long*>(ws + pl->counts_off[i]);
          x.rows = p.rows;
          x.cols = p.cols;
          x.alpha = p.alpha;
          x.pass0 = j * g.T;
          x.npasses = (j < L) ? std::min(g.T, p.k - j * g.T) : 0;
          x.prev_passes = (j >= 1 && j - 1 < L) ? std::min(g.T, p.k - (j - 1) * g.T) : 0;
          x.tiles_x = tg.tiles_x;
          if (g.maps && pl->map_half[i] > 0) {
            uint8_t* maps = ws + pl->map_off[i];
            // the first kDenseFirstLaunches launches run the dense kernel
            // and keep no maps
            x.map_in = (j > kDenseFirstLaunches) ? maps + size_t((j - 1) & 1) * pl->map_half[i]
                                                 : nullptr;
            x.map_out = (j >= kDenseFirstLaunches) ? maps + size_t(j & 1) * pl->map_half[i] : nullptr;
            x.seq = j;
            x.tile_base = pl->tile_base[i];
          }
          d[size_t(j) * g.images.size() + li] = x;
        }
        BatchFinishDesc f;
        std::memset(&f, 0, sizeof(f));
        f.counts = reinterpret_cast<const unsigned long long*>(ws + pl->counts_off[i]);
        f.changed = d_changed ? reinterpret_cast<unsigned long long*>(d_changed + pl->k_off[i]) : nullptr;
        f.iterations = d_iterations ? reinterpret_cast<int*>(d_iterations + i) : nullptr;
        f.first_src = in;
        f.buf_even_from_end = outp;
        f.buf_odd_from_end = wimg;
        f.out = outp;
        f.n = nb;
        f.k = p.k;
        f.T = g.T;
        f.launches = L;
        fin[i] = f;
      }
      h.put(g.descs_off, d.data(), d.size());
    }
    h.put(pl->stage_off, stage.data(), stage.size());
    h.put(pl->finish_off, fin.data(), fin.size());
    // upload only the descriptor region (everything after the images)
    size_t lo = pl->groups.empty() ? pl->stage_off : pl->groups.front().tiles_off;
    for (auto& g : pl->groups) lo = std::min(lo, g.tiles_off);
    e = hipMemcpyAsync(ws + lo, h.bytes.data() + lo, pl->ws_bytes - lo, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "batch upload sync");
    if (pl->exec) {
      (void)hipGraphExecDestroy(pl->exec);
      pl->exec = nullptr;
    }
    if (pl->graph) {
      (void)hipGraphDestroy(pl->graph);
      pl->graph = nullptr;
    }
    pl->key = key;
    pl->uploaded = true;
  }
  if (pl->fork == nullptr && pl->groups.size() > 1) {
    // side streams (default priority) and their events, once per plan
    e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&pl->side[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      release_streams(pl);
      return hip_fail(e, "batch streams");
    }
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if ((e = hipStreamIsCapturing(s, &cap)) != hipSuccess) return hip_fail(e, "capture query");
  if (cap != hipStreamCaptureStatusNone || s == nullptr) {
    // the caller is capturing (or uses the null stream): enqueue plainly
    return enqueue_run(pl, ws, s);
  }
  if (pl->exec == nullptr) {
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "begin capture");
    const int rc = enqueue_run(pl, ws, s);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (rc != PHGRMS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "end capture");
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "graph instantiate");
    }
    pl->graph = g;
    pl->exec = x;
  }
  if ((e = hipGraphLaunch(pl->exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
  return PHGRMS_OK;
}

void phgrms_plan_destroy(phgrms_plan* plan) {
  if (plan == nullptr) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  release_streams(plan);
  delete plan;
}

}  // extern "C"
