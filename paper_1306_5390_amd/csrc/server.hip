// server.hip -- continuous-batching request server (C ABI phgrms_server_*).
//
// A worker thread owns a HIP stream and loops:
//   1. admit queued requests in arrival order while the admission cap, the
//      active-request limit, the per-step tile table and a first-fit block
//      of the caller's arena allow;
//   2. build one step: for every active request its next launch (up to T
//      passes of the pass loop of Section 2), grouped by (beta, kernel
//      shape), as multi-image descriptor and tile tables in pinned host
//      memory; upload them, launch one multi_pass_kernel per group, finish
//      the requests whose last launch this was (totals, iteration count,
//      final image into the request's output), copy their results to the
//      host, record an event;
//   3. keep at most two steps in flight (descriptor slots are double
//      buffered); a completed step's finishing requests become done.
// Requests submitted with host buffers are copied in (host to device) in
// their first step, before its launches, and their result is copied out
// after the step's finish kernel, on the same stream.
// Requests join and leave at step boundaries; a request's arithmetic is the
// single-image pass loop, so its result does not depend on its neighbours.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "phgrms.h"
#include "phgrms_internal.hpp"
#include "pass_kernel.hpp"

using namespace phg;

namespace {

constexpr int kSlots = 2;
// Adaptive mode (passes_per_step < 0): a request admitted while at least
// this many others are active takes the batch path's shape (several passes
// per launch, more pixel-passes per second); otherwise one pass per step.
constexpr size_t kBusyActive = 8;
constexpr int kResStride = PHGRMS_K_MAX + 2;   // int64 per finishing request

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over byte offsets of the arena.
struct FirstFit {
  std::map<size_t, size_t> free_;   // offset -> size
  size_t in_use = 0;
  void init(size_t base, size_t size) {
    free_.clear();
    if (size) free_[base] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rem = it->second - bytes, noff = it->first + bytes;
      free_.erase(it);
      if (rem) free_[noff] = rem;
      in_use += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    in_use -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum ReqState { kPending = 0, kActive = 1, kFinishing = 2, kDone = 3, kFailed = 4 };

struct Req {
  uint64_t id = 0;
  phgrms_params p{};
  const uint8_t* in = nullptr;
  const uint8_t* h_in = nullptr;   // host request: input in host memory
  uint8_t* h_out = nullptr;        // host request: result copied here
  int state = kPending;
  int shape = 0, T = 1, L = 0, launched = 0;
  bool zeroed = false;   // count slots cleared on the device
  bool converged = false;   // a launch saw a pass with no change: no more launches
  long long tiles = 0;
  size_t off = 0, bytes = 0;
  unsigned long long* counts = nullptr;
  uint8_t* wsimg = nullptr;
  uint8_t* out = nullptr;
  double t_submit = 0, t_done = 0;
  int32_t iterations = 0;
  std::vector<int64_t> changed;
};

size_t request_bytes(const phgrms_params& p) {
  const size_t k1 = size_t(std::max(p.k, 1));
  const size_t n = size_t(std::max<int64_t>((int64_t)p.rows * p.cols, 1));
  return up256(sizeof(uint64_t) * kCountSlots * k1) + 2 * up256(n);
}

// The tuned shape if it runs `passes` passes per launch (or passes <= 0),
// else the default shape with that many passes: (1, 8, 4) for one pass
// (measured best for serving mixed sizes), the first such shape otherwise.
int shape_for(int beta, long long npx, int passes) {
  const int tuned = fused_shape(beta, npx);
  if (passes <= 0 || kShapes[tuned].T == passes) return tuned;
  if (passes == 1) return kDefaultShape;
  for (int s = 0; s < kNumShapes; ++s)
    if (kShapes[s].T == passes) return s;
  return tuned;
}

}  // namespace

struct phgrms_server {
  phgrms_server_cfg cfg{};
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  // per-slot layout (device region at the arena start, pinned host mirror)
  size_t tiles_off = 0, imgs_off = 0, fin_off = 0, stat_off = 0, res_off = 0, slot_bytes = 0;
  // tile-table entries per step: the arena holds at most arena/2 pixels of
  // admitted requests and a tile covers at least 2048 pixels, plus ragged
  // edge tiles
  size_t tiles_cap = 0;
  uint8_t* dslot[kSlots] = {nullptr, nullptr};
  uint8_t* hslot[kSlots] = {nullptr, nullptr};
  hipStream_t stream = nullptr;
  hipEvent_t ev[kSlots] = {nullptr, nullptr};
  FirstFit heap;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;
  std::deque<uint64_t> done_queue;   // completed, not yet reported by next_done
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;
  long long active_tiles = 0;
  uint64_t next_id = 1;
  struct Inflight {
    int slot;
    std::vector<uint64_t> finishing;
    std::vector<uint64_t> launched;   // in descriptor order: the step's status entries
  };
  std::deque<Inflight> inflight;
  bool slot_busy[kSlots] = {false, false};
  uint64_t n_submitted = 0, n_completed = 0, n_steps = 0;
  uint64_t generation = 0;   // bumped by submit and release
  bool stop = false;
  int error = PHGRMS_OK;
  uint64_t fault_id = 0;   // test hook: this request fails at its first launch (0: none)
  std::thread worker;
};

namespace {

// Kernel shape, passes per launch, launches and tiles of a request.
void set_shape(Req& r, int shape) {
  r.shape = shape;
  r.T = kShapes[shape].T;
  r.L = ((int64_t)r.p.rows * r.p.cols > 0) ? (r.p.k + r.T - 1) / r.T : 0;
  r.tiles = tile_geom(r.p, shape).ntiles;
}

// Admit the head of the queue if it fits (lock held).
bool try_admit(phgrms_server* S, Req& r) {
  if ((int)S->active.size() >= S->cfg.max_active) return false;
  if (S->cfg.passes_per_step < 0) {
    const long long npx = (long long)r.p.rows * r.p.cols;
    set_shape(r, S->active.size() >= kBusyActive ? batch_shape(r.p.beta, npx)
                                                 : shape_for(r.p.beta, npx, 1));
  }
  if (S->active_tiles + r.tiles > (long long)S->tiles_cap) return false;
  if (S->heap.in_use + r.bytes > S->cfg.cap_bytes) return false;
  size_t off = 0;
  if (!S->heap.alloc(r.bytes, &off)) return false;
  r.off = off;
  uint8_t* base = S->arena + off;
  r.counts = reinterpret_cast<unsigned long long*>(base);
  const size_t cbytes = up256(sizeof(uint64_t) * kCountSlots * size_t(std::max(r.p.k, 1)));
  const size_t n = size_t(std::max<int64_t>((int64_t)r.p.rows * r.p.cols, 1));
  r.wsimg = base + cbytes;
  r.out = base + cbytes + up256(n);
  // A host request's input is copied into the buffer its first launch does
  // not write (the workspace image when no launch runs).
  if (r.h_in != nullptr) r.in = (r.L >= 1 && (r.L - 1) % 2 == 1) ? r.out : r.wsimg;
  r.state = kActive;
  r.launched = 0;
  S->active.push_back(r.id);
  S->active_tiles += r.tiles;
  return true;
}

// Complete the oldest in-flight step (lock held; the event has completed).
void complete_oldest(phgrms_server* S) {
  const auto step = S->inflight.front();
  S->inflight.pop_front();
  S->slot_busy[step.slot] = false;
  const double t = now_s();
  // requests whose launch in this step found them converged get no more
  // launches (theirs would be no-ops) and finish in the next step built
  const int32_t* st = reinterpret_cast<const int32_t*>(S->hslot[step.slot] + S->stat_off);
  for (size_t i = 0; i < step.launched.size(); ++i) {
    if (st[i] == 0) continue;
    auto it = S->reqs.find(step.launched[i]);
    if (it != S->reqs.end() && it->second.state == kActive) it->second.converged = true;
  }
  const int64_t* res = reinterpret_cast<const int64_t*>(S->hslot[step.slot] + S->res_off);
  for (size_t f = 0; f < step.finishing.size(); ++f) {
    auto it = S->reqs.find(step.finishing[f]);
    if (it == S->reqs.end()) continue;
    Req& r = it->second;
    const int64_t* rr = res + f * kResStride;
    r.iterations = *reinterpret_cast<const int32_t*>(rr);
    r.changed.assign(rr + 2, rr + 2 + r.p.k);
    r.state = kDone;
    r.t_done = t;
    S->done_queue.push_back(r.id);
    S->n_completed++;
  }
  S->cv.notify_all();
}

void fail_all(phgrms_server* S, int code) {
  S->error = code;
  for (auto& kv : S->reqs)
    if (kv.second.state != kDone) kv.second.state = kFailed;
  S->pending.clear();
  S->active.clear();
  S->cv.notify_all();
}

// Build and enqueue one step over the active requests (lock held on entry
// and exit; released around the HIP calls).
int run_step(phgrms_server* S, std::unique_lock<std::mutex>& lk) {
  int slot = -1;
  for (int i = 0; i < kSlots; ++i)
    if (!S->slot_busy[i]) slot = i;
  if (slot < 0) return PHGRMS_OK;
  uint8_t* h = S->hslot[slot];
  uint8_t* d = S->dslot[slot];
  auto* dres = reinterpret_cast<int64_t*>(d + S->res_off);

  struct Launch {
    int beta, shape;
    size_t tiles_base, ntiles, imgs_base;
  };
  std::vector<Launch> launches;
  std::vector<uint64_t> finishing;
  std::vector<uint64_t> launched;
  // group active requests by (beta, shape)
  std::map<std::pair<int, int>, std::vector<uint64_t>> groups;
  // The step's descriptors are packed at the start of the slot, image
  // descriptors, then finish descriptors, then the tile table, so that one
  // copy uploads them: count them first.  (They fit: at most max_active
  // images and finishes, and the admitted tiles stay under the table's cap.)
  size_t ni_all = 0, nt_all = 0, nf_all = 0;
  // Test hook (PHGRMS_FAULT_INJECT): the chosen request fails on the host
  // before its first launch; nothing of it was enqueued, so its block is
  // free at once, and the other requests go on.
  if (S->fault_id != 0) {
    auto it = S->reqs.find(S->fault_id);
    if (it != S->reqs.end() && it->second.state == kActive && it->second.launched == 0) {
      Req& r = it->second;
      r.state = kFailed;
      r.t_done = now_s();
      S->active.erase(std::find(S->active.begin(), S->active.end(), r.id));
      S->active_tiles -= r.tiles;
      S->heap.release(r.off, r.bytes);
      S->done_queue.push_back(r.id);
      S->fault_id = 0;
      S->generation++;
      S->cv.notify_all();
    }
  }
  auto launches_now = [](const Req& r) { return r.launched < r.L && !r.converged; };
  for (uint64_t id : S->active) {
    Req& r = S->reqs[id];
    if (launches_now(r)) {
      groups[{r.p.beta, r.shape}].push_back(id);
      ++ni_all;
      nt_all += size_t(tile_geom(r.p, r.shape).ntiles);
    }
    if (r.converged || r.launched + (launches_now(r) ? 1 : 0) >= r.L) ++nf_all;
  }
  const size_t o_imgs = 0;
  const size_t o_fin = up256(o_imgs + ni_all * sizeof(ImageDesc));
  const size_t o_tiles = up256(o_fin + nf_all * sizeof(BatchFinishDesc));
  const size_t up_bytes = o_tiles + nt_all * sizeof(TileRef);
  if (up_bytes > S->stat_off) {   // cannot happen (see the slot layout); fail loudly if it does
    fail(PHGRMS_EDEVICE, "server step descriptors exceed the slot");
    fail_all(S, PHGRMS_EDEVICE);
    return PHGRMS_EDEVICE;
  }
  auto* htiles = reinterpret_cast<TileRef*>(h + o_tiles);
  auto* himgs = reinterpret_cast<ImageDesc*>(h + o_imgs);
  auto* dstat = reinterpret_cast<int*>(d + S->stat_off);
  auto* hfin = reinterpret_cast<BatchFinishDesc*>(h + o_fin);
  size_t nt = 0, ni = 0;
  for (auto& kv : groups) {
    Launch L{kv.first.first, kv.first.second, nt, 0, ni};
    int local = 0;
    for (uint64_t id : kv.second) {
      Req& r = S->reqs[id];
      const int j = r.launched;
      auto dst_of = [&](int jj) -> uint8_t* { return ((r.L - 1 - jj) % 2 == 0) ? r.out : r.wsimg; };
      const TileGeom tg = tile_geom(r.p, r.shape);
      ImageDesc x;
      std::memset(&x, 0, sizeof(x));
      x.src = (j == 0) ? r.in : dst_of(j - 1);
      x.dst = dst_of(j);
      x.counts = r.counts;
      x.rows = r.p.rows;
      x.cols = r.p.cols;
      x.alpha = r.p.alpha;
      x.pass0 = j * r.T;
      x.npasses = std::min(r.T, r.p.k - j * r.T);
      x.prev_passes = j >= 1 ? std::min(r.T, r.p.k - (j - 1) * r.T) : 0;
      x.tiles_x = tg.tiles_x;
      x.status = dstat + ni;
      launched.push_back(id);
      himgs[ni++] = x;
      for (long long t = 0; t < tg.ntiles; ++t) htiles[nt++] = TileRef{local, int(t)};
      ++local;
      r.launched++;
    }
    L.ntiles = nt - L.tiles_base;
    launches.push_back(L);
  }
  // requests whose last launch is in this step (or that need none) finish
  size_t nf = 0;
  for (uint64_t id : S->active) {
    Req& r = S->reqs[id];
    if (r.launched < r.L && !r.converged) continue;
    BatchFinishDesc f;
    std::memset(&f, 0, sizeof(f));
    f.counts = r.counts;
    f.changed = reinterpret_cast<unsigned long long*>(dres + nf * kResStride + 2);
    f.iterations = reinterpret_cast<int*>(dres + nf * kResStride);
    f.first_src = r.in;
    f.buf_even_from_end = r.out;
    f.buf_odd_from_end = r.wsimg;
    f.out = r.out;
    f.n = (long long)r.p.rows * r.p.cols;
    f.k = r.p.k;
    f.T = r.T;
    f.launches = r.L;
    hfin[nf++] = f;
    finishing.push_back(id);
    r.state = kFinishing;
  }
  for (uint64_t id : finishing) {
    S->active.erase(std::find(S->active.begin(), S->active.end(), id));
    S->active_tiles -= S->reqs[id].tiles;
  }
  // requests in their first step: clear their count slots (and copy a
  // host request's input in) before anything
  std::vector<uint8_t*> zero_counts;
  std::vector<size_t> zero_n;
  struct HostCopy {
    void* dst;
    const void* src;
    size_t n;
  };
  std::vector<HostCopy> uploads, downloads;
  auto zero_if_new = [&](Req& r) {
    if (r.zeroed) return;
    r.zeroed = true;
    zero_counts.push_back(reinterpret_cast<uint8_t*>(r.counts));
    zero_n.push_back(size_t(std::max(r.p.k, 1)) * kCountSlots);
    const size_t n = size_t((int64_t)r.p.rows * r.p.cols);
    if (r.h_in != nullptr && n > 0) uploads.push_back({const_cast<uint8_t*>(r.in), r.h_in, n});
  };
  for (auto& kv : groups)
    for (uint64_t id : kv.second) zero_if_new(S->reqs[id]);
  for (uint64_t id : finishing) {
    Req& r = S->reqs[id];
    zero_if_new(r);
    const size_t n = size_t((int64_t)r.p.rows * r.p.cols);
    if (r.h_out != nullptr && n > 0) downloads.push_back({r.h_out, r.out, n});
  }
  S->slot_busy[slot] = true;
  lk.unlock();

  hipError_t e = hipSuccess;
  hipStream_t s = S->stream;
  for (size_t z = 0; z < zero_counts.size() && e == hipSuccess; ++z) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(int(std::min<size_t>((zero_n[z] + 255) / 256, 256))),
                       dim3(256), 0, s, reinterpret_cast<unsigned long long*>(zero_counts[z]),
                       (long long)zero_n[z]);
    e = hipGetLastError();
  }
  for (size_t u = 0; u < uploads.size() && e == hipSuccess; ++u)
    e = hipMemcpyAsync(uploads[u].dst, uploads[u].src, uploads[u].n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && up_bytes > 0)
    e = hipMemcpyAsync(d, h, up_bytes, hipMemcpyHostToDevice, s);
  for (auto& L : launches) {
    if (e != hipSuccess || L.ntiles == 0) continue;
    MultiArgs a;
    a.images = reinterpret_cast<const ImageDesc*>(d + o_imgs) + L.imgs_base;
    a.tiles = reinterpret_cast<const TileRef*>(d + o_tiles) + L.tiles_base;
    a.ntiles = int(L.ntiles);
    void* args[] = {&a};
    const long long grid = std::min<long long>((L.ntiles + 7) / 8 * 8,
                                               max_workgroups(kShapes[L.shape].waves * 64));
    e = hipLaunchKernel(multi_kernel_ptr(L.beta, L.shape), dim3(int(grid)),
                        dim3(kShapes[L.shape].waves * 64), args, 0, s);
  }
  if (e == hipSuccess && nf > 0) {
    hipLaunchKernelGGL(batch_finish_kernel, dim3(64, int(std::min<size_t>(nf, 65535))), dim3(256), 0, s,
                       reinterpret_cast<const BatchFinishDesc*>(d + o_fin), int(nf));
    e = hipGetLastError();
  }
  // one copy back: the launches' convergence status and (when requests
  // finish) their results, which follow it in the slot
  const size_t back = nf > 0 ? (S->res_off - S->stat_off) + nf * kResStride * sizeof(int64_t)
                             : ni * sizeof(int32_t);
  if (e == hipSuccess && back > 0)
    e = hipMemcpyAsync(h + S->stat_off, d + S->stat_off, back, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && nf > 0) {
    for (size_t u = 0; u < downloads.size() && e == hipSuccess; ++u)
      e = hipMemcpyAsync(downloads[u].dst, downloads[u].src, downloads[u].n, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipEventRecord(S->ev[slot], s);
  lk.lock();
  if (e != hipSuccess) {
    hip_fail(e, "server step");
    fail_all(S, PHGRMS_EDEVICE);
    return PHGRMS_EDEVICE;
  }
  S->inflight.push_back({slot, finishing, launched});
  S->n_steps++;
  return PHGRMS_OK;
}

void worker_main(phgrms_server* S) {
  if (hipSetDevice(S->cfg.device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    fail_all(S, PHGRMS_EDEVICE);
    return;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  uint64_t seen = ~uint64_t(0);
  while (!S->stop) {
    // completions that are already there
    while (!S->inflight.empty() && hipEventQuery(S->ev[S->inflight.front().slot]) == hipSuccess)
      complete_oldest(S);
    // admission in arrival order
    while (!S->pending.empty()) {
      Req& r = S->reqs[S->pending.front()];
      if (!try_admit(S, r)) break;
      S->pending.pop_front();
    }
    bool slot_free = false;
    for (int i = 0; i < kSlots; ++i) slot_free |= !S->slot_busy[i];
    if (!S->active.empty() && slot_free) {
      if (run_step(S, lk) != PHGRMS_OK) break;
      continue;
    }
    if (!S->inflight.empty()) {
      const int slot = S->inflight.front().slot;
      lk.unlock();
      const hipError_t e = hipEventSynchronize(S->ev[slot]);
      lk.lock();
      if (e != hipSuccess) {
        hip_fail(e, "server event");
        fail_all(S, PHGRMS_EDEVICE);
        break;
      }
      complete_oldest(S);
      continue;
    }
    // nothing runs: wait for a submit or a release (the head of the queue
    // may be waiting for memory)
    seen = S->generation;
    S->cv.wait(lk, [&] { return S->stop || S->generation != seen; });
  }
  // let in-flight work finish before the stream goes away
  lk.unlock();
  (void)hipStreamSynchronize(S->stream);
}

}  // namespace

extern "C" {

int phgrms_server_create(const phgrms_server_cfg* cfg, void* d_arena, size_t arena_bytes,
                         phgrms_server** out) {
  if (cfg == nullptr || out == nullptr || d_arena == nullptr)
    return fail(PHGRMS_EINVAL, "null server argument");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 65535 || cfg->max_queue < 1 || cfg->passes_per_step < -1)
    return fail(PHGRMS_EINVAL, "bad server configuration");
  auto* S = new phgrms_server();
  S->cfg = *cfg;
  S->arena = static_cast<uint8_t*>(d_arena);
  S->arena_bytes = arena_bytes;
  const size_t na = size_t(cfg->max_active);
  S->tiles_cap = std::min<size_t>(arena_bytes / 4096 + 64 * na, size_t(16) << 20);
  S->tiles_off = 0;
  S->imgs_off = up256(S->tiles_off + S->tiles_cap * sizeof(TileRef));
  S->fin_off = up256(S->imgs_off + na * sizeof(ImageDesc));
  // (+512: a step packs the three tables from offset 0, with a 256-byte
  // alignment after each of the first two)
  S->stat_off = up256(S->fin_off + na * sizeof(BatchFinishDesc) + 512);
  S->res_off = up256(S->stat_off + na * sizeof(int32_t));
  S->slot_bytes = up256(S->res_off + na * kResStride * sizeof(int64_t));
  const size_t reserved = kSlots * S->slot_bytes;
  if (arena_bytes <= reserved + 4096) {
    delete S;
    return fail(PHGRMS_ENOSPC, "arena of %zu bytes; the server needs %zu for descriptors", arena_bytes,
                reserved);
  }
  if (S->cfg.cap_bytes == 0 || S->cfg.cap_bytes > arena_bytes - reserved)
    S->cfg.cap_bytes = arena_bytes - reserved;
  if (const char* fi = std::getenv("PHGRMS_FAULT_INJECT")) {
    char* end = nullptr;
    const unsigned long long v = std::strtoull(fi, &end, 10);
    if (end != fi && *end == '\0') S->fault_id = v;
  }
  S->heap.init(reserved, arena_bytes - reserved);
  hipError_t e = hipSetDevice(cfg->device);
  for (int i = 0; i < kSlots && e == hipSuccess; ++i) {
    S->dslot[i] = S->arena + size_t(i) * S->slot_bytes;
    e = hipHostMalloc(reinterpret_cast<void**>(&S->hslot[i]), S->slot_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    for (int i = 0; i < kSlots; ++i) {
      if (S->hslot[i]) (void)hipHostFree(S->hslot[i]);
      if (S->ev[i]) (void)hipEventDestroy(S->ev[i]);
    }
    delete S;
    return hip_fail(e, "server resources");
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return PHGRMS_OK;
}

}  // extern "C"

namespace {

int submit_request(phgrms_server* S, const uint8_t* d_img, const uint8_t* h_img, uint8_t* h_out,
                   phgrms_params p, uint64_t* req_id) {
  if (S == nullptr || req_id == nullptr) return fail(PHGRMS_EINVAL, "null argument");
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  if ((int64_t)p.rows * p.cols > 0 && d_img == nullptr && (h_img == nullptr || h_out == nullptr))
    return fail(PHGRMS_EINVAL, "null image");
  Req r;
  r.p = p;
  r.in = d_img;
  r.h_in = h_img;
  r.h_out = h_out;
  const long long npx = (long long)p.rows * p.cols;
  if (S->cfg.passes_per_step >= 0) {
    set_shape(r, shape_for(p.beta, npx, S->cfg.passes_per_step));
  } else {
    // adaptive: the shape is chosen at admission; the footprint check takes
    // the larger tile count of the two candidates
    set_shape(r, batch_shape(p.beta, npx));
    const long long t_batch = r.tiles;
    set_shape(r, shape_for(p.beta, npx, 1));
    r.tiles = std::max(r.tiles, t_batch);
  }
  r.bytes = request_bytes(p);
  r.t_submit = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->error != PHGRMS_OK) return fail(S->error, "server failed earlier");
  if (r.bytes > S->cfg.cap_bytes || r.tiles > (long long)S->tiles_cap)
    return fail(PHGRMS_EINVAL, "request footprint %zu bytes exceeds the cap %llu", r.bytes,
                (unsigned long long)S->cfg.cap_bytes);
  if ((int)S->pending.size() >= S->cfg.max_queue) return fail(PHGRMS_EBUSY, "queue full");
  r.id = S->next_id++;
  *req_id = r.id;
  S->reqs.emplace(r.id, std::move(r));
  S->pending.push_back(*req_id);
  S->n_submitted++;
  S->generation++;
  S->cv.notify_all();
  return PHGRMS_OK;
}

}  // namespace

extern "C" {

int phgrms_server_submit(phgrms_server* S, const uint8_t* d_img, phgrms_params p, uint64_t* req_id) {
  return submit_request(S, d_img, nullptr, nullptr, p, req_id);
}

int phgrms_server_submit_host(phgrms_server* S, const uint8_t* h_img, uint8_t* h_out,
                              phgrms_params p, uint64_t* req_id) {
  if ((int64_t)p.rows * p.cols > 0 && (h_img == nullptr || h_out == nullptr))
    return fail(PHGRMS_EINVAL, "null host buffer");
  if (h_img != nullptr && h_out != nullptr && p.rows > 0 && p.cols > 0) {
    const size_t n = size_t((int64_t)p.rows * p.cols);
    const uintptr_t a = reinterpret_cast<uintptr_t>(h_img), b = reinterpret_cast<uintptr_t>(h_out);
    if (a < b + n && b < a + n) return fail(PHGRMS_EINVAL, "host input and output overlap");
  }
  return submit_request(S, nullptr, h_img, h_out, p, req_id);
}

int phgrms_server_poll(phgrms_server* S, uint64_t req_id, uint8_t** d_out, int32_t* iterations,
                       int64_t* changed, double* latency_s) {
  if (S == nullptr) return fail(PHGRMS_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(PHGRMS_ENOTFOUND, "unknown request %llu", (unsigned long long)req_id);
  Req& r = it->second;
  if (r.state == kFailed) return fail(PHGRMS_EDEVICE, "request %llu failed", (unsigned long long)req_id);
  if (r.state != kDone) return PHGRMS_EAGAIN;
  if (d_out) *d_out = r.out;
  if (iterations) *iterations = r.iterations;
  if (changed && r.p.k > 0) std::memcpy(changed, r.changed.data(), sizeof(int64_t) * size_t(r.p.k));
  if (latency_s) *latency_s = r.t_done - r.t_submit;
  return PHGRMS_OK;
}

int phgrms_server_next_done(phgrms_server* S, uint64_t* ids, int32_t max) {
  if (S == nullptr || (ids == nullptr && max > 0) || max < 0) return fail(PHGRMS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  int n = 0;
  while (n < max && !S->done_queue.empty()) {
    ids[n++] = S->done_queue.front();
    S->done_queue.pop_front();
  }
  return n;
}

int phgrms_server_release(phgrms_server* S, uint64_t req_id) {
  if (S == nullptr) return fail(PHGRMS_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(PHGRMS_ENOTFOUND, "unknown request %llu", (unsigned long long)req_id);
  if (it->second.state != kDone && it->second.state != kFailed) return PHGRMS_EAGAIN;
  if (it->second.state == kDone) S->heap.release(it->second.off, it->second.bytes);
  S->reqs.erase(it);
  S->generation++;
  S->cv.notify_all();
  return PHGRMS_OK;
}

int phgrms_server_get_stats(phgrms_server* S, phgrms_server_stats* st) {
  if (S == nullptr || st == nullptr) return fail(PHGRMS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->n_submitted;
  st->completed = S->n_completed;
  st->queued = S->pending.size();
  st->active = S->active.size();
  st->steps = S->n_steps;
  st->bytes_in_use = S->heap.in_use;
  return S->error;
}

void phgrms_server_destroy(phgrms_server* S) {
  if (S == nullptr) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->pending.clear();
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (int i = 0; i < kSlots; ++i) {
    if (S->hslot[i]) (void)hipHostFree(S->hslot[i]);
    if (S->ev[i]) (void)hipEventDestroy(S->ev[i]);
  }
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
