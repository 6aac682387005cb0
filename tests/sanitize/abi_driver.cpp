// Host-side paths of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer, with no GPU: argument validation of every
// entry point (it runs before any HIP call), the batch planner, and the
// tuning cache reader and writer on valid, malformed and randomly mutated
// files.  Built host-only and run by tests/test_sanitizers.py; exit status
// 0 when every expectation holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "phgrms.h"

static int failures = 0;
#define EXPECT(c)                                                            \
  do {                                                                       \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "expectation failed at line %d: %s (%s)\n", __LINE__, #c, \
                   phgrms_last_error());                                     \
      failures++;                                                            \
    }                                                                        \
  } while (0)

static uint64_t rng = 88172645463325252ull;
static uint32_t rnd() {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return uint32_t(rng >> 16);
}

static bool write_file(const std::string& path, const std::string& text) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return false;
  std::fwrite(text.data(), 1, text.size(), f);
  std::fclose(f);
  return true;
}

static std::string read_file(const std::string& path) {
  std::string s;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return s;
  char b[4096];
  size_t n;
  while ((n = std::fread(b, 1, sizeof(b), f)) > 0) s.append(b, n);
  std::fclose(f);
  return s;
}

int main(int argc, char** argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  // pointers that are never dereferenced: validation fails first
  uint8_t* fake = reinterpret_cast<uint8_t*>(uintptr_t(0x100000));
  uint8_t* fake2 = reinterpret_cast<uint8_t*>(uintptr_t(0x200000));
  void* ws = reinterpret_cast<void*>(uintptr_t(0x10000000));

  for (int c = 1; c >= -8; --c) EXPECT(phgrms_status_str(c) != nullptr);
  EXPECT(phgrms_workspace_bytes({100, 37, 20, 1, 10}) > 0);
  EXPECT(phgrms_workspace_bytes({100, 37, 300, 1, 10}) == 0);
  EXPECT(phgrms_workspace_bytes({-1, 37, 20, 1, 10}) == 0);
  const phgrms_params p{64, 64, 20, 1, 4};
  const size_t need = phgrms_workspace_bytes(p);
  EXPECT(phgrms_denoise_async(fake, fake2, {64, 64, 20, 0, 4}, ws, need, nullptr, nullptr, nullptr) ==
         PHGRMS_EINVAL);
  EXPECT(phgrms_denoise_async(fake, fake2, {64, 64, 20, 9, 4}, ws, need, nullptr, nullptr, nullptr) ==
         PHGRMS_EUNSUPPORTED);
  EXPECT(phgrms_denoise_async(fake, fake2, p, ws, need - 1, nullptr, nullptr, nullptr) == PHGRMS_ENOSPC);
  EXPECT(phgrms_denoise_async(fake, fake + 1, p, ws, need, nullptr, nullptr, nullptr) == PHGRMS_EINVAL);
  EXPECT(phgrms_denoise_async(nullptr, fake2, p, ws, need, nullptr, nullptr, nullptr) == PHGRMS_EINVAL);
  EXPECT(phgrms_denoise_ex(fake, fake2, p, 8, ws, need, nullptr, nullptr, nullptr) == PHGRMS_EINVAL);
  EXPECT(phgrms_denoise_plain(fake, fake2, {64, 64, 20, 1, 2000}, ws, need, nullptr, nullptr, nullptr) ==
         PHGRMS_EINVAL);
  EXPECT(phgrms_cardinality(fake, 10, 10, 256, 1, nullptr, nullptr) == PHGRMS_EINVAL);
  EXPECT(phgrms_salt_pepper(fake, fake, -1, 0, 0, 0, nullptr) == PHGRMS_EINVAL);
  EXPECT(phgrms_change_map_bytes({8192, 8192, 20, 2, 1}) > 0);
  EXPECT(phgrms_run_passes(fake, fake2, {64, 64, 20, 1, 1}, 999, 0, nullptr, nullptr, nullptr) ==
         PHGRMS_EINVAL);
  const int ns = phgrms_num_shapes();
  for (int s = 0; s < ns; ++s) {
    int32_t t = 0, r = 0, w = 0;
    EXPECT(phgrms_shape_info(s, &t, &r, &w) == PHGRMS_OK && t >= 1 && r >= 1 && w >= 1);
    EXPECT(phgrms_shape_tracks_changes(s) >= 0 && phgrms_shape_skips_unchanged(s) >= 0);
  }

  // the batch planner (host only), with and without a tuning cache
  std::vector<phgrms_item> items;
  uint64_t off = 0;
  for (int i = 0; i < 40; ++i) {
    phgrms_params q{int32_t(1 + rnd() % 700), int32_t(1 + rnd() % 700), int32_t(rnd() % 256),
                    int32_t(1 + rnd() % 4), int32_t(rnd() % 40)};
    items.push_back({off, off, q});
    off += (uint64_t(q.rows) * q.cols + 255) / 256 * 256;
  }
  phgrms_plan* plan = nullptr;
  size_t pws = 0;
  EXPECT(phgrms_batch_plan(items.data(), int32_t(items.size()), nullptr, &plan, &pws) == PHGRMS_OK);
  EXPECT(plan != nullptr && pws > 0 && phgrms_batch_launches(plan) > 0);
  phgrms_plan_destroy(plan);
  plan = nullptr;
  const std::string cache = dir + "/tune.json";
  EXPECT(phgrms_save_tuning(cache.c_str()) == PHGRMS_OK);
  EXPECT(phgrms_load_tuning(cache.c_str()) == PHGRMS_OK);
  EXPECT(phgrms_batch_plan(items.data(), int32_t(items.size()), cache.c_str(), &plan, &pws) ==
         PHGRMS_OK);
  phgrms_plan_destroy(plan);
  EXPECT(phgrms_batch_plan(items.data(), int32_t(items.size()), (dir + "/none.json").c_str(), &plan,
                           &pws) == PHGRMS_ENOTFOUND);

  // the tuning cache reader on mutations of a valid file: OK or EINVAL,
  // never a crash, and a failed read changes nothing
  const std::string good = read_file(cache);
  EXPECT(!good.empty());
  int ok = 0, bad = 0;
  for (int trial = 0; trial < 3000; ++trial) {
    std::string t = good;
    const int edits = 1 + int(rnd() % 4);
    for (int e = 0; e < edits && !t.empty(); ++e) {
      const size_t at = rnd() % t.size();
      switch (rnd() % 4) {
        case 0: t[at] = char(rnd() & 0xFF); break;
        case 1: t.erase(at, 1 + rnd() % 8); break;
        case 2: t.insert(at, 1, "{}[],:\"\\0123456789-e.u"[rnd() % 22]); break;
        default: t.resize(at); break;
      }
    }
    const std::string path = dir + "/mut.json";
    EXPECT(write_file(path, t));
    int32_t before[4];
    for (int b = 1; b <= 4; ++b) before[b - 1] = phgrms_get_tuning_class(b, 2);
    const int rc = phgrms_load_tuning(path.c_str());
    EXPECT(rc == PHGRMS_OK || rc == PHGRMS_EINVAL);
    if (rc == PHGRMS_OK) {
      ++ok;
    } else {
      ++bad;
      for (int b = 1; b <= 4; ++b) EXPECT(phgrms_get_tuning_class(b, 2) == before[b - 1]);
    }
    const int wc = phgrms_save_tuning(path.c_str());
    EXPECT(wc == PHGRMS_OK || wc == PHGRMS_EINVAL);
  }
  EXPECT(ok > 0 && bad > 0);
  EXPECT(phgrms_load_tuning(cache.c_str()) == PHGRMS_OK);
  if (failures) {
    std::fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  std::printf("abi driver: all expectations held (%d mutated caches read, %d refused)\n", ok, bad);
  return 0;
}
