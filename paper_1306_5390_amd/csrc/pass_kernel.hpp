// pass_kernel.hpp -- gfx950 kernels of the P-HGRMS pass loop (Section 2 of
// the paper: Algorithm 1, Algorithm 2 and the temporary-image update).
//
// One launch of pass_kernel<BETA, T, R, WAVES> runs up to T passes of the
// method on a tile held in LDS:
//
//   * the workgroup loads its tile plus a T*BETA halo from HBM once
//     (dword loads, re-aligned to the image's byte offset);
//   * each pass reads one LDS buffer and writes the other (the temporary
//     image of Algorithm 2; every read of a pass sees the pre-pass image);
//     the region that is still exact shrinks by BETA rows and columns per
//     pass, so after T passes the owned region is exact;
//   * the owned region is stored back to HBM once.
//
// Per pixel the pass needs one fact from Algorithms 1-2 taken together: an
// interior pixel (more than BETA from the image border) is replaced iff at
// most 2 pixels of its window, itself included, lie in (x-alpha, x+alpha];
// border pixels are never replaced.  (Algorithm 2 counts every window
// position, so a border pixel can never have more than N-3 "outside"
// pixels; for an interior pixel "outside > N-3" is "inside <= 2", which also
// implies the cardinality gate C <= 2 of Algorithm 1.)
//
// The band test runs four pixels per 32-bit lane (byte SWAR).  For a byte y
// and the centre's clamped band [lo, hi]:
//   v_lerp_u8(y, 255-lo, 1) has bit 7 set iff y + 256 - lo >= 256, i.e. y >= lo
//   v_lerp_u8(y, 255-hi, 0) has bit 7 set iff y + 255 - hi >= 256, i.e. y >  hi
// and since y > hi implies y >= lo, their XOR has bit 7 set iff y is in the
// band.  "At least two other window pixels in the band" is accumulated with a
// carry-save majority / xor3 tree on v_bitop3_b32 (bit 7 of each byte only).
// Pixels that fail it are candidates: they go to a per-wave queue in LDS and
// are re-evaluated exactly, one lane per pixel, which also yields the root
// mean square of Algorithm 2 and the changed count.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phg {

constexpr int kRowBytes = 264;              // LDS row: pad 4 + 256 + pad 4
constexpr int kRowWords = kRowBytes / 4;    // 66
constexpr int kQueueCap = 512;              // pixel queue entries per wave (u16)
constexpr int kLaneQueueCap = 128;          // lane queue entries per wave (u32)
// Word 3 of a raw buffer descriptor on gfx9-family GPUs (32-bit data
// format, no swizzle, range-checked offsets).
constexpr int kBufferWord3 = 0x00020000;

struct PassArgs {
  const uint8_t* src;            // image before this launch's first pass
  uint8_t* dst;                  // image after this launch's last pass
  unsigned long long* changed;   // count slots, kCountSlots per pass, zeroed beforehand
  int rows, cols, alpha;
  int pass0;                     // index of this launch's first pass
  int npasses;                   // passes in this launch, 1..T
  int tiles_x;                   // tiles per tile row
  int ntiles;                    // tiles of the image (the grid is persistent)
  const uint8_t* map_in;         // change map of the previous pass, or null
  uint8_t* map_out;              // change map of this pass, or null
  const uint8_t* prev2;          // (one pass per launch) image two passes before this
                                 // launch's output, or null: count the pixels that differ
  unsigned long long* diff2;     // those counts, kCountSlots per pass (zeroed beforehand)
  int seq;                       // position of this launch in its sequence (one pass per
                                 // launch): stamps of the change maps, lists in use
  uint32_t* list_state;          // (skipping shapes) tile lists, see TileLists
  int list_cap;                  // tiles of the image (at least)
};

// Tile lists of the skipping shapes, in one uint32 array: the counts of
// three lists of kListShards shards each (one cache line per count), one
// mark per tile, then the lists.  A sequence of launches runs: launches 0
// and 1 with plain change tracking (TRACK 1; the pass loop runs them with
// the dense kernel instead, and clears the counts and marks beforehand),
// launch 2 over every tile (TRACK 2), launches
// j >= 3 over the tiles of list j % 3 (TRACK 3), the workgroups with index
// b = s (mod kListShards) taking the entries of shard s in turn.  Launches
// j >= 2 append each tile
// that can change in launch j+1 to list (j+1) % 3, once: the tile's mark is
// swapped for j+1, and the workgroup that finds an older mark appends it,
// to shard (workgroup index) % kListShards, with one atomic add per
// workgroup and tile (so that appends spread over the shards' counts); and
// they clear the counts of list (j+2) % 3, which launch j+1 fills.
constexpr int kListShards = 16;
constexpr int kListRound = 256;   // a multiple of kListShards
struct TileLists {
  static constexpr int kHead = 3 * kListShards * 16;
  __host__ __device__ static uint32_t* count(uint32_t* s, int l, int shard) {
    return s + 16 * (l * kListShards + shard);
  }
  __host__ __device__ static uint32_t* marks(uint32_t* s) { return s + kHead; }
  __host__ __device__ static uint32_t* shard(uint32_t* s, int cap, int l, int sh) {
    return s + kHead + size_t(cap) + (size_t(l) * kListShards + size_t(sh)) * size_t(cap);
  }
  __host__ __device__ static size_t words(int cap) {
    return size_t(kHead) + size_t(cap) * (1 + 3 * kListShards);
  }
};

// ---- small integer helpers -------------------------------------------------

__device__ __forceinline__ uint32_t bitop3_maj(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
__device__ __forceinline__ uint32_t bitop3_xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t bitop3_or3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xFE);
}

// Offset (dr, dc) of neighbour k of the window in ring order: k = 0..3 the
// 4-connected neighbours, 4..7 the diagonals, then ring d >= 2 (the 8d
// positions at Chebyshev distance d) from k = 4d(d-1): its top row, its
// bottom row, its left column, its right column.
__host__ __device__ constexpr void ring_offset(int k, int& dr, int& dc) {
  if (k < 4) {
    dr = (k == 0) ? -1 : (k == 1) ? 1 : 0;
    dc = (k == 2) ? -1 : (k == 3) ? 1 : 0;
    return;
  }
  if (k < 8) {
    dr = (k < 6) ? -1 : 1;
    dc = (k & 1) ? 1 : -1;
    return;
  }
  int d = 2;
  while (k >= 4 * d * (d + 1)) ++d;
  const int e = k - 4 * d * (d - 1);
  const int side = 2 * d + 1;
  if (e < side) { dr = -d; dc = e - d; return; }
  if (e < 2 * side) { dr = d; dc = e - side - d; return; }
  const int f = e - 2 * side;          // 0 .. 4d-3
  if (f < 2 * d - 1) { dr = f - d + 1; dc = -d; return; }
  dr = f - (2 * d - 1) - d + 1;
  dc = d;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per byte: min(a + b, 255) and max(a - b, 0), b given as (b<<8)|(b<<24).
// Bytes are moved to the high half of 16-bit lanes so that the saturating
// 16-bit add/sub (v_pk_add_u16 / v_pk_sub_u16 with clamp) saturates them.
__device__ __forceinline__ uint32_t sat_add_u8x4(uint32_t a, uint32_t b16) {
  const uint32_t hi = a & 0xFF00FF00u;
  const uint32_t lo = (a << 8) & 0xFF00FF00u;
  const u16x2 bb = __builtin_bit_cast(u16x2, b16);
  const uint32_t h = __builtin_bit_cast(uint32_t,
      __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, hi), bb));
  const uint32_t l = __builtin_bit_cast(uint32_t,
      __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, lo), bb));
  return __builtin_amdgcn_perm(h, l, 0x07030501u);
}
__device__ __forceinline__ uint32_t sat_sub_u8x4(uint32_t a, uint32_t b16) {
  const uint32_t hi = a & 0xFF00FF00u;
  const uint32_t lo = (a << 8) & 0xFF00FF00u;
  const u16x2 bb = __builtin_bit_cast(u16x2, b16);
  const uint32_t h = __builtin_bit_cast(uint32_t,
      __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, hi), bb));
  const uint32_t l = __builtin_bit_cast(uint32_t,
      __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, lo), bb));
  return __builtin_amdgcn_perm(h, l, 0x07030501u);
}

// floor(sqrt(q)) for q < 2^16, by setting result bits from the top.
__device__ __forceinline__ uint32_t isqrt16(uint32_t q) {
  uint32_t r = 0;
#pragma unroll
  for (uint32_t bit = 128; bit != 0; bit >>= 1) {
    const uint32_t t = r | bit;
    r = (t * t <= q) ? t : r;
  }
  return r;
}

// floor(S / F) for S < 2^24 and 1 <= F <= 2^8: a float estimate (the
// hardware reciprocal, relative error far below 2^-20, so the estimate is
// within one of the quotient) corrected to the exact integer quotient.
__device__ __forceinline__ uint32_t udiv_small(uint32_t S, uint32_t F) {
  uint32_t q = uint32_t(float(S) * __builtin_amdgcn_rcpf(float(F)));
  const int32_t r = int32_t(S) - int32_t(q * F);
  if (r < 0) --q;
  else if (uint32_t(r) >= F) ++q;
  return q;
}

// floor(sqrt(q)) for q < 2^16: the hardware square root, corrected to the
// exact integer square root by comparing squares.
__device__ __forceinline__ uint32_t isqrt_small(uint32_t q) {
  uint32_t r = uint32_t(__builtin_amdgcn_sqrtf(float(q)));
  if (r * r > q) --r;
  if ((r + 1) * (r + 1) <= q) ++r;
  return r;
}

// An aligned dword that overlaps [lo, hi) lies in the same page as a byte of
// that range, so reading it cannot fault even where it extends past the range.
__device__ __forceinline__ uint32_t load_dword_overlapping(uintptr_t a, uintptr_t lo,
                                                           uintptr_t hi) {
  return (a < hi && a + 4 > lo) ? *reinterpret_cast<const uint32_t*>(a) : 0u;
}

// Four bytes starting at byte address g (any alignment) of the range [lo, hi);
// bytes outside the range read as garbage or zero.
__device__ __forceinline__ uint32_t load_4bytes(uintptr_t g, uintptr_t lo, uintptr_t hi) {
  const uintptr_t a = g & ~uintptr_t(3);
  const uint32_t s = uint32_t(g & 3);
  const uint32_t w0 = load_dword_overlapping(a, lo, hi);
  if (s == 0) return w0;
  const uint32_t w1 = load_dword_overlapping(a + 4, lo, hi);
  return __builtin_amdgcn_alignbyte(w1, w0, s);
}

// Changed counts: each workgroup adds its per-pass count into one of
// kCountShards slots, kCountStride uint64 apart (one cache line each), so
// that the per-workgroup atomics of a launch do not all hit one address.
// Pass t's count is the sum of slots [t*kCountSlots + s*kCountStride].
constexpr int kCountShards = 32;
constexpr int kCountStride = 16;
constexpr int kCountSlots = kCountShards * kCountStride;

__device__ __forceinline__ unsigned long long pass_total(const unsigned long long* cnt, int t) {
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < kCountShards; ++k) s += cnt[t * kCountSlots + k * kCountStride];
  return s;
}

// 1 if pass t's count is zero, for a whole wave (every lane active): lane l <
// kCountShards loads shard l, and the count is zero iff no shard is (they
// are non-negative).  One load instruction and a ballot, in place of a
// serial sum over the shards.
__device__ __forceinline__ int pass_zero_wave(const unsigned long long* cnt, int t, int lane) {
  const unsigned long long v = lane < kCountShards ? cnt[t * kCountSlots + lane * kCountStride] : 0ull;
  return __builtin_amdgcn_ballot_w64(v != 0ull) == 0ull ? 1 : 0;
}

// Static XCD-aware schedule: workgroups are dispatched round-robin over the
// 8 XCDs (workgroup b runs on XCD b % 8); XCD x owns a contiguous range of
// tiles (row-major tile order), so vertically adjacent tiles mostly share
// an L2, and its gridDim/8 workgroups stride through that range.
struct TileRange {
  int first, end, stride;
};
__device__ __forceinline__ TileRange xcd_range(int b, int G, int ntiles) {
  const int x = b & 7, j = b >> 3;
  const int q = ntiles >> 3, rr = ntiles & 7;
  const int start = x * q + (x < rr ? x : rr);
  TileRange t;
  t.first = start + j;
  t.end = start + q + (x < rr ? 1 : 0);
  t.stride = G >> 3;
  return t;
}

// ---- the pass kernel ---------------------------------------------------------

// Shared memory of one workgroup of a pass kernel.
template <int BETA, int T, int R, int WAVES>
struct PassSmem {
  static constexpr int BROWS = WAVES * R + 2 * BETA;   // rows per LDS buffer
  uint32_t buf0[BROWS * kRowWords + 1];
  uint32_t buf1[BROWS * kRowWords + 1];
  uint16_t queue[WAVES][kQueueCap];
  uint32_t lanes[WAVES][kLaneQueueCap];
  int left[2 * WAVES];          // per wave: queue head, leftover count (end of a pass)
  unsigned dirty[2];            // bit i: owned row i may change in this pass (one-pass launches)
  unsigned copyin[2];           // bit i: owned row i changed in the previous launch
  unsigned chg[WAVES * R];      // owned row: change bits of this pass (one-pass launches)
  unsigned changed[T];
  unsigned diff2;               // owned pixels that differ from the image two passes before
  // what a tile needs only after its pass (kept here, not in scalar
  // registers, through the pass): this pass's change map and tile lists
  uint8_t* map_out;
  uint32_t* list_state;
  int seq;
  int list_cap;
  int tile_base;                // list index of the image's tile 0 (many images)
};

// After a tile's pass (skipping shapes, from the third launch of a
// sequence on): list the tiles that can change in the next launch -- this
// one if it changed, and each neighbour with a change of this tile within
// BETA of the shared edge or corner.  Lane l of wave 0 handles neighbour
// (l/3 - 1, l%3 - 1).  Called after the tile's stores are issued, so that
// they and the atomics are in flight together; reads sm.chg, which the next
// tile rewrites only after its loads' barrier.
template <int BETA, int T, int R, int WAVES>
__device__ __forceinline__ void mark_next_tiles(PassSmem<BETA, T, R, WAVES>& sm, int tile, int tiles_x,
                                                int rows) {
  constexpr int TH = WAVES * R;   // one pass per launch
  const int lane = threadIdx.x & 63;
  if ((threadIdx.x >> 6) != 0) return;
  uint32_t* const state = sm.list_state;
  const int sq = __builtin_amdgcn_readfirstlane(sm.seq);
  if (state == nullptr) return;
  const uint32_t c = lane < TH ? sm.chg[lane] : 0u;
  const unsigned long long any = __builtin_amdgcn_ballot_w64((c & 1u) != 0u);
  if (any == 0ull) return;   // no change in this tile: nothing to mark
  const unsigned long long lft = __builtin_amdgcn_ballot_w64((c & 2u) != 0u);
  const unsigned long long rgt = __builtin_amdgcn_ballot_w64((c & 4u) != 0u);
  constexpr unsigned long long top = (1ull << BETA) - 1ull;
  constexpr unsigned long long bot = top << (TH - BETA);
  if (lane < 9) {
    const int dy = lane / 3 - 1, dx = lane % 3 - 1;
    unsigned long long m = dx == 0 ? any : (dx < 0 ? lft : rgt);
    if (dy < 0) m &= top;
    if (dy > 0) m &= bot;
    const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
    const int tiles_y = int((uint32_t(rows) + uint32_t(TH - 1)) / uint32_t(TH));   // no int overflow
    const int ny = ty + dy, nx = tx + dx;
    bool fresh = false;
    uint32_t t = 0u;
    if (m != 0ull && ny >= 0 && ny < tiles_y && nx >= 0 && nx < tiles_x) {
      t = uint32_t(__builtin_amdgcn_readfirstlane(sm.tile_base) + ny * tiles_x + nx);
      fresh = atomicExch(TileLists::marks(state) + t, uint32_t(sq + 1)) != uint32_t(sq + 1);
    }
    // one append of all fresh tiles (lanes 0..8 of the wave)
    const unsigned long long fm = __builtin_amdgcn_ballot_w64(fresh);
    if (fm != 0ull) {
      const int cap = __builtin_amdgcn_readfirstlane(sm.list_cap);
      const int l = (sq + 1) % 3, sh = int(blockIdx.x) % kListShards;
      uint32_t at = 0u;
      if (lane == 0) at = atomicAdd(TileLists::count(state, l, sh), uint32_t(__builtin_popcountll(fm)));
      at = __shfl(at, 0);
      // (a list holds each tile once, so it never exceeds cap; bounded
      // anyway against marks left by a sequence that did not start at 0)
      // (a list holds each tile once, so it never exceeds cap; bounded
      // anyway against marks left by a sequence that did not start at 0)
      const uint32_t slot = at + __builtin_amdgcn_mbcnt_lo(uint32_t(fm), 0u);
      if (fresh && slot < uint32_t(cap)) TileLists::shard(state, cap, l, sh)[slot] = t;
    }
  }
}

// Run `npasses` (<= T) passes on tile `tile` of one image: load the tile
// and its halo from `src`, compute, store the owned region to `dst`, and add
// the tile's per-pass changed counts to sm.changed[].  Called by every
// thread of the workgroup; ends with a barrier.
// TRACK: 0 no change maps; 1 change maps, rows that cannot change are copied
// through untested; 2 as 1, and the tiles that can change in the next launch
// are listed; 3 as 2, over the listed tiles only, storing only the rows that
// can change (the destination already holds the rest).  See TileLists.
template <int BETA, int T, int R, int WAVES, int TRACK, bool CYC>
__device__ __forceinline__ void run_tile(PassSmem<BETA, T, R, WAVES>& sm, const uint8_t* src_img,
                                         uint8_t* dst_img, int rows, int cols, int alpha,
                                         int npasses, int tile, int tiles_x,
                                         const uint8_t* map_in, const uint8_t* prev2_img,
                                         int seq) {
  constexpr int NW = 2 * BETA + 1;            // window side
  constexpr int N = NW * NW;                  // window positions
  constexpr int NB = N - 1;                   // neighbours
  constexpr int CROWS = WAVES * R;            // rows computed per pass
  constexpr int BROWS = CROWS + 2 * BETA;     // rows held per LDS buffer
  constexpr int TH = CROWS - 2 * (T - 1) * BETA;  // owned rows
  constexpr int TW = 256 - 2 * (T - 1) * BETA;    // owned columns
  constexpr int COL_OFF = 4 + (T - 1) * BETA;     // LDS byte of owned column 0
  static_assert(BETA >= 1 && BETA <= 4, "halo pads hold at most 4 columns");
  static_assert(TH > 0 && TW > 0, "tile too small for T passes");
  static_assert(NB % 4 == 0, "neighbour count is 4*beta*(beta+1)");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wave index, wave-uniform: row logic and LDS row bases stay scalar
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  uint32_t* buf0 = sm.buf0;
  uint32_t* buf1 = sm.buf1;
  unsigned* s_changed = sm.changed;
  uint16_t* q = sm.queue[w];
  const uintptr_t sb = reinterpret_cast<uintptr_t>(src_img);
  const uintptr_t se = sb + uintptr_t(rows) * uintptr_t(cols);
  const uintptr_t db = reinterpret_cast<uintptr_t>(dst_img);
  const uint32_t am1_16 = uint32_t(alpha > 0 ? alpha - 1 : 0) * 0x01000100u;
  const uint32_t a_16 = uint32_t(alpha) * 0x01000100u;
  const uint32_t ones = 0x01010101u;

  const int ty = tile / tiles_x;
  const int tx = tile - ty * tiles_x;
  const int r0 = ty * TH;
  const int c0 = tx * TW;
  const int row_first = r0 - T * BETA;       // image row of LDS row 0
  const int col_first = c0 - COL_OFF;        // image column of LDS byte 0

  // Rows start on dword boundaries and LDS byte 0 is a dword boundary of
  // the image: loads and stores move whole aligned dwords (uniform test).
  const bool aligned = (COL_OFF % 4 == 0) && ((sb | db) & 3u) == 0 && (cols & 3) == 0;

  // ---- rows that can change (one pass per launch) -------------------------
  // A pixel can change in a pass only if some pixel of its window changed in
  // the previous pass: otherwise the pass sees the same window as the
  // previous one, where the pixel did not change.  The previous pass's change
  // map holds one byte per (image row, tile column): bit 0 a change in the
  // row's segment, bit 1 one within BETA columns of its left end, bit 2 one
  // within BETA columns of its right end.  An owned row is "dirty" if a row
  // within BETA of it changed in this tile column, or near the shared edge
  // of a neighbouring one.  Clean rows are copied through untested.  Wave 0
  // reads the map bytes (own tile column and both neighbours) of tile rows
  // r0-BETA .. r0+TH+BETA-1, one row per lane, right after issuing its tile
  // loads so that both latencies overlap; a ballot gives the rows that
  // changed, and an owned row is dirty if one within BETA of it did.  A map
  // byte carries the launch's sequence position (mod 32) in bits 3-7: a
  // byte of an older pass (a tile that did not run in the previous launch,
  // so changed nothing) reads as no change.
  constexpr bool kTrack = TRACK != 0 && (T == 1);
  constexpr int MROWS = TH + 2 * BETA;                  // map rows read
  constexpr int NCH = (MROWS + 63) / 64;                // lanes' rounds (<= 2)
  static_assert(!kTrack || TH <= 64, "dirty rows are one 64-bit mask");
  static_assert(!kTrack || BETA + TH <= 64, "owned rows' map bytes come from one round");
  const bool track_in = kTrack && map_in != nullptr;
  const uint32_t stamp_in = uint32_t(seq - 1) & 31u;
  auto publish_dirty = [&] {
    if (!kTrack || w != 0) return;
    unsigned long long cm[NCH], cp = 0ull;
#pragma unroll
    for (int h = 0; h < NCH; ++h) cm[h] = 0ull;
    if (track_in) {
      const uint32_t lmask = tx > 0 ? 4u : 0u, rmask = tx + 1 < tiles_x ? 2u : 0u;
      uint32_t v[NCH];
      bool cpy = false;
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        const int i = h * 64 + lane;
        const int rr = r0 - BETA + i;
        v[h] = 0u;
        if (i < MROWS && rr >= 0 && rr < rows) {
          const uint8_t* m = map_in + size_t(rr) * size_t(tiles_x) + size_t(tx);
          auto cur = [&](uint32_t b) { return (b >> 3) == stamp_in ? b : 0u; };
          const uint32_t mc = cur(m[0]);
          const uint32_t ml = lmask ? cur(m[-1]) : 0u;
          const uint32_t mr = rmask ? cur(m[1]) : 0u;
          v[h] = (mc & 1u) | ((ml & lmask) >> 2) | ((mr & rmask) >> 1);
          if (TRACK == 3 && h == 0) cpy = (mc & 1u) != 0u;
        }
      }
#pragma unroll
      for (int h = 0; h < NCH; ++h) cm[h] = __builtin_amdgcn_ballot_w64(v[h] != 0u);
      // map row BETA + i is owned row i: the rows that changed in the
      // previous pass (needed by launches over listed tiles only)
      if (TRACK == 3)
        cp = (__builtin_amdgcn_ballot_w64(cpy) >> BETA) & (TH >= 64 ? ~0ull : ((1ull << TH) - 1ull));
    }
    unsigned long long dm = ~0ull;
    if (track_in) {
      // bit i of dm: some map row r0-BETA+i+k, 0 <= k <= 2*BETA, changed
      dm = 0ull;
#pragma unroll
      for (int k = 0; k <= 2 * BETA; ++k) {
        unsigned long long x = cm[0] >> k;
        if (NCH > 1 && k > 0) x |= cm[NCH - 1] << (64 - k);
        dm |= x;
      }
    }
    if (lane == 0) {
      sm.dirty[0] = uint32_t(dm);
      sm.dirty[1] = uint32_t(dm >> 32);
      if (TRACK == 3) {
        sm.copyin[0] = uint32_t(cp);
        sm.copyin[1] = uint32_t(cp >> 32);
      }
    }
    if (lane < TH) sm.chg[lane] = 0u;
  };

  // ---- the image two passes before (period-2 stop) -----------------------
  // With CYC (one pass per launch), each stored pixel is compared with the
  // same pixel of prev2_img.  When the stores take the aligned dword path
  // and prev2_img is dword aligned, the wave's dwords of prev2_img for its
  // stored rows are loaded here, next to the tile loads, so that their
  // latency is hidden; otherwise they are read at the store.
  constexpr bool kCyc = CYC && (T == 1);
  constexpr int SPW = (TH + WAVES - 1) / WAVES;          // stored rows per wave
  const uintptr_t p2b = reinterpret_cast<uintptr_t>(prev2_img);
  const bool cmp2 = kCyc && prev2_img != nullptr;         // uniform
  const bool pre2 = cmp2 && (COL_OFF % 4 == 0) && ((sb | db | p2b) & 3u) == 0 && (cols & 3) == 0;
  uint32_t p2[kCyc ? SPW : 1];
  auto prefetch_prev2 = [&] {
    if (!kCyc || !pre2) return;
    const __amdgpu_buffer_rsrc_t rs2 = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(prev2_img), 0, int(uint32_t(uint32_t(rows) * uint32_t(cols))),
        kBufferWord3);
    const uint32_t cb = uint32_t(c0) + 4u * uint32_t(lane);
#pragma unroll
    for (int u = 0; u < (kCyc ? SPW : 1); ++u) {
      // rows past the image read as 0 (range check) and are not stored
      const uint32_t r = uint32_t(r0) + uint32_t(w + u * WAVES);
      p2[u] = __builtin_amdgcn_raw_buffer_load_b32(rs2, int(r * uint32_t(cols) + cb), 0, 0);
    }
  };

  // ---- unchanged rows (TRACK == 3) ----------------------------------------
  // Launch j writes pass j+1 into the buffer that holds pass j-1.  An owned
  // row that changed neither in pass j (its map's bit 0) nor in pass j+1 is
  // the same in passes j-1, j and j+1: the destination already holds it, and
  // only the other rows are stored.  (Tiles in which nothing can change do
  // not run at all: see TileLists.)
  constexpr bool kSkip = (TRACK >= 2) && (T == 1);
  static_assert(!kSkip || TH >= 16, "tile lists are sized for at least 16 owned rows");
  constexpr bool kDirtyOnly = (TRACK == 3) && (T == 1);
  const bool skip_mode = kDirtyOnly && track_in;   // uniform

  // ---- load the tile and its halo ----------------------------------------
  // Wave w loads LDS rows w, w+WAVES, ...  All loads of the wave are issued
  // before the first wait.  They are raw buffer loads over the image's
  // dwords, from its first byte rounded down to 4 to its end rounded up to
  // 4: a dword outside that span reads as 0 (hardware range check), so rows
  // above and below the image need no test.  Offsets are taken modulo 2^32.
  // A column outside the image may read a byte of a neighbouring row; such
  // bytes only feed pixels that are never replaced and are never stored.
  const uintptr_t base = sb & ~uintptr_t(3);
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>(base), 0, int(uint32_t(((se + 3) & ~uintptr_t(3)) - base)),
      kBufferWord3);
  const uint32_t head = uint32_t(sb & 3u);      // image byte 0 within the first dword
  if (aligned) {
    // LDS dword d of a row is image dword (r*cols + col_first)/4 + d.
    constexpr int RPW = (BROWS + WAVES - 1) / WAVES;
    uint32_t d0[RPW], d1[RPW];
    const uint32_t lane_b = uint32_t(col_first) + 4u * uint32_t(lane);
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      // (unsigned: halo rows past the last int row wrap, and read as 0)
      const uint32_t r = uint32_t(row_first) + uint32_t(w + u * WAVES);
      const uint32_t off = r * uint32_t(cols) + lane_b;
      d0[u] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(off), 0, 0);
      d1[u] = lane < 2 ? __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(off + 256u), 0, 0) : 0u;
    }
    prefetch_prev2();
    publish_dirty();
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int i = w + u * WAVES;
      if (i < BROWS) {
        buf0[i * kRowWords + lane] = d0[u];
        if (lane < 2) buf0[i * kRowWords + 64 + lane] = d1[u];
      }
    }
  } else {
    // For a row, lane l reads the aligned dword l of the row's byte range
    // (and lanes 0-2 dwords 64-66); LDS dword d is re-aligned from aligned
    // dwords d and d+1, the latter taken from the next lane.
    constexpr int RPW = (BROWS + WAVES - 1) / WAVES;
    uint32_t d0[RPW], d1[RPW];
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const uint32_t r = uint32_t(row_first) + uint32_t(w + u * WAVES);
      const uint32_t g = head + r * uint32_t(cols) + uint32_t(col_first);
      const uint32_t a0 = (g & ~3u) + 4u * uint32_t(lane);
      d0[u] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(a0), 0, 0);
      d1[u] = lane < 3 ? __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(a0 + 256u), 0, 0) : 0u;
    }
    prefetch_prev2();
    publish_dirty();
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int i = w + u * WAVES;
      if (i < BROWS) {
        const uint32_t r = uint32_t(row_first) + uint32_t(i);
        const uint32_t sh = (head + r * uint32_t(cols) + uint32_t(col_first)) & 3u;
        const uint32_t nx0 = __shfl_down(d0[u], 1);          // aligned dword lane+1
        const uint32_t x64 = __shfl(d1[u], 0);               // aligned dword 64
        const uint32_t hi = (lane == 63) ? x64 : nx0;
        buf0[i * kRowWords + lane] = __builtin_amdgcn_alignbyte(hi, d0[u], sh);
        const uint32_t nx1 = __shfl_down(d1[u], 1);          // dwords 65, 66 for lanes 0, 1
        if (lane < 2)
          buf0[i * kRowWords + 64 + lane] = __builtin_amdgcn_alignbyte(nx1, d1[u], sh);
      }
    }
  }
  __syncthreads();

  // Columns outside the border frame, per byte of the lane's dword (bit 7).
  uint32_t colmask = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = col_first + 4 + 4 * lane + b;
    if (c >= BETA && c < cols - BETA) colmask |= 0x80u << (8 * b);
  }

  uint32_t* src = buf0;
  uint32_t* dst = buf1;
  for (int t = 0; t < npasses; ++t) {
    const uint8_t* srcb = reinterpret_cast<const uint8_t*>(src);
    uint8_t* dstb = reinterpret_cast<uint8_t*>(dst);
    unsigned wave_changed = 0;
    int qhead = 0, qtail = 0;     // pixel queue q
    int dhead = 0, dtail = 0;     // lane queue dq
    // dirty owned rows (one-pass launches; published before the load barrier)
    unsigned long long dirty_rows = ~0ull;
    if (kTrack)
      dirty_rows = (uint64_t(__builtin_amdgcn_readfirstlane(sm.dirty[1])) << 32) |
                   uint64_t(__builtin_amdgcn_readfirstlane(sm.dirty[0]));

    // Exact evaluation of queued candidates, one lane each.  For the
    // candidate x at LDS (bc, bb), each window row is read as aligned dwords
    // and handled 4 bytes at a time: the band test as in the dense pass,
    // outside bytes masked, sum of their squares by v_dot4_u32_u8, their
    // count by v_bcnt_u32_b32.  Then Algorithm 2's test flag > N-3 and the
    // root mean square floor(sqrt(floor(S/F))).
    // A queue entry is (row within the tile's computed rows) << 8 | byte
    // within the row, so any wave can evaluate it.
    auto evaluate = [&](bool valid, unsigned e) {
      constexpr int NG = (NW + 3) / 4;          // 4-byte groups per window row
      bool ch = false;
      int crow = 0;                             // owned row of the pixel
      unsigned cbits = 0u;                      // its change-map bits
      if (valid) {
        const int bc = int(e >> 8) + BETA;           // LDS row of the pixel
        const int bb = 4 + int(e & 255u);            // LDS byte of the pixel
        const uint32_t x = srcb[bc * kRowBytes + bb];
        uint32_t nlo4 = 0, nhi4 = 0;
        if (alpha > 0) {
          const uint32_t nx4 = ~(x * 0x01010101u);
          nlo4 = sat_add_u8x4(nx4, am1_16);
          nhi4 = sat_sub_u8x4(nx4, a_16);
        }
        uint32_t S = 0, F = 0;
#pragma unroll
        for (int dr = -BETA; dr <= BETA; ++dr) {
          const int A = (bc + dr) * kRowBytes + bb - BETA;   // first byte of the window row
          const uint32_t* wp = src + (A >> 2);
          const uint32_t sh = uint32_t(A) & 3u;
          uint32_t wd[NG + 1];
#pragma unroll
          for (int g = 0; g <= NG; ++g) wd[g] = wp[g];
#pragma unroll
          for (int g = 0; g < NG; ++g) {
            const uint32_t grp = __builtin_amdgcn_alignbyte(wd[g + 1], wd[g], sh);
            const int nvalid = (NW - 4 * g) < 4 ? (NW - 4 * g) : 4;
            const uint32_t vm7 = 0x80808080u >> (8 * (4 - nvalid));
            uint32_t in7 = 0;
            if (alpha > 0)
              in7 = __builtin_amdgcn_lerp(grp, nlo4, ones) ^ __builtin_amdgcn_lerp(grp, nhi4, 0u);
            const uint32_t out7 = vm7 & ~in7;
            const uint32_t outfull = (out7 << 1) - (out7 >> 7);   // 0xFF per outside byte
            S = __builtin_amdgcn_udot4(grp & outfull, grp, S, false);
            F += uint32_t(__builtin_popcount(out7));
          }
        }
        uint32_t v = x;
        if (F > uint32_t(N - 3)) v = isqrt_small(udiv_small(S, F));
        dstb[bc * kRowBytes + bb] = uint8_t(v);
        const int r = row_first + bc;
        const int c = col_first + bb;
        const bool owned = bc >= T * BETA && bc < T * BETA + TH && bb >= COL_OFF &&
                           bb < COL_OFF + TW && r < rows && c < cols;
        ch = owned && (v != x);
        if (kTrack) {
          crow = bc - T * BETA;
          cbits = 1u | (bb - COL_OFF < BETA ? 2u : 0u) | (bb - COL_OFF >= TW - BETA ? 4u : 0u);
        }
      }
      const unsigned long long chm = __builtin_amdgcn_ballot_w64(ch);
      wave_changed += __builtin_popcountll(chm);
      if (kTrack) {
        // this pass's change bits, one LDS update per distinct row (the
        // entries of a round span few rows; per-lane atomics on one row
        // word would serialise)
        unsigned long long pend = chm;
        while (pend != 0ull) {
          const int l0 = __builtin_ctzll(pend);
          const int row0 = __builtin_amdgcn_readlane(crow, l0);
          const bool mine = ch && crow == row0;
          const unsigned long long same = __builtin_amdgcn_ballot_w64(mine);
          const unsigned bits = 1u | (__builtin_amdgcn_ballot_w64(mine && (cbits & 2u)) ? 2u : 0u) |
                                (__builtin_amdgcn_ballot_w64(mine && (cbits & 4u)) ? 4u : 0u);
          if (lane == l0) atomicOr(&sm.chg[row0], bits);
          pend &= ~same;
        }
      }
    };

    // Candidates are queued in two steps.  A row appends one entry per lane
    // that has candidates: its candidate bits (bit 7 of each byte) with the
    // lane in bits 0-5 and the row within the tile in bits 8-13.  Groups of
    // up to 64 such entries are expanded into one pixel entry per candidate:
    // a lane entry has c <= 4 candidates, and the offset of its first pixel
    // entry is the exclusive prefix sum of c over lower lanes, from ballots
    // of the three bits of c.
    uint32_t* dq = sm.lanes[w];
    auto sync_wave = [] {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto expand = [&](int n) {
      const uint32_t e = lane < n ? dq[(dhead + lane) & (kLaneQueueCap - 1)] : 0u;
      const uint32_t c = uint32_t(__builtin_popcount(e & 0x80808080u));
      const unsigned long long b0 = __builtin_amdgcn_ballot_w64(c & 1u);
      const unsigned long long b1 = __builtin_amdgcn_ballot_w64(c & 2u);
      const unsigned long long b2 = __builtin_amdgcn_ballot_w64(c & 4u);
      auto below = [](unsigned long long b) {
        return __builtin_amdgcn_mbcnt_hi(uint32_t(b >> 32),
                                         __builtin_amdgcn_mbcnt_lo(uint32_t(b), 0u));
      };
      int pos = qtail + int(below(b0) + 2 * below(b1) + 4 * below(b2));
      const uint32_t ent = (e & 0x3F00u) | ((e & 63u) << 2);   // row << 8 | first byte
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if ((e >> (8 * b + 7)) & 1u) {
          q[pos & (kQueueCap - 1)] = uint16_t(ent + b);
          ++pos;
        }
      }
      qtail += __builtin_popcountll(b0) + 2 * __builtin_popcountll(b1) +
               4 * __builtin_popcountll(b2);
      dhead += n;
      sync_wave();
      while (qtail - qhead >= 64) {
        evaluate(true, q[(qhead + lane) & (kQueueCap - 1)]);
        qhead += 64;
      }
    };

    // Register window: win[slot][dc+BETA] holds, for the LDS row in that
    // slot, the 4 bytes at columns (lane's 4 pixels) + dc.
    uint32_t win[NW][NW];
    auto load_row = [&](int i, uint32_t (&wr)[NW]) {
      const uint32_t* rp = src + (w * R + i) * kRowWords + lane;
      const uint32_t L = rp[0], C = rp[1], Rr = rp[2];
#pragma unroll
      for (int dc = -BETA; dc <= BETA; ++dc) {
        if (dc < 0)
          wr[dc + BETA] = (dc == -4) ? L : __builtin_amdgcn_alignbyte(C, L, 4 + dc);
        else if (dc == 0)
          wr[BETA] = C;
        else
          wr[dc + BETA] = (dc == 4) ? Rr : __builtin_amdgcn_alignbyte(Rr, C, dc);
      }
    };

#pragma unroll
    for (int i = 0; i < 2 * BETA; ++i) load_row(i, win[i]);

#pragma unroll 1
    for (int j0 = 0; j0 < R; j0 += NW) {
#pragma unroll
      for (int jj = 0; jj < NW; ++jj) {
        const int jc = j0 + jj;               // centre row within the strip
        if (jc < R) {
          load_row(jc + 2 * BETA, win[(jj + 2 * BETA) % NW]);
          const int bc = w * R + jc + BETA;   // LDS row of the centre
          const int r = row_first + bc;
          const uint32_t X = win[(jj + BETA) % NW][BETA];
          // Row r is interior or not, and dirty or not, for the whole wave.
          bool test = (r >= BETA) && (r < rows - BETA);
          if (kTrack) test = test && ((dirty_rows >> (w * R + jc)) & 1ull) != 0ull;
          uint32_t cand = test ? colmask : 0u;
          if (test && alpha > 0) {
            const uint32_t nx = ~X;
            const uint32_t nlo = sat_add_u8x4(nx, am1_16);   // 255 - max(x-alpha+1, 0)
            const uint32_t nhi = sat_sub_u8x4(nx, a_16);     // 255 - min(x+alpha, 255)
            uint32_t t1 = 0, t2 = 0;
            // neighbours 4g .. 4g+3 in ring order into the counters
            auto group = [&](int g) {
              uint32_t m[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                int dr = 0, dc = 0;
                ring_offset(4 * g + u, dr, dc);
                const uint32_t Y = win[(jj + BETA + dr + NW) % NW][dc + BETA];
                const uint32_t A = __builtin_amdgcn_lerp(Y, nlo, ones);
                const uint32_t B = __builtin_amdgcn_lerp(Y, nhi, 0u);
                m[u] = A ^ B;
              }
              const uint32_t cg = bitop3_maj(m[0], m[1], m[2]);
              const uint32_t sg = bitop3_xor3(m[0], m[1], m[2]);
              const uint32_t ug = bitop3_maj(t1, sg, m[3]);
              t2 = bitop3_or3(t2, cg, ug);
              t1 = bitop3_or3(t1, sg, m[3]);
            };
            // "At least two neighbours in the band" can only become true as
            // neighbours are added, so once it holds for every pixel of the
            // wave's row that could be replaced, the outer neighbours cannot
            // change the outcome and are skipped (wave-uniform branch).
            group(0);                                   // 4-connected
            cand = colmask & ~t2;
            bool more = __builtin_amdgcn_ballot_w64(cand != 0u) != 0ull;
            if (more) {
              group(1);                                 // diagonals
              cand = colmask & ~t2;
              more = __builtin_amdgcn_ballot_w64(cand != 0u) != 0ull;
            }
#pragma unroll
            for (int d = 2; d <= BETA; ++d) {           // ring d: groups d(d-1) .. d(d+1)-1
              if (more) {
#pragma unroll
                for (int g = d * (d - 1); g < d * (d + 1); ++g) group(g);
                cand = colmask & ~t2;
                if (d < BETA) more = __builtin_amdgcn_ballot_w64(cand != 0u) != 0ull;
              }
            }
          }
          dst[bc * kRowWords + 1 + lane] = X;   // copy-through; candidates patched below
          const unsigned long long hb = __builtin_amdgcn_ballot_w64(cand != 0u);
          if (hb != 0ull) {
            const int pos = dtail + int(__builtin_amdgcn_mbcnt_hi(
                                        uint32_t(hb >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(hb), 0u)));
            if (cand != 0u)
              dq[pos & (kLaneQueueCap - 1)] =
                  cand | uint32_t(lane) | (uint32_t(w * R + jc) << 8);
            dtail += __builtin_popcountll(hb);
            if (dtail - dhead >= 64) {
              sync_wave();
              expand(64);
            }
          }
        }
      }
    }
    if (dtail > dhead) {
      sync_wave();
      expand(dtail - dhead);
    }
    // Leftovers (fewer than 64 per wave) are evaluated together once every
    // wave has finished its rows, 64 per wave: the copy-through writes of
    // all rows are then done, so no result can be overwritten.
    if (lane == 0) {
      sm.left[2 * w] = qhead;
      sm.left[2 * w + 1] = qtail - qhead;
    }
    __syncthreads();
    {
      int pre[WAVES + 1];
      pre[0] = 0;
#pragma unroll
      for (int k = 0; k < WAVES; ++k)
        pre[k + 1] = pre[k] + __builtin_amdgcn_readfirstlane(sm.left[2 * k + 1]);
      for (int c = w; c * 64 < pre[WAVES]; c += WAVES) {
        const int g = c * 64 + lane;           // index in the waves' leftovers, in wave order
        int ww = 0, first = 0;
#pragma unroll
        for (int k = 1; k < WAVES; ++k)
          if (g >= pre[k]) { ww = k; first = pre[k]; }
        const int idx = (sm.left[2 * ww] + g - first) & (kQueueCap - 1);
        evaluate(g < pre[WAVES], sm.queue[ww][idx]);
      }
    }
    if (lane == 0 && wave_changed != 0u) atomicAdd(&s_changed[t], wave_changed);
    __syncthreads();
    uint32_t* tmp = src;
    src = dst;
    dst = tmp;
  }

  // This launch's change map (the pass loop ended with a barrier), stamped.
  uint8_t* const map_out = kTrack ? sm.map_out : nullptr;
  if (kTrack && map_out != nullptr && tid < TH && r0 + tid < rows)
    map_out[size_t(r0 + tid) * size_t(tiles_x) + size_t(tx)] =
        uint8_t(sm.chg[tid] | ((uint32_t(sm.seq) & 31u) << 3));
  // (the launch that builds the first lists marks before its stores; see
  // the end of this function)
  if constexpr (kSkip && !kDirtyOnly) mark_next_tiles(sm, tile, tiles_x, rows);

  // ---- store the owned region ----------------------------------------------
  // (skip mode: only the rows that changed in the previous launch or in
  // this one, read back from LDS rather than kept in registers through the
  // passes)
  unsigned long long put_rows = ~0ull;
  if (kSkip && skip_mode)
    put_rows = __builtin_amdgcn_ballot_w64(lane < TH && (sm.chg[lane < TH ? lane : 0] & 1u) != 0u) |
               (uint64_t(__builtin_amdgcn_readfirstlane(sm.copyin[1])) << 32) |
               uint64_t(__builtin_amdgcn_readfirstlane(sm.copyin[0]));
  // With prev2_img (CYC), each stored pixel is first compared with the same
  // pixel of the image two passes before; that image may be the destination
  // itself, so it is read before the store (prefetched above, or here), by
  // the thread that stores the pixel.  (Skip mode: a row not stored holds
  // the same bytes two passes before, so it adds no difference; a tile not
  // listed neither.)
  unsigned ndiff = 0;
  if (kCyc && pre2) {
    // as the aligned path below, with the prefetched dwords of prev2_img
    uint32_t* d32 = reinterpret_cast<uint32_t*>(dst_img);
    const int c = c0 + 4 * lane;
    const bool cok = (4 * lane < TW) && (c < cols);
#pragma unroll
    for (int u = 0; u < (kCyc ? SPW : 1); ++u) {
      const int i = w + u * WAVES;
      const int r = r0 + i;
      if (i >= TH || r >= rows) break;
      if (skip_mode && ((put_rows >> i) & 1ull) == 0ull) continue;   // unchanged row (uniform)
      if (cok) {
        const int idx = (r * cols + c) >> 2;
        const uint32_t nv = src[(T * BETA + i) * kRowWords + (COL_OFF >> 2) + lane];
        // bytes that differ: bit 7 of ((x & 0x7f..) + 0x7f..) | x is set iff
        // the byte of x is nonzero (no carry leaves a byte)
        const uint32_t x = p2[u] ^ nv;
        ndiff += __builtin_popcount((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u);
        d32[idx] = nv;
      }
    }
  } else if (aligned && (!cmp2 || (p2b & 3u) == 0)) {
    // lane l stores owned dword l of each owned row
    uint32_t* d32 = reinterpret_cast<uint32_t*>(dst_img);
    const uint32_t* p32 = reinterpret_cast<const uint32_t*>(prev2_img);
    const int c = c0 + 4 * lane;
    const bool cok = (4 * lane < TW) && (c < cols);
#pragma unroll 4
    for (int i = w; i < TH; i += WAVES) {
      const int r = r0 + i;
      if (r >= rows) break;
      if (skip_mode && ((put_rows >> i) & 1ull) == 0ull) continue;   // unchanged row (uniform)
      if (cok) {
        const int idx = (r * cols + c) >> 2;
        const uint32_t nv = src[(T * BETA + i) * kRowWords + (COL_OFF >> 2) + lane];
        if (cmp2) {
          // bytes that differ: bit 7 of ((x & 0x7f..) + 0x7f..) | x is set iff
          // the byte of x is nonzero (no carry leaves a byte)
          const uint32_t x = p32[idx] ^ nv;
          ndiff += __builtin_popcount((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u);
        }
        d32[idx] = nv;
      }
    }
  } else {
    const uint8_t* fin = reinterpret_cast<const uint8_t*>(src);
    const int len = (cols - c0) < TW ? (cols - c0) : TW;
#pragma unroll 4
    for (int i = w; i < TH; i += WAVES) {
      const int r = r0 + i;
      if (r >= rows) break;
      if (skip_mode && ((put_rows >> i) & 1ull) == 0ull) continue;   // unchanged row (uniform)
      const uintptr_t g = db + uintptr_t(r) * uintptr_t(cols) + uintptr_t(c0);
      const uintptr_t ge = g + uintptr_t(len);
      const uintptr_t a0 = g & ~uintptr_t(3);
      const int lrow = (T * BETA + i) * kRowBytes + COL_OFF;   // LDS byte of column c0
      for (int qd = lane; qd < 65; qd += 64) {
        const uintptr_t ad = a0 + 4u * uintptr_t(qd);
        if (ad >= ge) continue;
        if (ad >= g && ad + 4 <= ge) {
          const int off = lrow + int(ad - g);
          const uint32_t lo = src[off >> 2];
          const uint32_t v =
              (off & 3) ? __builtin_amdgcn_alignbyte(src[(off >> 2) + 1], lo, off & 3) : lo;
          if (cmp2) {
            const uint8_t* o = prev2_img + (ad - db);
#pragma unroll
            for (int b = 0; b < 4; ++b) ndiff += uint32_t(o[b]) != ((v >> (8 * b)) & 0xffu);
          }
          *reinterpret_cast<uint32_t*>(ad) = v;
        } else {
          const uintptr_t pb = ad > g ? ad : g;
          const uintptr_t pe = (ad + 4) < ge ? (ad + 4) : ge;
          for (uintptr_t p = pb; p < pe; ++p) {
            const uint8_t nv = fin[lrow + int(p - g)];
            if (cmp2) ndiff += prev2_img[p - db] != nv;
            *reinterpret_cast<uint8_t*>(p) = nv;
          }
        }
      }
    }
  }
  if (cmp2) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ndiff += __shfl_down(ndiff, off);
    if (lane == 0 && ndiff != 0u) atomicAdd(&sm.diff2, ndiff);
  }
  // The tiles of the next launch, marked once the stores are issued: the
  // marks' atomics and the stores are in flight together.  (Launches over
  // listed tiles only: in the one over every tile, which keeps many tiles
  // in flight per CU anyway, marking here costs registers the kernel does
  // not have to spare.)
  if constexpr (kSkip && kDirtyOnly) mark_next_tiles(sm, tile, tiles_x, rows);
  // The next tile's load overwrites buf0, which the store above reads.
  __syncthreads();
}

// Minimum waves per SIMD asked of the register allocator: beta = 2 with 8
// rows per wave and 2 or more waves per group fits 6 (at most 80 VGPRs, no
// spills; LDS allows 6 groups); the list-keeping kernels fit 5.
template <int BETA, int R, int WAVES, int TRACK = 0>
constexpr int min_waves_per_simd() {
  return (BETA == 2 && R <= 8 && WAVES >= 2) ? (TRACK >= 2 ? 5 : 6) : 1;
}

// Single image: tiles of one image, up to T passes per launch; with TRACK
// (one-pass shapes) the launch reads and writes change maps.
template <int BETA, int T, int R, int WAVES, int TRACK = 0, bool CYC = false>
__global__ __launch_bounds__(WAVES * 64, (min_waves_per_simd<BETA, R, WAVES, TRACK>())) void pass_kernel(PassArgs a) {
  __shared__ PassSmem<BETA, T, R, WAVES> sm;
  const int tid = threadIdx.x;
  // A launch after convergence does nothing: if a pass of the previous
  // launch changed no pixel, the image is a fixed point and the remaining
  // passes are no-ops.  (A skipped launch leaves its counts at zero, so the
  // next launch skips too.)  With the period-2 stop (diff2, one pass per
  // launch), a previous pass whose image equals the image two passes before
  // it also ends the run.  Every wave reads the counts of the previous
  // launch itself (they do not change during this one), so all of them
  // take the same decision before any tile load, with no barrier.
  // (A listed launch issues the loads of its list's count and first entry
  // here too, so that their latency overlaps the vote's.)
  constexpr bool kListed = TRACK == 3 && T == 1;
  const int G = gridDim.x;
  const int lq = int(blockIdx.x) / kListShards;
  const int lsh = (int(blockIdx.x) + int(blockIdx.x) / kListRound) % kListShards;
  uint32_t ln = 0u, lfirst = 0u;
  if (kListed) {
    uint32_t* ls = a.list_state;
    const int cur = a.seq % 3;
    ln = *TileLists::count(ls, cur, lsh);
    lfirst = lq < a.list_cap ? TileLists::shard(ls, a.list_cap, cur, lsh)[lq] : 0u;
  }
  int zw = 0;
  if (a.pass0 > 0)
#pragma unroll
    for (int u = 0; u < T; ++u) zw |= pass_zero_wave(a.changed, a.pass0 - T + u, tid & 63);
  if (CYC && T == 1 && a.diff2 != nullptr && a.pass0 >= 2)
    zw |= pass_zero_wave(a.diff2, a.pass0 - 1, tid & 63);
  if (zw) return;
  if (tid < T) sm.changed[tid] = 0;
  if (CYC && tid == 0) sm.diff2 = 0u;
  if (tid == 0) {
    // read after the tile's pass, behind its barriers
    sm.map_out = a.map_out;
    sm.list_state = a.list_state;
    sm.seq = a.seq;
    sm.list_cap = a.list_cap;
    sm.tile_base = 0;
  }
  constexpr bool kMarks = TRACK >= 2 && T == 1;
  uint32_t* ms = kMarks ? a.list_state : nullptr;
  auto one = [&](int tile) {
    run_tile<BETA, T, R, WAVES, TRACK, CYC>(sm, a.src, a.dst, a.rows, a.cols, a.alpha, a.npasses,
                                            tile, a.tiles_x, a.map_in, CYC ? a.prev2 : nullptr,
                                            a.seq);
  };
  // the counts of the list the launch after the next fills
  if (kMarks && ms != nullptr && blockIdx.x == 0 && tid < kListShards)
    *TileLists::count(ms, (a.seq + 2) % 3, tid) = 0u;
  if constexpr (kListed) {
    // The tiles the previous launch listed for this one (no other tile can
    // change, and the destination already holds them).  Workgroups come in
    // groups of kListShards consecutive indices; group q takes entry q of
    // every shard, one shard per workgroup, then entries q + G/kListShards,
    // ...  The shard of a workgroup rotates by one every kListRound
    // workgroups: on a device with kListRound CUs, workgroups b and
    // b + kListRound are dispatched to the same CU, and the rotation gives
    // each CU entries of several shards (shards differ in length) so that
    // the busy workgroups spread evenly.  The grid is a multiple of
    // kListShards (several times the resident one: see the host's grid
    // choice); the list is not written in this launch, so every wave takes
    // the same tiles.
    // (Counts and entries are bounded again here: a sequence that did not
    // start at launch 0 has no lists, only whatever its memory held.)
    const int gs = G / kListShards;                              // workgroups per shard
    const uint32_t* lst = TileLists::shard(ms, a.list_cap, a.seq % 3, lsh);
    const int n = min(int(__builtin_amdgcn_readfirstlane(ln)), a.list_cap);
    const int first = int(__builtin_amdgcn_readfirstlane(lfirst));
    if (lq < gs)
      for (int j = lq; j < n; j += gs) {
        const unsigned tile = unsigned(j == lq ? first : int(__builtin_amdgcn_readfirstlane(lst[j])));
        if (tile < unsigned(a.ntiles)) one(int(tile));
      }
  } else {
    const TileRange tr = xcd_range(blockIdx.x, gridDim.x, a.ntiles);
    for (int tile = tr.first; tile < tr.end; tile += tr.stride) one(tile);
  }
  const int shard = (blockIdx.x % kCountShards) * kCountStride;
  if (tid < a.npasses && sm.changed[tid] != 0u)
    atomicAdd(a.changed + (a.pass0 + tid) * kCountSlots + shard, (unsigned long long)sm.changed[tid]);
  if (CYC && T == 1 && tid == 0 && a.diff2 != nullptr && a.prev2 != nullptr && sm.diff2 != 0u)
    atomicAdd(a.diff2 + a.pass0 * kCountSlots + shard, (unsigned long long)sm.diff2);
}

// ---- many images per launch ------------------------------------------------------

// One image of a multi-image launch.
struct ImageDesc {
  const uint8_t* src;            // image before this launch
  uint8_t* dst;                  // image after this launch
  unsigned long long* counts;    // the image's count slots (kCountSlots per pass)
  int rows, cols, alpha;
  int pass0;                     // the image's index of this launch's first pass
  int npasses;                   // passes for this image in this launch (0: idle)
  int prev_passes;               // passes of its previous launch (0: none)
  int tiles_x;
  int pad;
  int* status;                   // or null: set to 1 if the image had converged before
                                 // this launch (its previous launch had a pass with no
                                 // change), else 0; written by the workgroup of tile 0
  // change maps of the image (one-pass launches of a tracking kernel, else
  // null): the previous launch's, this launch's, and the launch's position
  // in the image's sequence (the maps' stamp)
  const uint8_t* map_in;
  uint8_t* map_out;
  int seq;
  int tile_base;                 // index of the image's tile 0 in the tile table
};

// One tile of a multi-image launch: image index and tile index within it.
struct TileRef {
  int image;
  int tile;
};

struct MultiArgs {
  const ImageDesc* images;
  const TileRef* tiles;
  int ntiles;
  int seq;                       // launch index (skipping kernels: the lists' rotation)
  uint32_t* list_state;          // skipping kernels: the group's TileLists (entries index
  int list_cap;                  // `tiles`), capacity ntiles; else null
};

// Many images, one tile per workgroup (a static tile table in place of a
// work queue: no atomics to hand out work).  Each image keeps its own
// parameters, pass index, pass count and convergence state.
// TRACK (one pass per launch), as in the single-image kernel: 1 each image
// keeps change maps (rows that cannot change are copied through untested);
// 2 also lists the tiles that can change in the next launch, in one set of
// lists for all the images of the launch (entries index the tile table);
// 3 as 2, over the listed tiles only.
template <int BETA, int T, int R, int WAVES, int TRACK = 0>
__global__ __launch_bounds__(WAVES * 64, (min_waves_per_simd<BETA, R, WAVES, TRACK>())) void multi_pass_kernel(MultiArgs a) {
  static_assert(TRACK == 0 || T == 1, "many images: change maps of one-pass launches only");
  __shared__ PassSmem<BETA, T, R, WAVES> sm;
  const int tid = threadIdx.x;
  constexpr bool kMarks = TRACK >= 2;
  constexpr bool kListed = TRACK == 3;
  if (kMarks && tid == 0) {
    // read after a tile's pass, behind its barriers
    sm.list_state = a.list_state;
    sm.list_cap = a.list_cap;
  }
  // the counts of the list the launch after the next fills
  if (kMarks && blockIdx.x == 0 && tid < kListShards)
    *TileLists::count(a.list_state, (a.seq + 2) % 3, tid) = 0u;
  auto one = [&](int t) {
    const TileRef ref = a.tiles[t];
    const ImageDesc d = a.images[ref.image];
    if (d.npasses <= 0) return;   // uniform: the whole workgroup reads the same entry
    // Convergence of this image, before any of its tile loads: every wave
    // reads the counts of the image's previous launch (unchanged during
    // this one), so all take the same decision (uniform loop bound: the
    // descriptor is).
    int zw = 0;
    for (int u = 0; u < d.prev_passes; ++u)
      zw |= pass_zero_wave(d.counts, d.pass0 - d.prev_passes + u, tid & 63);
    if (ref.tile == 0 && tid == 0 && d.status != nullptr) *d.status = zw ? 1 : 0;
    if (zw) return;   // this image has converged
    if (tid < T) sm.changed[tid] = 0;
    if (TRACK && tid == 0) {
      // read after the tile's pass, behind its barriers (the previous
      // tile's reads ended at its closing barrier)
      sm.map_out = d.map_out;
      sm.seq = d.seq;
      sm.tile_base = d.tile_base;
    }
    run_tile<BETA, T, R, WAVES, TRACK, false>(sm, d.src, d.dst, d.rows, d.cols, d.alpha, d.npasses,
                                              ref.tile, d.tiles_x, TRACK ? d.map_in : nullptr,
                                              nullptr, d.seq);
    if (tid < d.npasses && sm.changed[tid] != 0u)
      atomicAdd(d.counts + (d.pass0 + tid) * kCountSlots + (blockIdx.x % kCountShards) * kCountStride,
                (unsigned long long)sm.changed[tid]);
  };
  if constexpr (kListed) {
    // the entries the previous launch listed, handed out as in the
    // single-image listed launch (a grid that is a multiple of kListShards)
    const int gs = int(gridDim.x) / kListShards;
    const int lq = int(blockIdx.x) / kListShards;
    const int lsh = (int(blockIdx.x) + int(blockIdx.x) / kListRound) % kListShards;
    const uint32_t* lst = TileLists::shard(a.list_state, a.list_cap, a.seq % 3, lsh);
    const int n = min(int(__builtin_amdgcn_readfirstlane(*TileLists::count(a.list_state, a.seq % 3, lsh))),
                      a.list_cap);
    if (lq < gs)
      for (int j = lq; j < n; j += gs) {
        const unsigned t = __builtin_amdgcn_readfirstlane(lst[j]);
        if (t < unsigned(a.ntiles)) one(int(t));
      }
  } else {
    const TileRange tr = xcd_range(blockIdx.x, gridDim.x, a.ntiles);
    for (int t = tr.first; t < tr.end; t += tr.stride) one(t);
  }
}

// ---- small kernels -------------------------------------------------------------

// Zero n uint64 values.
[[maybe_unused]] static __global__ void zero_u64_kernel(unsigned long long* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Zero two ranges of uint64 values (n2 may be 0).
[[maybe_unused]] static __global__ void zero2_u64_kernel(unsigned long long* p1, long long n1,
                                                         unsigned long long* p2, long long n2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n1 + n2;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < n1) p1[i] = 0ull;
    else p2[i - n1] = 0ull;
  }
}

// Copy n bytes, any alignment of either pointer; ranges must not overlap.
// When both pointers have the same offset within 16 bytes, the aligned
// middle moves as 16-byte vectors and the ends as bytes; otherwise each
// thread writes whole aligned destination dwords (bytes at the ends).
__device__ __forceinline__ void copy_range(const uint8_t* s, uint8_t* d, long long n) {
  const uintptr_t sb = reinterpret_cast<uintptr_t>(s);
  const uintptr_t db = reinterpret_cast<uintptr_t>(d);
  const long long gtid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long gstride = (long long)gridDim.x * blockDim.x;
  if (((sb ^ db) & 15u) == 0) {
    const long long head = (long long)((16u - (db & 15u)) & 15u) < n
                               ? (long long)((16u - (db & 15u)) & 15u) : n;
    const long long nv = (n - head) / 16;
    for (long long i = gtid; i < head; i += gstride) d[i] = s[i];
    const uint4* sv = reinterpret_cast<const uint4*>(s + head);
    uint4* dv = reinterpret_cast<uint4*>(d + head);
    for (long long i = gtid; i < nv; i += gstride) dv[i] = sv[i];
    for (long long i = head + nv * 16 + gtid; i < n; i += gstride) d[i] = s[i];
    return;
  }
  const uintptr_t de = db + uintptr_t(n);
  const uintptr_t a0 = db & ~uintptr_t(3);
  const long long nd = (long long)((de - a0 + 3) >> 2);
  for (long long qd = blockIdx.x * (long long)blockDim.x + threadIdx.x; qd < nd;
       qd += (long long)gridDim.x * blockDim.x) {
    const uintptr_t ad = a0 + 4u * uintptr_t(qd);
    if (ad >= db && ad + 4 <= de) {
      *reinterpret_cast<uint32_t*>(ad) = load_4bytes(sb + (ad - db), sb, sb + uintptr_t(n));
    } else {
      const uintptr_t pb = ad > db ? ad : db;
      const uintptr_t pe = (ad + 4) < de ? (ad + 4) : de;
      for (uintptr_t p = pb; p < pe; ++p) *reinterpret_cast<uint8_t*>(p) = s[p - db];
    }
  }
}

[[maybe_unused]] static __global__ void copy_bytes_kernel(const uint8_t* __restrict__ s, uint8_t* __restrict__ d,
                                  long long n) {
  copy_range(s, d, n);
}

struct FinishArgs {
  const unsigned long long* counts;  // per-pass shard slots (kCountSlots per pass)
  const unsigned long long* diff2;   // period-2 stop: pixels differing from two passes
                                     // before, same layout (one pass per launch), or null
  unsigned long long* changed;       // out: per-pass totals, k entries (may be null)
  int k;            // passes requested
  int T;            // passes per launch
  int launches;     // launches enqueued
  const uint8_t* buf_even_from_end;  // dst of launches j with (launches-1-j) even
  const uint8_t* buf_odd_from_end;   // dst of launches j with (launches-1-j) odd
  const uint8_t* first_src;          // image when no launch ran
  uint8_t* out;
  long long n;
  int* iterations;  // may be null
};

// Decide, from changed[], how many passes and launches ran, and move the
// final image to `out` if it is elsewhere.
[[maybe_unused]] static __global__ void finish_kernel(FinishArgs f) {
  __shared__ int s_first_zero;
  if (threadIdx.x == 0) s_first_zero = f.k;
  __syncthreads();
  for (int t = threadIdx.x; t < f.k; t += blockDim.x) {
    const unsigned long long tot = pass_total(f.counts, t);
    if (blockIdx.x == 0 && f.changed) f.changed[t] = tot;
    // a pass that changed nothing, or (period-2 stop, t >= 1) whose image
    // equals the image two passes before, is the last one
    if (tot == 0ull || (f.diff2 != nullptr && t >= 1 && pass_total(f.diff2, t) == 0ull))
      atomicMin(&s_first_zero, t);
  }
  __syncthreads();
  const int z = s_first_zero;
  const int iters = (z < f.k) ? z + 1 : f.k;
  int J = z / f.T + 1;  // launches that ran: launch j runs iff no zero before its first pass
  if (J > f.launches) J = f.launches;
  if (f.k == 0) J = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && f.iterations) *f.iterations = iters;
  const uint8_t* fin = (J == 0) ? f.first_src
                       : (((f.launches - J) % 2) == 0 ? f.buf_even_from_end : f.buf_odd_from_end);
  if (fin == f.out) return;
  copy_range(fin, f.out, f.n);
}

// ---- many-image helpers ----------------------------------------------------------

struct CopyDesc {
  const uint8_t* src;
  uint8_t* dst;
  long long n;   // 0: nothing to copy
};

// grid (X, ncopies): blocks (., y) copy descriptor y.
[[maybe_unused]] static __global__ void multi_copy_kernel(const CopyDesc* d, int ncopies) {
  for (int y = blockIdx.y; y < ncopies; y += gridDim.y) {
    const CopyDesc c = d[y];
    if (c.n > 0) copy_range(c.src, c.dst, c.n);
  }
}

struct BatchFinishDesc {
  const unsigned long long* counts;  // the image's count slots
  unsigned long long* changed;       // out: per-pass totals (k entries), may be null
  int* iterations;                   // out, may be null
  const uint8_t* first_src;          // image when no launch ran
  const uint8_t* buf_even_from_end;  // dst of launches j with (launches-1-j) even
  const uint8_t* buf_odd_from_end;   // the other buffer
  uint8_t* out;
  long long n;
  int k, T, launches, pad;
};

// grid (X, nimages): per image, the totals, the iteration count, and the
// final image moved to `out` if it ended in the workspace.
[[maybe_unused]] static __global__ void batch_finish_kernel(const BatchFinishDesc* descs, int nimages) {
  __shared__ int s_first_zero;
  for (int y = blockIdx.y; y < nimages; y += gridDim.y) {
    const BatchFinishDesc f = descs[y];
    __syncthreads();
    if (threadIdx.x == 0) s_first_zero = f.k;
    __syncthreads();
    for (int t = threadIdx.x; t < f.k; t += blockDim.x) {
      const unsigned long long tot = pass_total(f.counts, t);
      if (blockIdx.x == 0 && f.changed) f.changed[t] = tot;
      if (tot == 0ull) atomicMin(&s_first_zero, t);
    }
    __syncthreads();
    const int z = s_first_zero;
    const int iters = (z < f.k) ? z + 1 : f.k;
    int J = z / f.T + 1;
    if (J > f.launches) J = f.launches;
    if (f.k == 0) J = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && f.iterations) *f.iterations = iters;
    const uint8_t* fin = (J == 0) ? f.first_src
                         : (((f.launches - J) % 2) == 0 ? f.buf_even_from_end : f.buf_odd_from_end);
    if (fin != f.out && f.n > 0) copy_range(fin, f.out, f.n);
  }
}

// Exhaustive check of udiv_small (S < 2^23, 1 <= F <= 81: every quotient
// the kernels form has S <= 81 * 255^2 < 2^23) and isqrt_small (q < 2^16)
// against their definitions; fails[0], fails[1] count wrong results.
[[maybe_unused]] static __global__ void selftest_kernel(unsigned long long* fails) {
  const long long nd = (1ll << 23) * 81;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned bad_div = 0, bad_sqrt = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nd; i += stride) {
    const uint32_t S = uint32_t(i >> 0) & ((1u << 23) - 1);
    const uint32_t F = uint32_t(i >> 23) + 1;
    const uint32_t qq = udiv_small(S, F);
    const unsigned long long lo = (unsigned long long)qq * F;
    bad_div += !(lo <= S && S < lo + F);
    if (i < 65536) {
      const uint32_t r = isqrt_small(uint32_t(i));
      bad_sqrt += !(r * r <= uint32_t(i) && (unsigned long long)(r + 1) * (r + 1) > (unsigned long long)i) ||
                  r != isqrt16(uint32_t(i));
    }
  }
  if (bad_div) atomicAdd(fails, (unsigned long long)bad_div);
  if (bad_sqrt) atomicAdd(fails + 1, (unsigned long long)bad_sqrt);
}

// Algorithm 1 by gathering: card[p] = #{q in window(p), q in image,
// |I(q) - I(p)| < alpha}.  One thread per pixel, bytes read from HBM.
[[maybe_unused]] static __global__ void cardinality_kernel(const uint8_t* __restrict__ img, int rows, int cols,
                                   int alpha, int beta, uint16_t* __restrict__ card) {
  const long long n = (long long)rows * cols;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const int r = int(p / cols);
    const int c = int(p - (long long)r * cols);
    const int x = img[p];
    int cnt = 0;
    // the window clipped to the image (in 64 bits: r + beta may pass INT_MAX)
    const int i0 = r - beta < 0 ? 0 : r - beta;
    const int i1 = int((long long)r + beta < rows ? (long long)r + beta : rows - 1);
    const int j0 = c - beta < 0 ? 0 : c - beta;
    const int j1 = int((long long)c + beta < cols ? (long long)c + beta : cols - 1);
    for (int i = i0; i <= i1; ++i) {
      for (int j = j0; j <= j1; ++j) {
        const int y = img[(long long)i * cols + j];
        cnt += (y < x + alpha && y > x - alpha) ? 1 : 0;
      }
    }
    card[p] = uint16_t(cnt);
  }
}

}  // namespace phg
