// calib.hip -- the two ceilings the pass kernels are measured against,
// taken on the device they run on: a streaming copy (the HBM bandwidth a
// kernel can reach) and loops of independent integer VALU instructions of
// one kind (the issue rate of the vector ALUs).  Measurement only; no
// part of the pass uses them.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "phgrms.h"
#include "phgrms_internal.hpp"

using namespace phg;

namespace {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;        // 16-byte vectors in flight per lane
constexpr int kValuChains = 8;        // independent registers per lane
constexpr int kValuUnroll = 16;       // steps of all chains per loop trip
constexpr int kValuPerTrip = kValuChains * kValuUnroll;
constexpr int kValuKinds = 9;         // instruction kinds the issue loop can time
constexpr int kMixGroupInstr = 17;    // kind 8: one group of four band tests
constexpr int kMixPerTrip = 2 * kValuChains * kMixGroupInstr;

typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

// Grid-stride copy of n16 16-byte vectors: every lane issues kCopyUnroll
// loads, then the stores, so each wave keeps several lines in flight.
// Lane i of a workgroup touches vector base + i (+ 256 u), so a wave's
// accesses are 1 KiB contiguous.  Loads and stores are non-temporal
// (streamed past the caches; about 10 % faster than cached ones here).
__global__ __launch_bounds__(kCopyThreads) void calib_copy_kernel(const v4u32* __restrict__ src,
                                                                  v4u32* __restrict__ dst,
                                                                  size_t n16) {
  const size_t chunk = size_t(kCopyThreads) * kCopyUnroll;
  const size_t step = size_t(gridDim.x) * chunk;
  size_t base = size_t(blockIdx.x) * chunk + threadIdx.x;
  for (; base + (kCopyUnroll - 1) * kCopyThreads < n16; base += step) {
    v4u32 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u)
      v[u] = __builtin_nontemporal_load(src + base + size_t(u) * kCopyThreads);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u)
      __builtin_nontemporal_store(v[u], dst + base + size_t(u) * kCopyThreads);
  }
  // the ragged end: fewer than kCopyUnroll vectors of this lane remain
  for (; base < n16; base += kCopyThreads) dst[base] = src[base];
}

// Each lane runs `trips` x kValuPerTrip VALU instructions of one kind on
// kValuChains registers.  A step updates chain j from chains j+1 and j+3,
// so no instruction waits on the one before it and the compiler can
// neither fold nor drop them (they are written as single instructions).
// The kinds are the integer instructions the pass kernels issue most:
// 0 v_add_u32, 1 v_lerp_u8, 2 v_xor_b32, 3 v_bitop3_b32, 4 v_add3_u32,
// 5 v_alignbyte_b32, 6 v_pk_add_u16, 7 v_dot4_u32_u8.
template <int KIND>
__global__ __launch_bounds__(256) void calib_valu_kernel(uint32_t* out, int trips) {
  uint32_t a[kValuChains];
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kValuChains; ++j) a[j] = tid * 0x9e3779b9u + uint32_t(j) * 0x7f4a7c15u;
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < kValuUnroll; ++u) {
#pragma unroll
      for (int j = 0; j < kValuChains; ++j) {
        const uint32_t b = a[(j + 1) % kValuChains], c = a[(j + 3) % kValuChains];
        if constexpr (KIND == 0)
          asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else if constexpr (KIND == 1)
          asm volatile("v_lerp_u8 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 2)
          asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else if constexpr (KIND == 3)
          asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 4)
          asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 5)
          asm volatile("v_alignbyte_b32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
        else if constexpr (KIND == 6)
          asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        else
          asm volatile("v_dot4_u32_u8 %0, %1, %2, %0" : "+v"(a[j]) : "v"(b), "v"(c));
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < kValuChains; ++j) r ^= a[j];
  out[tid] = r;
}

// Kind 8, the band test's instruction mix: each group tests four neighbour
// words against one centre's two band limits (two v_lerp_u8 and one
// v_xor_b32 per neighbour) and adds the four in-band bits to two saturating
// counters (five v_bitop3_b32), as the pass kernels' inner loop does.
// Chain j's centre limits are a[j] and a[j+5], its neighbours a[j+1..j+4];
// the counters t1, t2 accumulate over the whole loop.
__global__ __launch_bounds__(256) void calib_mix_kernel(uint32_t* out, int trips) {
  uint32_t a[kValuChains], t1[kValuChains], t2[kValuChains];
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kValuChains; ++j) {
    a[j] = tid * 0x9e3779b9u + uint32_t(j) * 0x7f4a7c15u;
    t1[j] = 0u;
    t2[j] = 0u;
  }
  const uint32_t ones = 0x01010101u;
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int j = 0; j < kValuChains; ++j) {
        // one asm block per group: no hazard padding between its instructions
        uint32_t lo, hi, m0, m1, m2, m3, cg, sg, ug;
        asm volatile(
            "v_lerp_u8 %[lo], %[y0], %[nlo], %[one]\n\t"
            "v_lerp_u8 %[hi], %[y0], %[nhi], 0\n\t"
            "v_xor_b32 %[m0], %[lo], %[hi]\n\t"
            "v_lerp_u8 %[lo], %[y1], %[nlo], %[one]\n\t"
            "v_lerp_u8 %[hi], %[y1], %[nhi], 0\n\t"
            "v_xor_b32 %[m1], %[lo], %[hi]\n\t"
            "v_lerp_u8 %[lo], %[y2], %[nlo], %[one]\n\t"
            "v_lerp_u8 %[hi], %[y2], %[nhi], 0\n\t"
            "v_xor_b32 %[m2], %[lo], %[hi]\n\t"
            "v_lerp_u8 %[lo], %[y3], %[nlo], %[one]\n\t"
            "v_lerp_u8 %[hi], %[y3], %[nhi], 0\n\t"
            "v_xor_b32 %[m3], %[lo], %[hi]\n\t"
            "v_bitop3_b32 %[cg], %[m0], %[m1], %[m2] bitop3:0xe8\n\t"
            "v_bitop3_b32 %[sg], %[m0], %[m1], %[m2] bitop3:0x96\n\t"
            "v_bitop3_b32 %[ug], %[t1], %[sg], %[m3] bitop3:0xe8\n\t"
            "v_bitop3_b32 %[t2], %[t2], %[cg], %[ug] bitop3:0xfe\n\t"
            "v_bitop3_b32 %[t1], %[t1], %[sg], %[m3] bitop3:0xfe"
            : [t1] "+v"(t1[j]), [t2] "+v"(t2[j]), [lo] "=&v"(lo), [hi] "=&v"(hi),
              [m0] "=&v"(m0), [m1] "=&v"(m1), [m2] "=&v"(m2), [m3] "=&v"(m3),
              [cg] "=&v"(cg), [sg] "=&v"(sg), [ug] "=&v"(ug)
            : [y0] "v"(a[(j + 1) % kValuChains]), [y1] "v"(a[(j + 2) % kValuChains]),
              [y2] "v"(a[(j + 3) % kValuChains]), [y3] "v"(a[(j + 4) % kValuChains]),
              [nlo] "v"(a[j]), [nhi] "v"(a[(j + 5) % kValuChains]), [one] "v"(ones));
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < kValuChains; ++j) r ^= t1[j] ^ (t2[j] * 3u);
  out[tid] = r;
}

}  // namespace

extern "C" int phgrms_calib_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
  if (bytes == 0) return PHGRMS_OK;
  if (d_src == nullptr || d_dst == nullptr) return fail(PHGRMS_EINVAL, "null pointer");
  if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst) | bytes) & 15u)
    return fail(PHGRMS_EINVAL, "pointers and size must be multiples of 16 bytes");
  const uintptr_t s = reinterpret_cast<uintptr_t>(d_src), d = reinterpret_cast<uintptr_t>(d_dst);
  if (s < d + bytes && d < s + bytes) return fail(PHGRMS_EINVAL, "source and destination overlap");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  const size_t n16 = bytes / 16;
  const size_t chunk = size_t(kCopyThreads) * kCopyUnroll;
  // 32 workgroups of 4 waves per CU (measured best with 16-64), fewer when
  // the copy is small
  const size_t blocks = std::min<size_t>(size_t(cus) * 32, (n16 + chunk - 1) / chunk);
  hipLaunchKernelGGL(calib_copy_kernel, dim3(unsigned(blocks)), dim3(kCopyThreads), 0,
                     static_cast<hipStream_t>(stream), static_cast<const v4u32*>(d_src),
                     static_cast<v4u32*>(d_dst), n16);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return PHGRMS_OK;
}

extern "C" int phgrms_calib_valu(uint32_t* d_out, int32_t blocks, int32_t trips, int32_t kind,
                                 uint64_t* h_valu_per_wave, void* stream) {
  if (d_out == nullptr) return fail(PHGRMS_EINVAL, "null pointer");
  if (blocks < 1 || blocks > (1 << 20)) return fail(PHGRMS_EINVAL, "blocks %d", blocks);
  if (trips < 1 || trips > (1 << 24)) return fail(PHGRMS_EINVAL, "trips %d", trips);
  if (kind < 0 || kind >= kValuKinds) return fail(PHGRMS_EINVAL, "kind %d", kind);
  if (h_valu_per_wave)
    *h_valu_per_wave = uint64_t(trips) * (kind == kValuKinds - 1 ? kMixPerTrip : kValuPerTrip);
  hipStream_t s = static_cast<hipStream_t>(stream);
  static constexpr void (*kKernels[kValuKinds])(uint32_t*, int) = {
      calib_valu_kernel<0>, calib_valu_kernel<1>, calib_valu_kernel<2>, calib_valu_kernel<3>,
      calib_valu_kernel<4>, calib_valu_kernel<5>, calib_valu_kernel<6>, calib_valu_kernel<7>,
      calib_mix_kernel};
  hipLaunchKernelGGL(kKernels[kind], dim3(blocks), dim3(256), 0, s, d_out, trips);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "valu launch");
  return PHGRMS_OK;
}
