// scatter.hip -- Algorithm 1 in the form the paper prints it (Section 2):
// every pixel p adds one to the cardinality of each pixel q of its window
// whose grey level lies in p's strict band (I(p) - alpha, I(p) + alpha).
// The printed kernel does the increments without atomics, so concurrent
// threads can lose updates; here they are atomic, first in LDS, then one
// global atomic per touched cell.  Because the band relation is symmetric
// the result equals the gather form (phgrms_cardinality); this path exists
// to show that on the GPU, not for speed.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phgrms.h"
#include "phgrms_internal.hpp"

using namespace phg;

namespace {

constexpr int kSW = 64;   // source tile columns per workgroup
constexpr int kSH = 16;   // source tile rows per workgroup

__global__ void zero_u32_kernel(uint32_t* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// One workgroup: the kSH x kSW source pixels of its tile scatter into an
// LDS count array covering the tile plus a BETA halo, which is then added to
// the global counts.  LDS: the image region as ints and the counts.
template <int BETA>
__global__ __launch_bounds__(256) void scatter_card_kernel(const uint8_t* img, int rows, int cols,
                                                           int alpha, int tiles_x, int ntiles,
                                                           uint32_t* card) {
  constexpr int RW = kSW + 2 * BETA, RH = kSH + 2 * BETA;   // region
  __shared__ int val[RH * RW];
  __shared__ uint32_t cnt[RH * RW];
  // (a grid smaller than the tile count takes the rest in strides)
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int r0 = ty * kSH - BETA, c0 = tx * kSW - BETA;     // image coords of region (0, 0)
    for (int k = threadIdx.x; k < RH * RW; k += blockDim.x) {
      const long long r = (long long)r0 + k / RW, c = (long long)c0 + k % RW;
      const bool in = r >= 0 && r < rows && c >= 0 && c < cols;
      val[k] = in ? int(img[size_t(r) * size_t(cols) + size_t(c)]) : -1;   // -1: outside
      cnt[k] = 0u;
    }
    __syncthreads();
    // thread t: column t % kSW of the tile, rows t / kSW, + 4, + 8, + 12
    for (int s = threadIdx.x; s < kSH * kSW; s += blockDim.x) {
      const int pr = s / kSW + BETA, pc = s % kSW + BETA;     // region coords of p
      const int x = val[pr * RW + pc];
      if (x < 0) continue;                                    // p outside the image
      for (int dr = -BETA; dr <= BETA; ++dr)
        for (int dc = -BETA; dc <= BETA; ++dc) {
          const int q = (pr + dr) * RW + (pc + dc);
          const int y = val[q];
          if (y >= 0 && y > x - alpha && y < x + alpha) atomicAdd(&cnt[q], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < RH * RW; k += blockDim.x) {
      const uint32_t v = cnt[k];
      if (v != 0u) {
        const long long r = (long long)r0 + k / RW, c = (long long)c0 + k % RW;  // (val >= 0: in the image)
        atomicAdd(&card[size_t(r) * size_t(cols) + size_t(c)], v);
      }
    }
    __syncthreads();   // the next tile overwrites val and cnt
  }
}

template <int BETA>
hipError_t launch(const uint8_t* img, int rows, int cols, int alpha, uint32_t* card,
                  hipStream_t s) {
  const int tiles_x = int((static_cast<long long>(cols) + kSW - 1) / kSW);
  const int tiles_y = int((static_cast<long long>(rows) + kSH - 1) / kSH);
  const int ntiles = tiles_x * tiles_y;   // < 2^31 (checked by the caller)
  const int grid = int(std::min<long long>(ntiles, max_workgroups(256)));
  hipLaunchKernelGGL(scatter_card_kernel<BETA>, dim3(grid), dim3(256), 0, s, img, rows, cols,
                     alpha, tiles_x, ntiles, card);
  return hipGetLastError();
}

}  // namespace

extern "C" int phgrms_cardinality_scatter(const uint8_t* d_img, int32_t rows, int32_t cols,
                                          int32_t alpha, int32_t beta, uint32_t* d_card,
                                          void* stream) {
  phgrms_params p{rows, cols, alpha, beta, 0};
  int rc = validate_params(p);
  if (rc != PHGRMS_OK) return rc;
  const long long n = (long long)rows * cols;
  if (n == 0) return PHGRMS_OK;
  if (d_img == nullptr || d_card == nullptr) return fail(PHGRMS_EINVAL, "null pointer");
  if (((static_cast<long long>(rows) + kSH - 1) / kSH) * ((static_cast<long long>(cols) + kSW - 1) / kSW) >
      0x7fffffffll)
    return fail(PHGRMS_EINVAL, "too many tiles");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int zb = int(std::min<long long>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(zero_u32_kernel, dim3(zb), dim3(256), 0, s, d_card, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  switch (beta) {
    case 1: e = launch<1>(d_img, rows, cols, alpha, d_card, s); break;
    case 2: e = launch<2>(d_img, rows, cols, alpha, d_card, s); break;
    case 3: e = launch<3>(d_img, rows, cols, alpha, d_card, s); break;
    case 4: e = launch<4>(d_img, rows, cols, alpha, d_card, s); break;
    default: return fail(PHGRMS_EUNSUPPORTED, "beta %d", beta);
  }
  if (e != hipSuccess) return hip_fail(e, "scatter launch");
  return PHGRMS_OK;
}
