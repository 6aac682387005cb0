// quality.hip -- the steps around the pass loop in the paper's experiments
// (Section 3): salt-and-pepper noise at a given density, the input the
// method is measured on (Tables 1-2), and the sum of squared differences
// behind the peak signal-to-noise ratio, the restoration measure of Table 2.
//
// Both are memory-bound streams (1 B read + 1 B written, or 2 B read, per
// pixel); they are not part of the pass loop.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phgrms.h"
#include "phgrms_internal.hpp"

using namespace phg;

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;   // SplitMix64 increment

// Output i (0-based) of a SplitMix64 generator seeded with `seed`: its
// state after i+1 steps is seed + (i+1)*gamma, and an output is that state
// through the generator's two xor-shift-multiply rounds and a final
// xor-shift (Steele, Lea and Flood's generator, with the mixing constants of
// its reference implementation).  Random access by pixel index makes the
// noise independent of the launch shape.
__device__ __forceinline__ uint64_t splitmix64_output(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1u) * kGamma;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Pixel i becomes pepper (0) if u < t_pepper, salt (255) if
// t_pepper <= u < t_salt, else keeps its value; u = the top 32 bits of
// output i.  Each thread reads and writes only its own pixels, so in place
// is fine.
__global__ void salt_pepper_kernel(const uint8_t* in, uint8_t* out, long long n, uint64_t seed,
                                   uint32_t t_pepper, uint32_t t_salt) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const uint32_t u = uint32_t(splitmix64_output(seed, uint64_t(i)) >> 32);
    uint8_t v = in[i];
    if (u < t_pepper)
      v = 0;
    else if (u < t_salt)
      v = 255;
    out[i] = v;
  }
}

__global__ void zero_one_kernel(unsigned long long* p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0ull;
}

// Sum over i of (a[i] - b[i])^2 into *sum (zeroed beforehand): a per-thread
// partial, a wave reduction, a workgroup reduction in LDS, one atomic per
// workgroup.
__global__ __launch_bounds__(256) void sq_diff_kernel(const uint8_t* a, const uint8_t* b,
                                                      long long n, unsigned long long* sum) {
  unsigned long long s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int d = int(a[i]) - int(b[i]);
    s += (unsigned long long)(d * d);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  __shared__ unsigned long long part[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = part[0] + part[1] + part[2] + part[3];
    if (t != 0ull) atomicAdd(sum, t);
  }
}

int grid_for(long long n) {
  const long long g = (n + 255) / 256;
  return int(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

extern "C" {

int phgrms_salt_pepper(const uint8_t* d_in, uint8_t* d_out, int64_t n, uint64_t seed,
                       uint32_t t_pepper, uint32_t t_salt, void* stream) {
  if (n < 0) return fail(PHGRMS_EINVAL, "negative pixel count");
  if (t_pepper > t_salt) return fail(PHGRMS_EINVAL, "t_pepper %u > t_salt %u", t_pepper, t_salt);
  if (n == 0) return PHGRMS_OK;
  if (d_in == nullptr || d_out == nullptr) return fail(PHGRMS_EINVAL, "null image pointer");
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_in), b = reinterpret_cast<uintptr_t>(d_out);
  if (a != b && a < b + uintptr_t(n) && b < a + uintptr_t(n))
    return fail(PHGRMS_EINVAL, "input and output overlap without being the same buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(salt_pepper_kernel, dim3(grid_for(n)), dim3(256), 0, s, d_in, d_out,
                     (long long)n, seed, t_pepper, t_salt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "noise launch");
  return PHGRMS_OK;
}

int phgrms_sq_diff_sum(const uint8_t* d_a, const uint8_t* d_b, int64_t n, int64_t* d_sum,
                       void* stream) {
  if (n < 0) return fail(PHGRMS_EINVAL, "negative pixel count");
  if (d_sum == nullptr) return fail(PHGRMS_EINVAL, "null result pointer");
  if (n > 0 && (d_a == nullptr || d_b == nullptr)) return fail(PHGRMS_EINVAL, "null image pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* sum = reinterpret_cast<unsigned long long*>(d_sum);
  hipLaunchKernelGGL(zero_one_kernel, dim3(1), dim3(64), 0, s, sum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "zero launch");
  if (n > 0) {
    hipLaunchKernelGGL(sq_diff_kernel, dim3(grid_for(n)), dim3(256), 0, s, d_a, d_b,
                       (long long)n, sum);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "sum launch");
  }
  return PHGRMS_OK;
}

}  // extern "C"
