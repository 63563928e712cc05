// Streaming device copy with 16-byte lanes.  Not part of the method: it is the practical HBM
// ceiling the step kernels are measured against, and the kernel of known traffic (bytes read plus
// bytes written) that calibrates the hardware byte counters of a profile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "lbm.h"

namespace {

constexpr int COPY_NT = 256;
constexpr int COPY_UNROLL = 4;  // 16-byte loads in flight per thread before its stores

// Each workgroup copies contiguous blocks of COPY_NT * COPY_UNROLL vectors (16 KiB), striding over
// the buffer by the grid; a thread issues its COPY_UNROLL loads first, then the stores.
__global__ __launch_bounds__(COPY_NT) void copy16_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         size_t n16) {
  constexpr size_t BLOCK = (size_t)COPY_NT * COPY_UNROLL;
  for (size_t b = (size_t)blockIdx.x * BLOCK; b < n16; b += (size_t)gridDim.x * BLOCK) {
    uint4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
      const size_t i = b + (size_t)u * COPY_NT + threadIdx.x;
      if (i < n16) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
      const size_t i = b + (size_t)u * COPY_NT + threadIdx.x;
      if (i < n16) dst[i] = v[u];
    }
  }
}

}  // namespace

extern "C" lbm_status lbm_device_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst || bytes % 16 != 0 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0)
    return LBM_E_INVAL;
  if (bytes == 0) return LBM_OK;
  const size_t n16 = bytes / 16;
  const size_t blocks = (n16 + (size_t)COPY_NT * COPY_UNROLL - 1) / ((size_t)COPY_NT * COPY_UNROLL);
  // enough workgroups to fill the 256 compute units several times over
  const int grid = (int)std::min<size_t>(blocks, 256 * 16);
  copy16_kernel<<<grid, COPY_NT, 0, (hipStream_t)hip_stream>>>((const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}
