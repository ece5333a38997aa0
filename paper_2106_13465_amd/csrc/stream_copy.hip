// stream_copy.hip -- a plain streaming copy kernel, the bandwidth reference of
// the measurements (hydro_stream_copy): not part of the method.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace hydro {

// Plain copy of n16 16-byte words as 4-byte lanes: each block copies one
// contiguous 8 KiB chunk (2048 words, eight per thread, all loads issued
// before the stores), with streaming loads and stores.  Measured on MI355X
// over 2 GiB: 6.4 TB/s, against 6.3 TB/s with 8-byte and 5.9 TB/s with
// 16-byte lanes in the same chunks, 5.2 TB/s for the best grid-stride form,
// 5.7 TB/s for 64 KiB chunks and 5.0 TB/s for a device-to-device hipMemcpy.
constexpr int kCopyChunk = 2048;  // 4-byte words per block
constexpr int kCopyPer = kCopyChunk / 256;
__global__ __launch_bounds__(256) void k_stream_copy(unsigned* __restrict__ dst,
                                                     const unsigned* __restrict__ src, long long n4) {
  const long long i = (long long)blockIdx.x * kCopyChunk + threadIdx.x;
  if (i + (kCopyChunk - 256) < n4) {
    unsigned v[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) v[k] = __builtin_nontemporal_load(src + i + k * 256);
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) __builtin_nontemporal_store(v[k], dst + i + k * 256);
  } else {
    for (int k = 0; k < kCopyPer; ++k)
      if (i + k * 256 < n4)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i + k * 256), dst + i + k * 256);
  }
}

hipError_t launch_stream_copy(void* dst, const void* src, long long n16, hipStream_t s) {
  const long long n4 = 4 * n16;
  const long long blocks = (n4 + kCopyChunk - 1) / kCopyChunk;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned*>(dst), static_cast<const unsigned*>(src), n4);
  return hipGetLastError();
}

}  // namespace hydro
