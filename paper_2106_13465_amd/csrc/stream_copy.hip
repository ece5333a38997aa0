// stream_copy.hip -- a plain streaming copy kernel, the bandwidth reference of
// the measurements (hydro_stream_copy): not part of the method.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace hydro {

// Plain copy of n16 16-byte words: each block copies one contiguous 8 KiB
// chunk (512 words, two per thread, both loads issued before the stores).
// Measured on MI355X over 2 GiB: 6.0 TB/s, against 5.2 TB/s for the best
// grid-stride form, 5.7 TB/s for 64 KiB chunks and 5.0 TB/s for a
// device-to-device hipMemcpy.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyChunk = 512;  // 16-byte words per block
__global__ __launch_bounds__(256) void k_stream_copy(u32x4* __restrict__ dst,
                                                     const u32x4* __restrict__ src, long long n16) {
  const long long i = (long long)blockIdx.x * kCopyChunk + threadIdx.x;
  if (i + 256 < n16) {
    const u32x4 a = __builtin_nontemporal_load(src + i);
    const u32x4 b = __builtin_nontemporal_load(src + i + 256);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + 256);
  } else if (i < n16) {
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  }
}

hipError_t launch_stream_copy(void* dst, const void* src, long long n16, hipStream_t s) {
  const long long blocks = (n16 + kCopyChunk - 1) / kCopyChunk;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<u32x4*>(dst), static_cast<const u32x4*>(src), n16);
  return hipGetLastError();
}

}  // namespace hydro
