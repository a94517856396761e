// Streaming ceilings of the HBM: plain read-only, write-only and copy kernels
// that move 16-byte words with non-temporal hints and nothing else.  They
// are the reference the fused kernels' bandwidth is set against (a
// measurement aid, no operation of the paper).
//
// The grid-stride kernels walk the buffer as thread t of the grid handling
// 16-byte words t, t + G, t + 2G, ... (G = threads in the grid); the chunked
// ones give each workgroup one contiguous chunk, walked by its 256 threads.
// Both take U words per step with all U loads issued before any use, so a
// wave keeps U * 1 KiB in flight.  The read kernel folds its words into one value per
// thread and stores it only if it equals a pattern no input produces here
// (the caller passes a zero buffer and a non-zero pattern), so the loads
// cannot be removed and nothing is written back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/adct.h"
#include "adct_internal.hpp"

namespace adct {

int set_error(int status, const char* msg);

namespace {

constexpr int kBS = 256;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ __launch_bounds__(kBS) void read_words(const u32x4* __restrict__ src, int64_t words,
                                                  uint32_t pattern, uint32_t* __restrict__ sink) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBS;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (U - 1) * stride < words; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < words; i += stride) {
    const u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == pattern) sink[0] = acc;
}

template <int U>
__global__ __launch_bounds__(kBS) void write_words(u32x4* __restrict__ dst, int64_t words,
                                                   uint32_t value) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBS;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
  const u32x4 v = {value, value, value, value};
  for (; i < words; i += stride) __builtin_nontemporal_store(v, dst + i);
}

template <int U>
__global__ __launch_bounds__(kBS) void copy_words(const u32x4* __restrict__ src,
                                                  u32x4* __restrict__ dst, int64_t words) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBS;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kBS + threadIdx.x;
  for (; i + (U - 1) * stride < words; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < words; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Chunked: workgroup b owns words [b C, (b + 1) C) (C a multiple of 256 U
// words), its threads striding by 256.  MODE 0 reads, 1 writes, 2 copies.
template <int U, int MODE>
__global__ __launch_bounds__(kBS) void chunk_words(const u32x4* __restrict__ src,
                                                   u32x4* __restrict__ dst, int64_t words,
                                                   int64_t chunk, uint32_t pattern) {
  const int64_t begin = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t end = min(begin + chunk, words);
  int64_t i = begin + threadIdx.x;
  uint32_t acc = 0;
  const u32x4 z = {pattern, pattern, pattern, pattern};
  for (; i + (U - 1) * kBS < end; i += U * kBS) {
    u32x4 v[U];
    if constexpr (MODE != 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * kBS);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (MODE == 0) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      else if constexpr (MODE == 1) __builtin_nontemporal_store(z, dst + i + u * kBS);
      else __builtin_nontemporal_store(v[u], dst + i + u * kBS);
    }
  }
  for (; i < end; i += kBS) {
    if constexpr (MODE == 0) {
      const u32x4 v = __builtin_nontemporal_load(src + i);
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    } else if constexpr (MODE == 1) {
      __builtin_nontemporal_store(z, dst + i);
    } else {
      __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    }
  }
  if constexpr (MODE == 0)
    if (acc == pattern) reinterpret_cast<uint32_t*>(dst)[0] = acc;
}

template <int U>
hipError_t launch_u(int pattern, void* dst, const void* src, int64_t words, int blocks,
                    hipStream_t s) {
  if (pattern >= 3) {
    const int64_t step = static_cast<int64_t>(kBS) * U;
    const int64_t per = (words + blocks - 1) / blocks;
    const int64_t chunk = (per + step - 1) / step * step;
    const u32x4* sv = static_cast<const u32x4*>(src);
    u32x4* dv = static_cast<u32x4*>(dst);
    if (pattern == 3) chunk_words<U, 0><<<blocks, kBS, 0, s>>>(sv, dv, words, chunk, 0x9e3779b9u);
    else if (pattern == 4) chunk_words<U, 1><<<blocks, kBS, 0, s>>>(sv, dv, words, chunk, 0u);
    else chunk_words<U, 2><<<blocks, kBS, 0, s>>>(sv, dv, words, chunk, 0u);
    return hipGetLastError();
  }
  switch (pattern) {
    case 0:
      read_words<U><<<blocks, kBS, 0, s>>>(static_cast<const u32x4*>(src), words, 0x9e3779b9u,
                                            static_cast<uint32_t*>(dst));
      break;
    case 1:
      write_words<U><<<blocks, kBS, 0, s>>>(static_cast<u32x4*>(dst), words, 0u);
      break;
    default:
      copy_words<U><<<blocks, kBS, 0, s>>>(static_cast<const u32x4*>(src),
                                            static_cast<u32x4*>(dst), words);
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

ADCT_API int adct_stream_ceiling(int pattern, void* d_dst, const void* d_src, int64_t bytes,
                                 int blocks, int unroll, adct_stream_t stream) {
  if (pattern < 0 || pattern > 5 || bytes < 0 || bytes % 16 || blocks < 1 ||
      (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8))
    return set_error(ADCT_E_ARG, "stream_ceiling: bad pattern, size, grid or unroll");
  if ((pattern != 1 && pattern != 4 && d_src == nullptr) || d_dst == nullptr)
    return set_error(ADCT_E_ARG, "stream_ceiling: null buffer");
  if ((reinterpret_cast<uintptr_t>(d_src) % 16) || (reinterpret_cast<uintptr_t>(d_dst) % 16))
    return set_error(ADCT_E_ALIGN, "stream_ceiling: buffers must be 16-byte aligned");
  if (bytes == 0) return set_error(ADCT_OK, "");
  const int64_t words = bytes / 16;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  switch (unroll) {
    case 1: e = launch_u<1>(pattern, d_dst, d_src, words, blocks, s); break;
    case 2: e = launch_u<2>(pattern, d_dst, d_src, words, blocks, s); break;
    case 4: e = launch_u<4>(pattern, d_dst, d_src, words, blocks, s); break;
    default: e = launch_u<8>(pattern, d_dst, d_src, words, blocks, s);
  }
  if (e != hipSuccess) return set_error(ADCT_E_HIP, hipGetErrorString(e));
  return set_error(ADCT_OK, "");
}

}  // extern "C"
