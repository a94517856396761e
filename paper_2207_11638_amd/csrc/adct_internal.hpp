// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/adct.h"
#include "butterflies.hpp"

namespace adct {

enum : int { DT_U8 = 0, DT_I16 = 1 };

// Image-set geometry, strides in pixels.
struct Geom {
  int64_t pitch;
  int64_t image_stride;
  int batch;
  int tiles_y;  // per image
  int tiles_x;  // per image
};

// Per-(transform, n, qstep) constant tables.  The diagonal of T T^T takes at
// most four distinct values for every transform and block length, so the
// tables are indexed by row classes: entry [cls[v] * 4 + cls[u]].
struct Tables {
  float s2[16];    // s_v s_u, rounded once from double
  int32_t mq[16];  // quantiser multipliers (2^24 fixed point)
  int32_t dq[16];  // dequantiser factors (one fractional bit)
  uint8_t cls[64]; // row class of each frequency
};

// Arguments of one pass over an image set.
struct PassParams {
  const void* src;        // pixels in (forward, compress)
  void* dst;              // pixels out (inverse, compress recon, decompress)
  const int32_t* cin;     // coefficients in (inverse, decompress)
  int32_t* cout;          // coefficients out (forward, compress kept)
  float* scaled;          // compress: scaled coefficients (nullable)
  unsigned long long* sse;  // compress: per-image error energy (nullable)
  Geom g;
  int r;
  int qstep;
  int gpw;                // compress: tile groups per workgroup along a tile row
  int spread;             // compress, n = 8: images interleaved in dispatch order
  Tables t;
};

// Tile groups one fused workgroup walks along its tile row.  Every workgroup
// adds its image's error energy with one 64-bit atomic, and all workgroups
// resident at a time work on one or two images, so those atomics meet on one
// or two addresses; walking several groups divides their number.  Capped at 8
// and lowered while the grid would hold fewer than 8192 workgroups.
inline int groups_per_wg(int groups_x, int64_t rows) {
  int gpw = groups_x < 8 ? groups_x : 8;
  while (gpw > 1 && static_cast<int64_t>((groups_x + gpw - 1) / gpw) * rows < 8192) gpw >>= 1;
  return gpw < 1 ? 1 : gpw;
}

// Sum of v over the 64 lanes of a wave (every lane active), as a uniform
// value.  Data-parallel-primitive steps: shifts right by 1, 2, 4 and 8 within
// each row of 16 lanes leave every row's sum in its lane 15; the broadcast of
// lane 15 into the next row and of lane 31 into rows 2 and 3 then gathers the
// four row sums in lane 63.  Lanes whose source lies outside the row (or in a
// row the step does not write) add zero.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Sum e over the BS threads of a workgroup and add it to *sse with one
// atomic (none when the sum is zero).  red: BS / 64 words of LDS (unused for
// a single wave).  Every thread of the workgroup calls it, with every lane of
// its wave active.  Each e must be below 2^48 (the largest per-thread error
// energy of the kernels is below 2^41): its low 24 and high 24 bits are summed
// over the wave as two 32-bit values (64 terms below 2^24 each).
template <int BS>
__device__ __forceinline__ void block_add_sse(unsigned long long* sse, unsigned long long e,
                                              unsigned long long* red) {
  const uint32_t lo = wave_sum_u32(static_cast<uint32_t>(e) & 0xffffffu);
  const uint32_t hi = wave_sum_u32(static_cast<uint32_t>(e >> 24));
  const unsigned long long w = static_cast<unsigned long long>(lo) +
                               (static_cast<unsigned long long>(hi) << 24);
  if constexpr (BS == 64) {
    if (threadIdx.x == 0 && w != 0) atomicAdd(sse, w);
  } else {
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long sum = 0;
#pragma unroll
      for (int i = 0; i < BS / 64; ++i) sum += red[i];
      if (sum != 0) atomicAdd(sse, sum);
    }
  }
}

// Quantiser multiplier MQ (2^24 fixed point) as the float64 m = MQ / 2^24
// (exact).
__device__ __forceinline__ double quant_mult(int32_t mq) {
  return static_cast<double>(mq) * 0x1p-24;
}

// Quantisation level sign(b) floor(|b| MQ / 2^24 + 1/2), evaluated in
// float64 as the truncation toward zero of sign(b) (|b| m + 1/2): |b| MQ <
// 2^47, so |b| m + 1/2 is exact (a numerator below 2^48 over 2^24) and the
// fused multiply-add rounds nothing; truncating the non-negative value
// floors it.  Four full-rate instructions (convert, multiply-add with |b| as
// a source modifier, sign copy, convert), where the 64-bit integer product
// takes a quarter-rate multiply and a sign fix-up.
__device__ __forceinline__ int quantise_level(int b, double m) {
  const double x = static_cast<double>(b);
  return static_cast<int>(__builtin_copysign(__builtin_fma(__builtin_fabs(x), m, 0.5), x));
}

enum class Mode : int { Compress = 0, Forward = 1, Inverse = 2, Decompress = 3 };

// Kernel launchers (return hipError_t as int).
int launch_n8(Mode mode, int kind, int dtype, const PassParams& p, hipStream_t stream);
int launch_jam(Mode mode, int kind, int n, int dtype, const PassParams& p, hipStream_t stream);
// The exact 8-point DCT in float32, fused zonal compress (kernels_dct.hip).
int launch_dct8(int dtype, const PassParams& p, hipStream_t stream);
// Quality measures (quality.hip): coefficient and pixel moments per image,
// the measured and the AR(1) coding gain, PSNR from error energies.
int launch_moments(int kind, int n, int dtype, const void* src, const Geom& g,
                   unsigned long long* mom, hipStream_t s);
int launch_coding_gain(int kind, int n, int basis, const unsigned long long* mom, int count,
                       float* cg, hipStream_t s);
int launch_coding_gain_ar1(int kind, int n, int basis, const float* rho, int count, float* cg,
                           float* cg_klt, hipStream_t s);
int launch_psnr(const unsigned long long* sse, int count, int64_t pixels, float* psnr,
                hipStream_t s);
// Mean SSIM of each image pair (ssim.hip); acc: batch float64 accumulators
// (zeroed here).  APE of values against references, in percent.
int launch_ssim(const uint8_t* x, const uint8_t* y, int batch, int height, int width,
                int64_t pitch, int64_t image_stride, double* acc, float* out, hipStream_t s);
int launch_ape(const float* value, const float* ref, int count, float* out, hipStream_t s);
// Zero `words` 64-bit words with a fill kernel (no memset node in a graph).
int launch_fill_zero(unsigned long long* p, int64_t words, hipStream_t s);
// Fused 8x8 compress (uint8, zonal) on the int8 matrix cores; t = T[v][i] and
// u = (8 T^-1)[i][v], row-major.
int launch_n8_mfma(int kind, const PassParams& p, const int8_t* t, const int8_t* u,
                   hipStream_t stream);

}  // namespace adct
