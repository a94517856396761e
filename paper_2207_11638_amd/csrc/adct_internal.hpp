// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
  uint8_t cls[32]; // row class of each frequency
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
  Tables t;
};

enum class Mode : int { Compress = 0, Forward = 1, Inverse = 2, Decompress = 3 };

// Kernel launchers (return hipError_t as int).
int launch_n8(Mode mode, int kind, int dtype, const PassParams& p, hipStream_t stream);
int launch_jam(Mode mode, int kind, int n, int dtype, const PassParams& p, hipStream_t stream);

}  // namespace adct
