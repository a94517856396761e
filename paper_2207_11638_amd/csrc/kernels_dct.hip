// The exact 8-point DCT-II in float32: the reference transform that section 5
// compares the approximations with (its PSNR is the denominator of the
// absolute percentage error).
//
// The forward transform is Chen's factorization of eqs. 1-3 with the exact
// parameters (alpha = cos(pi/4), beta_n = cos((2n+1) pi/16), gamma_n =
// cos((2n+1) pi/8)): the flowgraph of the approximations with its sixteen
// multiplications restored (Table 2: 16 multiplications, 26 additions).  With
// these parameters it computes 2 C8 x, and every factor is orthogonal up to a
// power of two, so the transposed flowgraph computes 2 C8^T X: the inverse of
// the orthonormal C8 is its transpose.  The 2D transforms scale by 1/4 (a
// power of two, no rounding).
//
// One thread owns one 8 x 8 tile (as in the integer 8-point kernels): load,
// level shift, forward rows and columns, zonal retention of the first r
// zig-zag coefficients, the orthonormal coefficients of the kept positions
// as output, inverse columns and rows, round half away from zero, +128 and
// clip (or saturate to int16), store, error energy.
#include <algorithm>

#include "tile8.hpp"

namespace adct {
namespace {

using namespace t8;

struct ChenConst {
  float a, b0, b1, b2, b3, g0, g1;
};

// cos(pi/4), cos(pi/16), cos(3pi/16), cos(5pi/16), cos(7pi/16), cos(pi/8),
// cos(3pi/8), rounded to float32
constexpr ChenConst kC = {0.70710678118654752f, 0.98078528040323045f, 0.83146961230254524f,
                          0.55557023301960218f, 0.19509032201612826f, 0.92387953251128676f,
                          0.38268343236508977f};

__device__ __forceinline__ void chen8(float (&x)[8]) {
  const float y0 = x[0] + x[7], y1 = x[1] + x[6], y2 = x[2] + x[5], y3 = x[3] + x[4];
  const float y4 = x[3] - x[4], y5 = x[2] - x[5], y6 = x[1] - x[6], y7 = x[0] - x[7];
  // M4 = diag(B4, A3(alpha))
  const float z0 = y0 + y3, z1 = y1 + y2, z2 = y1 - y2, z3 = y0 - y3;
  const float z4 = y7, z5 = kC.a * (y5 + y6), z6 = kC.a * (y6 - y5), z7 = y4;
  // M3 = diag(C~(alpha, gamma), A2)
  const float w0 = kC.a * (z0 + z1), w1 = kC.a * (z0 - z1);
  const float w2 = kC.g1 * z3 - kC.g0 * z2, w3 = kC.g1 * z2 + kC.g0 * z3;
  const float w4 = z4 + z5, w5 = z4 - z5, w6 = z7 - z6, w7 = z6 + z7;
  // M2 = diag(P4, A1(beta)), then M1 and P8
  x[0] = w0;
  x[1] = kC.b0 * w4 + kC.b3 * w7;
  x[2] = w3;
  x[3] = kC.b1 * w5 - kC.b2 * w6;
  x[4] = w1;
  x[5] = kC.b2 * w5 + kC.b1 * w6;
  x[6] = w2;
  x[7] = kC.b3 * w4 - kC.b0 * w7;
}

// The transposed flowgraph: 2 C8^T X.  A1, C~, A2 and B4 are symmetric, A3
// transposes to rows [0,0,0,1], [0,a,-a,0], [0,a,a,0], [1,0,0,0].
__device__ __forceinline__ void chen8_t(float (&X)[8]) {
  const float w0 = X[0], w3 = X[2], w1 = X[4], w2 = X[6];
  const float v4 = X[1], v6 = X[3], v5 = X[5], v7 = X[7];
  const float w4 = kC.b0 * v4 + kC.b3 * v7, w5 = kC.b2 * v5 + kC.b1 * v6;
  const float w6 = kC.b1 * v5 - kC.b2 * v6, w7 = kC.b3 * v4 - kC.b0 * v7;
  const float z0 = kC.a * (w0 + w1), z1 = kC.a * (w0 - w1);
  const float z2 = kC.g1 * w3 - kC.g0 * w2, z3 = kC.g1 * w2 + kC.g0 * w3;
  const float z4 = w4 + w5, z5 = w4 - w5, z6 = w7 - w6, z7 = w6 + w7;
  const float y0 = z0 + z3, y1 = z1 + z2, y2 = z1 - z2, y3 = z0 - z3;
  const float y4 = z7, y5 = kC.a * (z5 - z6), y6 = kC.a * (z5 + z6), y7 = z4;
  X[0] = y0 + y7;
  X[1] = y1 + y6;
  X[2] = y2 + y5;
  X[3] = y3 + y4;
  X[4] = y3 - y4;
  X[5] = y2 - y5;
  X[6] = y1 - y6;
  X[7] = y0 - y7;
}

// round half away from zero of a float
__device__ __forceinline__ int round_away(float v) {
  const float m = floorf(fabsf(v) + 0.5f);
  return static_cast<int>(v < 0.0f ? -m : m);
}

template <int DT, int RB>
__global__ __launch_bounds__(kWave) void compress8_dct(PassParams p) {
  __shared__ int lds[kWave * row_stride(RB)];
  constexpr int RS = row_stride(RB);
  const WaveTiles w = wave_tiles_interleaved(p.g, p.spread);
  const int lane = w.lane;
  const int r = p.r;
  Raw<DT> raw;
  load_raw<DT>(p.src, w.pix, p.g.pitch, w.active, raw);
  int ai[kN][kN];
  unpack<DT>(raw, ai);
  float a[kN][kN];
#pragma unroll
  for (int i = 0; i < kN; ++i)
#pragma unroll
    for (int j = 0; j < kN; ++j) a[i][j] = static_cast<float>(DT == DT_U8 ? ai[i][j] - 128 : ai[i][j]);
#pragma unroll
  for (int i = 0; i < kN; ++i) chen8(a[i]);
#pragma unroll
  for (int j = 0; j < kN; ++j) {
    float c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    chen8(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = 0.25f * c[i];   // orthonormal coefficients
  }
  // retained orthonormal coefficients in zig-zag order, staged for coalesced stores
  if (p.scaled != nullptr) {
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k < r) lds[lane * RS + k] = __builtin_bit_cast(int, a[kZZ.v[k]][kZZ.u[k]]);
    __syncthreads();
    uint32_t* g = reinterpret_cast<uint32_t*>(p.scaled + w.tile0 * r);
    if (r == RB) copy_tiles_out<RB, true>(g, lds, w.nact, lane);
    else copy_tiles_out_rt<true>(g, lds, r, RS, w.nact, lane);
  }
  if (p.dst == nullptr && p.sse == nullptr) return;
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) {
      const int pos = zz_pos(kN, v, u);
      if (pos >= RB || pos >= r) a[v][u] = 0.0f;
    }
#pragma unroll
  for (int j = 0; j < kN; ++j) {
    float c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    chen8_t(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = c[i];
  }
  Raw<DT> rec;
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    chen8_t(a[i]);
    int y[kN];
#pragma unroll
    for (int j = 0; j < kN; ++j) {
      const int q = round_away(0.25f * a[i][j]);
      y[j] = DT == DT_U8 ? min(max(q + 128, 0), 255) : min(max(q, -32768), 32767);
    }
    if constexpr (DT == DT_U8) {
      rec.w[i][0] = y[0] | (y[1] << 8) | (y[2] << 16) | (static_cast<uint32_t>(y[3]) << 24);
      rec.w[i][1] = y[4] | (y[5] << 8) | (y[6] << 16) | (static_cast<uint32_t>(y[7]) << 24);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        rec.w[i][j] = (y[2 * j] & 0xffff) | (static_cast<uint32_t>(y[2 * j + 1]) << 16);
    }
  }
  if (p.dst != nullptr && w.active) store_raw<DT, true>(p.dst, w.pix, p.g.pitch, rec);
  const unsigned long long e = p.sse != nullptr && w.active ? tile_sse<DT>(raw, rec) : 0ull;
  if (p.sse != nullptr) block_add_sse<kWave>(p.sse + w.img, e, nullptr);
}

constexpr int kRB[] = {1, 3, 6, 10, 15, 16, 21, 28, 36, 45, 64};
constexpr int kNumRB = sizeof(kRB) / sizeof(kRB[0]);

template <int DT, int I>
void launch_rb(const PassParams& p, hipStream_t s, dim3 grid) {
  if constexpr (I < kNumRB) {
    if (p.r <= kRB[I]) {
      compress8_dct<DT, kRB[I]><<<grid, kWave, 0, s>>>(p);
      return;
    }
    launch_rb<DT, I + 1>(p, s, grid);
  }
}

}  // namespace

int launch_dct8(int dtype, const PassParams& p_in, hipStream_t s) {
  PassParams p = p_in;
  p.spread = std::min(p.g.batch, p.r <= 16 ? 64 : (p.r <= 45 ? 16 : 2));
  const dim3 grid((p.g.tiles_x + kWave - 1) / kWave, p.g.tiles_y, p.g.batch);
  if (dtype == DT_U8) launch_rb<DT_U8, 0>(p, s, grid);
  else launch_rb<DT_I16, 0>(p, s, grid);
  return hipGetLastError();
}

}  // namespace adct
