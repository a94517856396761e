// 8 x 8 kernels: one thread owns one tile.
//
// A thread loads its 8 rows with one 8-byte (uint8) or 16-byte (int16) load
// per row -- the 64 threads of a wave cover 64 horizontally adjacent tiles, so
// each row load of a wave is one contiguous 512 B / 1 KB segment -- and keeps
// the whole tile in 64 registers.  Row and column butterflies, zonal masking
// or quantisation, the inverse butterflies and rounding all run in registers;
// nothing is exchanged between threads except the final error-energy
// reduction.  The level shift of 8-bit input is folded into the DC
// coefficient: every AC row of T sums to zero, so T (A - 128) T^T differs from
// T A T^T only in b[0][0], by 128 N^2.
#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kN = 8;
constexpr int kBlock = 256;

struct ZigZag8 {
  int v[64];
  int u[64];
};

constexpr ZigZag8 make_zigzag8() {
  ZigZag8 z{};
  for (int v = 0; v < kN; ++v)
    for (int u = 0; u < kN; ++u) {
      const int k = zz_pos(kN, v, u);
      z.v[k] = v;
      z.u[k] = u;
    }
  return z;
}

constexpr ZigZag8 kZZ = make_zigzag8();

// ---------------------------------------------------------------- pixel I/O
template <int DT>
__device__ __forceinline__ void load_tile(const void* src, int64_t off, int64_t pitch,
                                          bool active, int (&a)[kN][kN]) {
  if constexpr (DT == DT_U8) {
    const uint8_t* p = static_cast<const uint8_t*>(src) + off;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      uint2 w = make_uint2(0x80808080u, 0x80808080u);
      if (active) w = *reinterpret_cast<const uint2*>(p + i * pitch);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[i][j] = (w.x >> (8 * j)) & 0xff;
        a[i][j + 4] = (w.y >> (8 * j)) & 0xff;
      }
    }
  } else {
    const int16_t* p = static_cast<const int16_t*>(src) + off;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (active) w = *reinterpret_cast<const uint4*>(p + i * pitch);
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[i][2 * j] = static_cast<int>(ws[j] << 16) >> 16;
        a[i][2 * j + 1] = static_cast<int>(ws[j]) >> 16;
      }
    }
  }
}

// Round the inverse result z / 2^S (half away from zero), shift/clip, store,
// and return the squared error against the original tile ``x``.
template <int DT, int S>
__device__ __forceinline__ unsigned long long store_tile(void* dst, int64_t off, int64_t pitch,
                                                         bool active, const int (&z)[kN][kN],
                                                         const int (&x)[kN][kN], bool want_sse) {
  unsigned long long err = 0;
  if constexpr (DT == DT_U8) {
    uint8_t* p = static_cast<uint8_t*>(dst) + off;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      int y[kN];
#pragma unroll
      for (int j = 0; j < kN; ++j) {
        y[j] = min(max(round_shift_offset<S, 128>(z[i][j]), 0), 255);
        const int d = y[j] - x[i][j];
        acc += static_cast<uint32_t>(__mul24(d, d));
      }
      if (dst != nullptr && active) {
        uint2 w;
        w.x = y[0] | (y[1] << 8) | (y[2] << 16) | (y[3] << 24);
        w.y = y[4] | (y[5] << 8) | (y[6] << 16) | (y[7] << 24);
        *reinterpret_cast<uint2*>(p + i * pitch) = w;
      }
    }
    err = want_sse ? acc : 0u;
  } else {
    int16_t* p = static_cast<int16_t*>(dst) + off;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      int y[kN];
#pragma unroll
      for (int j = 0; j < kN; ++j) {
        y[j] = min(max(round_shift<S>(z[i][j]), -32768), 32767);
        const long long d = y[j] - x[i][j];
        err += static_cast<unsigned long long>(d * d);
      }
      if (dst != nullptr && active) {
        uint4 w;
        w.x = (y[0] & 0xffff) | (static_cast<uint32_t>(y[1]) << 16);
        w.y = (y[2] & 0xffff) | (static_cast<uint32_t>(y[3]) << 16);
        w.z = (y[4] & 0xffff) | (static_cast<uint32_t>(y[5]) << 16);
        w.w = (y[6] & 0xffff) | (static_cast<uint32_t>(y[7]) << 16);
        *reinterpret_cast<uint4*>(p + i * pitch) = w;
      }
    }
    if (!want_sse) err = 0;
  }
  return err;
}

// ------------------------------------------------------------ 2D transforms
template <int KIND>
__device__ __forceinline__ void forward2d(int (&a)[kN][kN]) {
#pragma unroll
  for (int i = 0; i < kN; ++i) fwd8<KIND>(a[i]);          // rows:    A T^T
#pragma unroll
  for (int j = 0; j < kN; ++j) {                          // columns: T (A T^T)
    int c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    fwd8<KIND>(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = c[i];
  }
}

template <int KIND>
__device__ __forceinline__ void inverse2d(int (&a)[kN][kN]) {
#pragma unroll
  for (int j = 0; j < kN; ++j) {                          // columns: K B
    int c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    inv8<KIND>(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = c[i];
  }
#pragma unroll
  for (int i = 0; i < kN; ++i) inv8<KIND>(a[i]);          // rows:    (K B) K^T
}

__device__ __forceinline__ int quantise(int b, int32_t mq) {
  const uint32_t mag = static_cast<uint32_t>(b < 0 ? -b : b);
  const uint64_t prod = static_cast<uint64_t>(mag) * static_cast<uint32_t>(mq) + (1ull << 23);
  const int lev = static_cast<int>(prod >> 24);
  return b < 0 ? -lev : lev;
}

__device__ __forceinline__ int table_index(const Tables& t, int v, int u) {
  return t.cls[v] * 4 + t.cls[u];
}

__device__ __forceinline__ void add_sse(unsigned long long* sse, int img, unsigned long long e) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0 && e != 0) atomicAdd(sse + img, e);
}

struct TileCoord {
  int tx, ty, img;
  bool active;
  int64_t tile;
  int64_t pix;
};

__device__ __forceinline__ TileCoord tile_coord(const Geom& g) {
  TileCoord c;
  c.tx = blockIdx.x * blockDim.x + threadIdx.x;
  c.ty = blockIdx.y;
  c.img = blockIdx.z;
  c.active = c.tx < g.tiles_x;
  c.tile = (static_cast<int64_t>(c.img) * g.tiles_y + c.ty) * g.tiles_x + c.tx;
  c.pix = static_cast<int64_t>(c.img) * g.image_stride +
          static_cast<int64_t>(c.ty) * kN * g.pitch + static_cast<int64_t>(c.tx) * kN;
  return c;
}

// ------------------------------------------------------------------ kernels
// Fused forward -> retain/quantise -> inverse -> round -> store -> SSE.
// RB is a compile-time bound on r: zig-zag positions >= RB are known to be
// zero, so the compiler drops the arithmetic that only feeds or reads them.
template <int KIND, int DT, int RB, bool QUANT>
__global__ __launch_bounds__(kBlock) void compress8(PassParams p) {
  const TileCoord c = tile_coord(p.g);
  int x[kN][kN];
  load_tile<DT>(p.src, c.pix, p.g.pitch, c.active, x);
  int a[kN][kN];
#pragma unroll
  for (int i = 0; i < kN; ++i)
#pragma unroll
    for (int j = 0; j < kN; ++j) a[i][j] = x[i][j];
  forward2d<KIND>(a);
  if constexpr (DT == DT_U8) a[0][0] -= 128 * kN * kN;

  const int r = p.r;
  // retained outputs (zig-zag order)
  if (c.active && p.scaled != nullptr) {
    float* sp = p.scaled + c.tile * r;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k < r) {
        const int v = kZZ.v[k], u = kZZ.u[k];
        sp[k] = static_cast<float>(a[v][u]) * p.t.s2[table_index(p.t, v, u)];
      }
  }
  // mask (and quantise) in place
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) {
      const int pos = zz_pos(kN, v, u);
      if (pos >= RB) {
        a[v][u] = 0;
      } else {
        int b = pos < r ? a[v][u] : 0;
        if constexpr (QUANT) {
          const int ti = table_index(p.t, v, u);
          b = quantise(b, p.t.mq[ti]);
        }
        a[v][u] = b;
      }
    }
  if (c.active && p.cout != nullptr) {
    int32_t* kp = p.cout + c.tile * r;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k < r) kp[k] = a[kZZ.v[k]][kZZ.u[k]];
  }
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < kN; ++v)
#pragma unroll
      for (int u = 0; u < kN; ++u)
        if (zz_pos(kN, v, u) < RB) a[v][u] = __mul24(a[v][u], p.t.dq[table_index(p.t, v, u)]);
  }
  if (p.dst == nullptr && p.sse == nullptr) return;
  inverse2d<KIND>(a);
  // zonal: y = round(Z / (4 N^2)); quantised (one fractional bit): Z / (8 N^2)
  constexpr int S = QUANT ? 9 : 8;
  const unsigned long long e =
      store_tile<DT, S>(p.dst, c.pix, p.g.pitch, c.active, a, x, p.sse != nullptr);
  if (p.sse != nullptr) add_sse(p.sse, c.img, e);
}

template <int KIND, int DT>
__global__ __launch_bounds__(kBlock) void forward8(PassParams p) {
  const TileCoord c = tile_coord(p.g);
  int a[kN][kN];
  load_tile<DT>(p.src, c.pix, p.g.pitch, c.active, a);
  forward2d<KIND>(a);
  if constexpr (DT == DT_U8) a[0][0] -= 128 * kN * kN;
  if (!c.active) return;
  int4* out = reinterpret_cast<int4*>(p.cout + c.tile * kN * kN);
#pragma unroll
  for (int v = 0; v < kN; ++v) {
    out[2 * v] = make_int4(a[v][0], a[v][1], a[v][2], a[v][3]);
    out[2 * v + 1] = make_int4(a[v][4], a[v][5], a[v][6], a[v][7]);
  }
}

// Inverse from natural-order coefficients (DECOMP = false) or from the
// zig-zag-ordered retained coefficients of adct_compress (DECOMP = true).
template <int KIND, int DT, bool QUANT, bool DECOMP>
__global__ __launch_bounds__(kBlock) void inverse8(PassParams p) {
  const TileCoord c = tile_coord(p.g);
  const int r = p.r;
  int a[kN][kN];
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) a[v][u] = 0;
  if (c.active) {
    if constexpr (DECOMP) {
      const int32_t* kp = p.cin + c.tile * r;
#pragma unroll
      for (int k = 0; k < kN * kN; ++k)
        if (k < r) a[kZZ.v[k]][kZZ.u[k]] = kp[k];
    } else {
      const int4* in = reinterpret_cast<const int4*>(p.cin + c.tile * kN * kN);
#pragma unroll
      for (int v = 0; v < kN; ++v) {
        const int4 lo = in[2 * v], hi = in[2 * v + 1];
        a[v][0] = lo.x; a[v][1] = lo.y; a[v][2] = lo.z; a[v][3] = lo.w;
        a[v][4] = hi.x; a[v][5] = hi.y; a[v][6] = hi.z; a[v][7] = hi.w;
      }
#pragma unroll
      for (int v = 0; v < kN; ++v)
#pragma unroll
        for (int u = 0; u < kN; ++u)
          if (zz_pos(kN, v, u) >= r) a[v][u] = 0;
    }
  }
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < kN; ++v)
#pragma unroll
      for (int u = 0; u < kN; ++u) a[v][u] = __mul24(a[v][u], p.t.dq[table_index(p.t, v, u)]);
  }
  inverse2d<KIND>(a);
  constexpr int S = QUANT ? 9 : 8;
  int dummy[kN][kN];
#pragma unroll
  for (int i = 0; i < kN; ++i)
#pragma unroll
    for (int j = 0; j < kN; ++j) dummy[i][j] = 0;
  (void)store_tile<DT, S>(p.dst, c.pix, p.g.pitch, c.active, a, dummy, false);
}

// ---------------------------------------------------------------- dispatch
constexpr int kRB[] = {1, 3, 6, 10, 15, 16, 21, 28, 36, 45, 64};
constexpr int kNumRB = sizeof(kRB) / sizeof(kRB[0]);

dim3 grid_for(const Geom& g, int* block) {
  int bs = kBlock;
  if (g.tiles_x < kBlock) bs = ((g.tiles_x + 63) / 64) * 64;
  *block = bs;
  return dim3((g.tiles_x + bs - 1) / bs, g.tiles_y, g.batch);
}

template <int KIND, int DT, int I>
hipError_t launch_compress_rb(const PassParams& p, hipStream_t s, int bs, dim3 grid) {
  if constexpr (I >= kNumRB) {
    return hipErrorInvalidValue;
  } else {
    if (p.r <= kRB[I]) {
      compress8<KIND, DT, kRB[I], false><<<grid, bs, 0, s>>>(p);
      return hipGetLastError();
    }
    return launch_compress_rb<KIND, DT, I + 1>(p, s, bs, grid);
  }
}

template <int KIND, int DT>
hipError_t launch_typed(Mode mode, const PassParams& p, hipStream_t s) {
  int bs = 0;
  const dim3 grid = grid_for(p.g, &bs);
  const bool quant = p.qstep > 0;
  switch (mode) {
    case Mode::Compress:
      if (quant) {
        compress8<KIND, DT, 64, true><<<grid, bs, 0, s>>>(p);
        return hipGetLastError();
      }
      return launch_compress_rb<KIND, DT, 0>(p, s, bs, grid);
    case Mode::Forward:
      forward8<KIND, DT><<<grid, bs, 0, s>>>(p);
      return hipGetLastError();
    case Mode::Inverse:
      if (quant) inverse8<KIND, DT, true, false><<<grid, bs, 0, s>>>(p);
      else inverse8<KIND, DT, false, false><<<grid, bs, 0, s>>>(p);
      return hipGetLastError();
    case Mode::Decompress:
      if (quant) inverse8<KIND, DT, true, true><<<grid, bs, 0, s>>>(p);
      else inverse8<KIND, DT, false, true><<<grid, bs, 0, s>>>(p);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace

int launch_n8(Mode mode, int kind, int dtype, const PassParams& p, hipStream_t stream) {
  if (kind == KIND_SIGN)
    return dtype == DT_U8 ? launch_typed<KIND_SIGN, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_SIGN, DT_I16>(mode, p, stream);
  return dtype == DT_U8 ? launch_typed<KIND_ROUND, DT_U8>(mode, p, stream)
                        : launch_typed<KIND_ROUND, DT_I16>(mode, p, stream);
}

}  // namespace adct
